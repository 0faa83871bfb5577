"""Compression curve of pMMF (the analogue of the paper's Fig. 3 experiment): for a growing core
size delta, the relative Frobenius error of the factorization ||A - U^T H U||_F / ||A||_F (the
library's FP64 residual) against that of the best approximation of the same rank budget,
||A - A_delta||_F / ||A||_F, with A_delta the truncated eigendecomposition (Eckart-Young: the
squared error is the sum of the squared eigenvalues left out, by decreasing |lambda|).

    python -m paper_1507_04396_amd.compression --workload knn2d --n 4096 --cores 64,256,1024

prints one JSON line per core size.  The eigenvalues come from an FP64 dense eigensolver on the
device (torch.linalg.eigvalsh), so n is limited to what a dense n x n FP64 matrix allows.
"""
import argparse
import json
import math
import os
import sys

import numpy as np
import torch


def eigenvalues_fp64(csr, device="cuda") -> np.ndarray:
    """Eigenvalues of the symmetric CSR matrix, FP64, sorted by decreasing |lambda|."""
    n = len(csr.rowptr) - 1
    rows = np.repeat(np.arange(n), np.diff(csr.rowptr))
    a = torch.zeros((n, n), dtype=torch.float64, device=device)
    a[torch.from_numpy(rows).to(device), torch.from_numpy(csr.colind.astype(np.int64)).to(device)] = \
        torch.from_numpy(csr.val.astype(np.float64)).to(device)
    lam = torch.linalg.eigvalsh(0.5 * (a + a.T)).cpu().numpy()
    return lam[np.argsort(-np.abs(lam), kind="stable")]


def best_rank_error2(lam_sorted: np.ndarray, rank: int) -> float:
    """||A - A_rank||_F^2 from eigenvalues sorted by decreasing |lambda|."""
    tail = lam_sorted[rank:]
    return float(np.dot(tail, tail))


def compression_curve(csr, cores, *, k=2, eta=0.5, cluster=(0, 0), seed=0, lam=None,
                      cut_clusters=False):
    """One record per core size: relative errors of pMMF and of the best rank-delta approximation
    and their ratio, with the factorization time.  ``cut_clusters`` selects the data-driven
    clustering (boundaries that separate the fewest active-matrix entries)."""
    from .api import Factorization
    if lam is None:
        lam = eigenvalues_fp64(csr)
    fro2 = float(np.dot(lam, lam))
    out = []
    for core in cores:
        f = Factorization.from_csr(csr, k=k, eta=eta, core=int(core), cluster=tuple(cluster),
                                   seed=seed, cut_clusters=cut_clusters)
        inf = f.info()
        f.close()
        err2 = max(float(inf["loss"]), 0.0)
        best2 = best_rank_error2(lam, int(core))
        out.append(dict(core=int(core), rel_err=math.sqrt(err2 / fro2),
                        best_rel_err=math.sqrt(best2 / fro2),
                        ratio=math.sqrt(err2 / best2) if best2 > 0 else math.inf,
                        fro2_a=float(inf["fro2_a"]), factor_ms=float(inf["factor_ms"])))
    return out


def _matrix(name, n, seed):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads
    if name == "knn2d":
        return workloads.knn_points_matrix(n, 2, 8, 0.01, seed)
    if name == "knn3d":
        return workloads.knn_points_matrix(n, 3, 10, 0.01, seed)
    if name == "grid2d":
        side = int(round(math.sqrt(n)))
        return workloads.small_grid((side, side), sigma=1.0, shift=0.0, seed=seed)
    if name == "rbf":
        return workloads.rbf_kernel_matrix(n, 2, 50.0, seed)
    raise SystemExit(f"unknown workload {name}")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="knn2d", choices=["knn2d", "knn3d", "grid2d", "rbf"])
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--cores", default="64,128,256,512,1024,2048")
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--cluster", default="512,2048")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cut-clusters", action="store_true",
                    help="data-driven clusters (fewest separated entries) instead of seeded sizes")
    a = ap.parse_args(argv)
    csr = _matrix(a.workload, a.n, 0)
    cores = [int(c) for c in a.cores.split(",")]
    lo, hi = (int(v) for v in a.cluster.split(","))
    for rec in compression_curve(csr, cores, k=a.k, cluster=(lo, hi), seed=a.seed,
                                 cut_clusters=a.cut_clusters):
        rec.update(workload=a.workload, n=len(csr.rowptr) - 1, k=a.k, cluster=[lo, hi],
                   clustering="cut" if a.cut_clusters else "seeded")
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
