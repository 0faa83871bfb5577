"""Shared helpers for the parity tests (no arithmetic of the method lives here)."""
import numpy as np

TIE = 1e-5  # relative decision margin below which two choices are both correct


def oracle_log(fac):
    """An oracle factorization in the mmf_import layout."""
    k = fac.k
    R = len(fac.rotations)
    ids = np.array([r.ids for r in fac.rotations], dtype=np.int32).reshape(R, k)
    o = np.array([r.O for r in fac.rotations], dtype=np.float32).reshape(R, k, k)
    ret = np.array([r.retired for r in fac.rotations], dtype=np.int32)
    return dict(n=fac.n, k=k, core=len(fac.core_ids),
                stage_sizes=[st["size"] for st in fac.stages],
                stage_clusters=[len(st["cluster_sizes"]) for st in fac.stages],
                cluster_sizes=[c for st in fac.stages for c in st["cluster_sizes"]],
                rot_ids=ids, rot_o=o, rot_retired=ret, hdiag=fac.hdiag.astype(np.float32),
                core_ids=fac.core_ids.astype(np.int32), hcore=fac.hcore.astype(np.float32))


def first_divergence(gpu_export, fac):
    """Index of the first rotation whose tuple or retired index differs, or None."""
    ids = gpu_export["rot_ids"]
    ret = gpu_export["rot_retired"]
    for t, r in enumerate(fac.rotations):
        if list(ids[t]) != list(r.ids) or int(ret[t]) != int(r.retired):
            return t
    return None


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def grid_sub_instance():
    """Leading 1,024 x 1,024 principal submatrix of the 256 x 256 grid Laplacian (4 grid rows)."""
    import workloads
    A = workloads.make_matrix("grid2d_n65536").to_scipy()[:1024, :1024]
    return workloads._csr_from_scipy(A)


def import_oracle(ref):
    """Load an oracle factorization into the HIP library through mmf_import."""
    from paper_1507_04396_amd.api import Factorization
    lg = oracle_log(ref)
    return Factorization.import_log(lg["n"], lg["k"], lg["core"], lg["stage_sizes"],
                                    lg["stage_clusters"], lg["cluster_sizes"], lg["rot_ids"],
                                    lg["rot_o"], lg["rot_retired"], lg["hdiag"], lg["core_ids"],
                                    lg["hcore"])
