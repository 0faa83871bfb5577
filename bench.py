"""Benchmark of the pMMF hot path on one MI355X.

A step is one pMMF factorization (mmf_factor: every stage's clustering, cluster Grams, greedy
rotation search, two-sided rotation and peeling, and the core) of the n = 262,144 kNN Laplacian
(3-point rotations, clusters of 512-2048, core 1,024).  The headline value is rotations per second
= (n - core) / wall time per factorization, with the CSR already resident in HBM.

Beside it the same JSON line reports the matrix-free apply and the adjoint (mmf_apply,
mmf_backward) on the factorization of the 256 x 256 grid Laplacian with 256 right-hand sides, as
algorithmic GB/s, 50 steps of angle refinement on that factorization, preconditioned CG on the
101 x 101 x 103 grid with 128 right-hand sides, the two Gram forms with their matrix-core rates,
the per-stage phase split, a roofline entry for the dominant kernel, and the FP64 oracle on the
host: it replays the whole headline factorization (CPU baseline and loss against the oracle).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 (matrix and vector)
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 matrix


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def device_csr(A, torch):
    rp = torch.from_numpy(A.rowptr).cuda()
    ci = torch.from_numpy(A.colind).cuda()
    cv = torch.from_numpy(A.val).cuda()
    return rp, ci, cv


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter summary
    (profiles/<kernel>_<workload>_traffic.md), or None when there is none or the kernel's source
    file changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    src = os.path.join(ROOT, "paper_1507_04396_amd", "csrc", "factor_kernels.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"source_sha256\s*=\s*([0-9a-f]{64})", text)
    m_b = re.search(r"traffic_bytes_per_launch\s*=\s*(\d+)", text)
    if not (m_sha and m_b):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_sha.group(1):
        return None
    return int(m_b.group(1))


def sweep_rows(stages):
    """sum over stages of |S_{p-1}| (rows each U-sweep reads and writes)."""
    return sum(st["size"] for st in stages)


def measure_apply(args, torch, workloads, Factorization, log):
    """Apply, adjoint and angle refinement on the apply workload's factorization."""
    log(f"[bench] factor {args.apply_workload} for apply/backward")
    B = workloads.make_matrix(args.apply_workload)
    bprm = dict(workloads.WORKLOADS[args.apply_workload]["params"])
    fb = Factorization.from_csr(B, **bprm)
    bstages = fb.stage_info()
    X = torch.from_numpy(workloads.gaussian_block(B.n, args.nrhs, seed=1000)).cuda()
    Yb = torch.from_numpy(workloads.gaussian_block(B.n, args.nrhs, seed=1001)).cuda()
    Y = torch.empty_like(X)
    fb.apply(X, out=Y)
    fb.backward(X, Yb)
    torch.cuda.synchronize()
    nrep = max(3, args.steps)
    st_ = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st_)
    for _ in range(nrep):
        fb.apply(X, out=Y)
    e1.record(st_)
    torch.cuda.synchronize()
    apply_ms = e0.elapsed_time(e1) / nrep
    e0.record(st_)
    for _ in range(nrep):
        fb.backward(X, Yb)
    e1.record(st_)
    torch.cuda.synchronize()
    back_ms = e0.elapsed_time(e1) / nrep
    rows = sweep_rows(bstages)
    nr, core, kk = args.nrhs, bprm["core"], bprm["k"]
    Rb = B.n - core
    log_bytes = Rb * (kk * 4 + kk * kk * 4)
    usweep = 2 * 4 * nr * rows
    apply_bytes = 2 * usweep + 2 * log_bytes + core * core * 4 + 2 * core * nr * 4
    s1 = bstages[0]["size"]
    back_bytes = (2 * usweep                                   # forward sweeps of x and ybar
                  + 4 * 4 * nr * rows                          # reverse: read 4 vectors
                  + 4 * 4 * nr * (rows - s1) + 4 * nr * s1     # reverse writes (xbar at stage 1)
                  + 3 * log_bytes + 3 * core * core * 4 + Rb * 4 + B.n * 4)
    apply_gbs = apply_bytes / (apply_ms * 1e-3) / 1e9
    back_gbs = back_bytes / (back_ms * 1e-3) / 1e9
    # ----------------------------------------------------------------- angle refinement
    from paper_1507_04396_amd.refine import AngleRefiner
    log(f"[bench] angle refinement on {args.apply_workload}: {args.refine_steps} Adam steps, "
        f"{args.nrhs} probes")
    rpB, ciB, cvB = device_csr(B, torch)
    refiner = AngleRefiner(fb, rpB, ciB, cvB, lr=1e-3, optimizer="adam")
    refiner.run(2, args.nrhs, seed=5)
    torch.cuda.synchronize()
    e0.record(st_)
    hist = refiner.run(args.refine_steps, args.nrhs, seed=6)
    e1.record(st_)
    torch.cuda.synchronize()
    refine_ms = e0.elapsed_time(e1) / max(1, args.refine_steps)
    hist = hist.cpu().numpy()
    refine = {"workload": f"{args.apply_workload} factorization, Hutchinson estimate of "
                          f"||A - U^T H U||_F^2 with {args.nrhs} fresh N(0,1) probes per step, "
                          f"Adam lr 1e-3 on theta and H",
              "steps": args.refine_steps, "ms_per_step": round(refine_ms, 4),
              "loss_first5": round(float(hist[:5].mean()), 4),
              "loss_last5": round(float(hist[-5:].mean()), 4)}
    fb.close()
    apply_res = {"workload": f"{args.apply_workload} factorization, {args.nrhs} RHS",
                 "ms": round(apply_ms, 4), "algorithmic_GBps": round(apply_gbs, 1),
                 "frac_hbm": round(apply_gbs / HBM_PEAK_GBS, 4)}
    back_res = {"workload": f"{args.apply_workload} factorization, {args.nrhs} RHS",
                "ms": round(back_ms, 4), "algorithmic_GBps": round(back_gbs, 1),
                "frac_hbm": round(back_gbs / HBM_PEAK_GBS, 4)}
    return apply_res, back_res, refine


def measure_pcg(args, torch, workloads, Factorization, log):
    """Preconditioned CG with the pMMF inverse on the 101 x 101 x 103 grid (Sec. 4)."""
    wl = args.pcg_workload
    log(f"[bench] pcg: factor {wl}")
    A = workloads.make_matrix(wl)
    prm = dict(workloads.WORKLOADS[wl]["params"])
    rp, ci, cv = device_csr(A, torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fac = Factorization.factor(rp, ci, cv, **prm)
    torch.cuda.synchronize()
    factor_ms = 1e3 * (time.perf_counter() - t0)
    stages = fac.stage_info()
    nr = args.pcg_nrhs
    B = torch.from_numpy(workloads.gaussian_block(A.n, nr, seed=2)).cuda()
    # one preconditioner application: A~^{-1} X
    Y = torch.empty_like(B)
    fac.apply(B, out=Y, inverse=True)
    torch.cuda.synchronize()
    st_ = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st_)
    for _ in range(3):
        fac.apply(B, out=Y, inverse=True)
    e1.record(st_)
    torch.cuda.synchronize()
    inv_ms = e0.elapsed_time(e1) / 3
    core, kk = prm["core"], prm["k"]
    log_bytes = (A.n - core) * (kk * 4 + kk * kk * 4)
    inv_bytes = (2 * 2 * 4 * nr * sweep_rows(stages) + 2 * log_bytes + core * core * 4
                 + 2 * core * nr * 4)
    log(f"[bench] pcg: solve {nr} right-hand sides")
    X, info = fac.pcg(rp, ci, cv, B, tol=1e-6, max_iter=2000)
    torch.cuda.synchronize()
    fac.close()
    it = max(1, info["iterations"])
    return {"workload": f"{wl}: 7-point 101x101x103 grid, lognormal(0,1.5) weights, D - W + 1e-2 I "
                        f"(n={A.n}), {nr} N(0,1) right-hand sides, pMMF inverse (k={prm['k']}, "
                        f"clusters {prm['cluster'][0]}-{prm['cluster'][1]}, core {core}) as "
                        f"preconditioner, FP64 residual tolerance 1e-6",
            "factor_ms": round(factor_ms, 2), "iterations": info["iterations"],
            "refinements": info["refinements"], "converged": info["converged"],
            "max_rel_residual": info["max_rel_residual"], "solve_ms": round(info["solve_ms"], 2),
            "ms_per_iteration": round(info["solve_ms"] / it, 4),
            "apply_inverse_ms": round(inv_ms, 4),
            "apply_inverse_algorithmic_GBps": round(inv_bytes / (inv_ms * 1e-3) / 1e9, 1),
            "apply_inverse_frac_hbm": round(inv_bytes / (inv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def gram_rates(stages, peak_tflops):
    """Matrix-core Gram (stages in a dense form): performed and useful flop rates."""
    dense = [st for st in stages if st["dense_gram"]]
    if not dense:
        return None
    ms = sum(st["gram_ms"] for st in dense)
    perf = sum(st["gram_flops"] for st in dense)
    useful = sum(st["gram_useful_flops"] for st in dense)
    rate = perf / (ms * 1e-3) / 1e12
    return {"stages": [i + 1 for i, st in enumerate(stages) if st["dense_gram"]],
            "ms": round(ms, 3), "performed_tflops": round(rate, 3),
            "useful_tflops": round(useful / (ms * 1e-3) / 1e12, 3),
            "useful_fraction": round(useful / perf, 4) if perf else None,
            "peak_tflops": peak_tflops, "mfma_utilisation": round(rate / peak_tflops, 5)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="knn3d_n262144")
    ap.add_argument("--apply-workload", default="grid2d_n65536")
    ap.add_argument("--nrhs", type=int, default=256)
    ap.add_argument("--refine-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gram-seeds", type=int, default=5,
                    help="algorithm seeds for the FP32-vs-BF16 Gram comparison (0 = skip)")
    ap.add_argument("--factor-only", action="store_true",
                    help="time the factorization and the copy reference only (counter runs)")
    ap.add_argument("--pcg-workload", default="grid3d_n1050703")
    ap.add_argument("--pcg-nrhs", type=int, default=128)
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--gram-mode", type=int, default=0,
                    help="Gram form of the timed factorizations (0 FP32, 1 BF16 with rescoring)")
    ap.add_argument("--apply-only", action="store_true",
                    help="time apply, adjoint and refinement only (counter runs of the sweeps)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the factorization shards by cluster, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_1507_04396_amd import _lib
    from paper_1507_04396_amd.api import Factorization
    _lib.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    # ----------------------------------------------------------------- HBM reference: plain copy
    copy_elems = 1 << 28                     # 1 GiB of float32 read, 1 GiB written
    src = torch.ones(copy_elems, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_ms = c0.elapsed_time(c1) / 5
    copy_gbs = 2 * 4 * copy_elems / (copy_ms * 1e-3) / 1e9
    del src, dst

    if args.apply_only:
        apply_res, back_res, refine = measure_apply(args, torch, workloads, Factorization, log)
        print(json.dumps({"apply": apply_res, "backward": back_res, "refine": refine}), flush=True)
        return

    # ----------------------------------------------------------------- factorization (headline)
    wl = workloads.WORKLOADS[args.workload]
    prm = dict(wl["params"])
    if args.gram_mode:
        if not args.factor_only:
            raise SystemExit("--gram-mode applies to --factor-only runs")
        prm["gram_mode"] = args.gram_mode
    log(f"[bench] generating {args.workload}")
    A = workloads.make_matrix(args.workload)
    rp, ci, cv = device_csr(A, torch)
    torch.cuda.synchronize()
    R = A.n - prm["core"]
    for w in range(args.warmup):
        log(f"[bench] warmup factor {w}")
        Factorization.factor(rp, ci, cv, **prm).close()
    torch.cuda.synchronize()
    times = []
    fac = None
    for s in range(args.steps):
        if fac is not None:
            fac.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = Factorization.factor(rp, ci, cv, **prm)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"[bench] factor step {s}: {times[-1] * 1e3:.2f} ms")
    info = fac.info()
    stages = fac.stage_info()
    ex = fac.export()
    ms_per_step = 1e3 * float(np.mean(times))
    rot_per_s = R / (ms_per_step / 1e3)
    find_ms = sum(st["find_ms"] for st in stages)
    gram_ms = sum(st["gram_ms"] for st in stages)
    rot_ms = sum(st["rotate_ms"] for st in stages)
    fbytes = sum(st["find_bytes"] for st in stages)
    fac.close()

    # ----------------------------------------------------------------- Gram forms over seeds
    gram_forms = None
    if args.gram_seeds > 0 and not args.factor_only:
        gram_forms = {}
        for mode, label in ((0, "fp32"), (1, "bf16_rescored")):
            t_ms, losses = [], []
            for sd in range(args.gram_seeds):
                p2 = dict(prm)
                p2["seed"] = sd
                # an untimed run first: a seed's cluster sizes give new stage shapes, whose launch
                # configurations the tuner measures once
                Factorization.factor(rp, ci, cv, gram_mode=mode, **p2).close()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                f2 = Factorization.factor(rp, ci, cv, gram_mode=mode, **p2)
                torch.cuda.synchronize()
                t_ms.append(1e3 * (time.perf_counter() - t0))
                losses.append(f2.info()["loss"])
                if sd == 0:
                    st0 = f2.stage_info()
                f2.close()
            log(f"[bench] gram form {label}: {np.round(t_ms, 1)} ms, loss {np.round(losses, 2)}")
            gram_forms[label] = {"seeds": args.gram_seeds,
                                 "factor_ms_median": round(float(np.median(t_ms)), 3),
                                 "loss_mean": round(float(np.mean(losses)), 4),
                                 "loss_std": round(float(np.std(losses)), 4),
                                 "gram_ms": round(sum(st["gram_ms"] for st in st0), 3),
                                 "matrix_core_gram": gram_rates(
                                     st0, FP32_PEAK_TFLOPS if mode == 0 else BF16_PEAK_TFLOPS)}
    # ----------------------------------------------------------------- clustering forms
    # the seeded contiguous clusters (the FP32 Gram form above) against the data-driven
    # clusters that cut the fewest active-matrix entries, over the same algorithm seeds
    clustering = None
    if gram_forms is not None:
        t_ms, losses = [], []
        for sd in range(args.gram_seeds):
            p2 = dict(prm)
            p2["seed"] = sd
            Factorization.factor(rp, ci, cv, cut_clusters=True, **p2).close()  # tuner, untimed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f2 = Factorization.factor(rp, ci, cv, cut_clusters=True, **p2)
            torch.cuda.synchronize()
            t_ms.append(1e3 * (time.perf_counter() - t0))
            losses.append(f2.info()["loss"])
            f2.close()
        log(f"[bench] cut clusters: {np.round(t_ms, 1)} ms, loss {np.round(losses, 2)}")
        clustering = {"seeded": gram_forms["fp32"],
                      "cut": {"seeds": args.gram_seeds,
                              "factor_ms_median": round(float(np.median(t_ms)), 3),
                              "loss_mean": round(float(np.mean(losses)), 4),
                              "loss_std": round(float(np.std(losses)), 4)}}
    # ----------------------------------------------------------------- two eliminations per rotation
    two_elim = None
    if not args.factor_only and prm["k"] == 3:
        t_ms = []
        Factorization.factor(rp, ci, cv, elims=2, **prm).close()  # tuner, untimed
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f2 = Factorization.factor(rp, ci, cv, elims=2, **prm)
            torch.cuda.synchronize()
            t_ms.append(1e3 * (time.perf_counter() - t0))
            inf2, st2 = f2.info(), f2.stage_info()
            f2.close()
        two_elim = {"factor_ms_median": round(float(np.median(t_ms)), 3),
                    "find_ms": round(sum(st["find_ms"] for st in st2), 3),
                    "loss": inf2["loss"],
                    "retired_per_s": round(R / (float(np.median(t_ms)) / 1e3), 1)}
        log(f"[bench] two eliminations per rotation: {np.round(t_ms, 1)} ms, loss {inf2['loss']:.6g}")
    del rp, ci, cv

    # ----------------------------------------------------------------- apply / adjoint
    apply_res = back_res = refine = None
    if not args.factor_only:
        apply_res, back_res, refine = measure_apply(args, torch, workloads, Factorization, log)

    # ----------------------------------------------------------------- roofline (dominant kernel)
    find_launches = len(stages)
    find_gbs = fbytes / (find_ms * 1e-3) / 1e9
    roofline = {"kernel": "k_search (greedy rotation search, one launch per stage)",
                "bound": "hbm", "achieved": round(find_gbs, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(find_gbs / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic("k_search", "knn3d_n262144"),
                "launches": find_launches,
                "avg_launch_ms": round(find_ms / max(1, find_launches), 4),
                "algorithmic_bytes_per_launch": int(fbytes / max(1, find_launches)),
                "measured_copy_peak": round(copy_gbs, 1),
                "frac_of_measured_copy": round(find_gbs / copy_gbs, 5)}

    # ----------------------------------------------------------------- PCG (Sec. 4)
    pcg = None
    if not args.factor_only and not args.no_pcg:
        pcg = measure_pcg(args, torch, workloads, Factorization, log)

    # ----------------------------------------------------------------- CPU baseline (oracle)
    # the FP64 oracle factors the same matrix on the host's cores (one process per cluster of a
    # stage), replaying the GPU's log: it takes the GPU's choice only where its own decision is a
    # near-tie, so its loss is comparable with the GPU's
    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        try:
            ncores = len(os.sched_getaffinity(0))
        except AttributeError:
            ncores = os.cpu_count() or 1
        workers = max(1, min(16, ncores))
        log(f"[bench] cpu baseline: FP64 oracle replay of the {args.workload} factorization on "
            f"{workers} processes")
        t0 = time.perf_counter()
        ref = oracle.factor(A, replay=dict(rot_ids=ex["rot_ids"], rot_retired=ex["rot_retired"],
                                           rot_o=ex["rot_o"]), workers=workers, **prm)
        dt = time.perf_counter() - t0
        cpu = {"value": round(len(ref.rotations) / dt, 2), "unit": "rotations/s",
               "cores": workers, "kind": "oracle",
               "sample": f"the whole {args.workload} factorization ({len(ref.rotations)} "
                         f"rotations, {ref.num_stages} stages) by the FP64 oracle in {dt:.1f} s, "
                         f"clusters of a stage in {workers} processes, replaying the GPU's log "
                         f"(the GPU's choice taken at near-ties only)"}
        adopted = sum(len(r.adopted) for r in ref.rotations)
        parity = {"oracle_loss": ref.loss, "gpu_loss": info["loss"],
                  "oracle_loss_rel_err": abs(info["loss"] - ref.loss) / ref.loss,
                  "near_tie_decisions_taken_from_gpu": adopted,
                  "divergences": len(ref.divergences),
                  "hdiag_max_rel_err": float(np.abs(ex["hdiag"] - ref.hdiag).max()
                                             / np.abs(ref.hdiag).max()),
                  "hcore_max_rel_err": float(np.abs(ex["hcore"] - ref.hcore).max()
                                             / np.abs(ref.hcore).max())}
        log(f"[bench] oracle loss {ref.loss:.10g}, gpu {info['loss']:.10g}, rel "
            f"{parity['oracle_loss_rel_err']:.2e}, {adopted} near-ties taken, "
            f"{len(ref.divergences)} divergences")

    out = {
        "metric": "rotations/sec + factor time at n=262k; apply+backward GB/s vs roofline",
        "value": round(rot_per_s, 1), "unit": "rotations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: pMMF factor of the kNN (k=10) normalized "
                               f"Laplacian on {A.n} uniform points in [0,1]^3, "
                               f"{prm['k']}-point rotations, clusters {prm['cluster'][0]}-"
                               f"{prm['cluster'][1]}, eta {prm['eta']}, core {prm['core']}",
                   "n": A.n, "nnz": A.nnz, "rotations": R},
        "factor_ms": round(ms_per_step, 3),
        "factor_device_ms": round(info["factor_ms"], 3),
        "factor_phase_ms": {"gram": round(gram_ms, 3), "find": round(find_ms, 3),
                            "rotate": round(rot_ms, 3)},
        "factor_loss": info["loss"],
        "apply": apply_res,
        "backward": back_res,
        "hbm_copy": {"bytes": 8 * copy_elems, "ms": round(copy_ms, 4),
                     "GBps": round(copy_gbs, 1), "kind": "1 GiB float32 device copy (torch)"},
        "refine": refine,
        "gram_forms": gram_forms,
        "clustering": clustering,
        "two_eliminations": two_elim,
        "pcg": pcg,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "stages": [{k2: (round(v, 4) if isinstance(v, float) else v) for k2, v in st.items()}
                   for st in stages],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
