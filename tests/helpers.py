"""Shared helpers for the parity tests (no arithmetic of the method lives here)."""
import numpy as np

import os

TIE = 1e-5  # relative decision margin below which two choices are both correct


def oracle_workers():
    """Processes for the oracle's per-cluster work: the host's CPU share, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


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


def replay_log(gpu_export):
    """The GPU's decisions in the layout ``oracle.factor(replay=...)`` takes."""
    return dict(rot_ids=gpu_export["rot_ids"], rot_retired=gpu_export["rot_retired"],
                rot_o=gpu_export["rot_o"])


def check_factor_parity(A, params, fac, name, say=print, exact=False, loss_rtol=1e-4,
                        workers=None):
    """A GPU factorization against the oracle replaying its log (R13 of the oracle).

    The oracle runs Alg. 1 / Alg. 2 itself and takes the GPU's choice only where its own decision
    is a near-tie; every other differing decision is a divergence and fails the check.  With the
    decision sequences then equal, every rotation block, H and the loss are compared: O within
    max(1e-5, the oracle's bound on how far an FP32 G[T,T] moves the eigenvectors + 2 u32), H to
    1e-5 relative, the loss to ``loss_rtol``.  ``exact``: no decision may differ at all."""
    import numpy as np
    import oracle
    inf = fac.info()
    ex = fac.export()
    say(f"[parity] {name}: oracle replay of {inf['num_rotations']} rotations")
    rep = oracle.factor(A, replay=replay_log(ex), workers=workers or oracle_workers(), **params)
    R = len(rep.rotations)
    assert inf["num_rotations"] == R
    assert inf["num_stages"] == rep.num_stages
    # properties that hold for any valid factorization
    assert abs(inf["trace_h"] - inf["trace_a"]) <= 1e-5 * max(1.0, abs(inf["trace_a"]))
    fro_gap = inf["fro2_a"] - inf["fro2_h"]
    assert abs(fro_gap - inf["loss"]) <= 1e-4 * inf["fro2_a"] + 1e-4 * inf["loss"]
    assert inf["loss_literal"] >= inf["loss"] * (1 - 1e-5)
    k = fac.k
    O = ex["rot_o"].astype(np.float64)
    orth = np.abs(np.einsum("rij,rkj->rik", O, O) - np.eye(k)[None]).max() if R else 0.0
    assert orth <= 1e-5
    retired = ex["rot_retired"]
    assert len(set(retired.tolist())) == R
    assert sorted(set(retired.tolist()) | set(ex["core_ids"].tolist())) == list(range(A.n))
    # decisions
    adopted = [(t, w, ok) for t, r in enumerate(rep.rotations) for w, ok, _ in r.adopted]
    say(f"[parity] {name}: {len(adopted)} near-tie decisions taken from the GPU, "
        f"{len(rep.divergences)} divergences")
    assert not rep.divergences, f"decisions that are not near-ties differ: {rep.divergences[:5]}"
    if exact:
        assert not adopted, f"decisions differ: {adopted[:5]}"
    ids = np.array([r.ids for r in rep.rotations]).reshape(R, k) if R else ex["rot_ids"]
    np.testing.assert_array_equal(ex["rot_ids"], ids)
    np.testing.assert_array_equal(retired, rep.retired_order)
    np.testing.assert_array_equal(ex["core_ids"], rep.core_ids)
    # rotation blocks, H and the loss
    if R:
        Oref = np.array([r.O for r in rep.rotations]).reshape(O.shape)
        dO = np.abs(O - Oref).reshape(R, -1).max(axis=1)
        tol = np.maximum(1e-5, np.array([r.o_err for r in rep.rotations]) + 2 * oracle.U32)
        say(f"[parity] {name}: rotation blocks max |dO| {dO.max():.3g}, "
            f"largest |dO| / tolerance {(dO / tol).max():.3g}")
        assert np.all(dO <= tol), f"rotation {int(np.argmax(dO / tol))}: |dO| {dO.max():.3g}"
    eh, ec = rel_err(ex["hdiag"], rep.hdiag), rel_err(ex["hcore"], rep.hcore)
    lrel = abs(inf["loss"] - rep.loss) / max(rep.loss, 1e-300)
    say(f"[parity] {name}: H diag {eh:.2e} core {ec:.2e}; loss gpu {inf['loss']:.10g} "
        f"oracle {rep.loss:.10g} rel {lrel:.2e}")
    assert eh <= 1e-5 and ec <= 1e-5
    assert lrel <= loss_rtol
    return rep
