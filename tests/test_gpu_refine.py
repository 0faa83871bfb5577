"""Angle refinement: gradient steps on the probe estimate of Eq. 1's objective ||A - A~||_F^2.

The GPU loop (mmf_spmm, mmf_apply, mmf_backward, torch optimizer) is compared with the same loop
in FP64 built from the oracle's apply and adjoint, on the 1,024-row grid sub-instance.  With plain
gradient steps the two trajectories agree to FP32 accuracy; Adam rescales every coordinate by its
own gradient history, so coordinates whose gradient is below FP32 resolution may move either way,
and for Adam the test checks instead that the exact objective (dense, FP64) goes down.
"""
import sys

import numpy as np
import pytest

import oracle
import oracle.pmmf_oracle as om
import workloads
from helpers import grid_sub_instance, import_oracle, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1507_04396_amd import _lib
    _lib.load()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _device_csr(A):
    return (torch.from_numpy(A.rowptr).cuda(), torch.from_numpy(A.colind).cuda(),
            torch.from_numpy(A.val).cuda())


@pytest.mark.parametrize("nrhs", [1, 7, 64, 65])
def test_spmm_matches_scipy(nrhs):
    from paper_1507_04396_amd.refine import spmm
    dense = workloads.random_symmetric(97, density=0.1, seed=4).to_dense()
    dense[5, :] = 0.0
    dense[:, 5] = 0.0  # an empty row
    A = workloads.csr_from_dense(dense)
    X = workloads.gaussian_block(A.n, nrhs, seed=11)
    _say(f"[spmm] n={A.n} nnz={A.nnz} nrhs={nrhs}")
    Y = spmm(*_device_csr(A), torch.from_numpy(X).cuda()).cpu().numpy()
    ref = A.to_scipy().astype(np.float64) @ X.astype(np.float64)
    assert rel_err(Y, ref) <= 1e-6
    assert np.all(Y[5] == 0.0)


def _fp64_steps(ref, A, theta0, hdiag0, hcore0, probes, lr):
    """Plain gradient steps in FP64 on (1/N) ||A X - A~ X||_F^2 (oracle apply and adjoint)."""
    A64 = A.to_scipy().astype(np.float64)
    th, hd, hc = theta0.copy(), hdiag0.copy(), hcore0.copy()
    losses = []
    for X in probes:
        X = X.astype(np.float64)
        f = om.with_angles(ref, th, hd, hc)
        R = om.apply(f, X) - A64 @ X
        N = X.shape[1]
        losses.append(float((R * R).sum() / N))
        _, hdb, hcb, thb = om.backward(f, X, 2.0 * R / N)
        th -= lr * thb
        hd -= lr * hdb
        hc -= lr * hcb
    return np.array(losses), th, hd, hc


def test_sgd_refinement_matches_fp64_loop():
    from paper_1507_04396_amd.refine import AngleRefiner
    A = grid_sub_instance()
    ref = oracle.factor(A, k=2, eta=0.5, core=64, cluster=(256, 512), seed=0)
    fac = import_oracle(ref)
    th0, hd0, hc0 = (t.cpu().numpy().astype(np.float64) for t in fac.params())
    probes = [workloads.gaussian_block(A.n, 16, seed=3000 + t) for t in range(3)]
    lr = 1e-4
    _say("[refine] gpu: 3 plain gradient steps")
    R = AngleRefiner(fac, *_device_csr(A), lr=lr, optimizer="sgd")
    hist = R.run(3, lambda t: torch.from_numpy(probes[t]).cuda()).cpu().numpy()
    th, hd, hc = (t.detach().cpu().numpy().astype(np.float64)
                  for t in (R.theta, R.hdiag, R.hcore))
    _say("[refine] fp64 oracle loop")
    l_ref, th_ref, hd_ref, hc_ref = _fp64_steps(ref, A, th0, hd0, hc0, probes, lr)
    _say(f"[refine] losses gpu {hist} fp64 {l_ref}")
    assert np.all(np.abs(hist - l_ref) <= 1e-5 * np.abs(l_ref))
    # the parameters moved, and moved as in FP64
    for got, want, start in ((th, th_ref, th0), (hd, hd_ref, hd0), (hc, hc_ref, hc0)):
        step = np.linalg.norm(want - start)
        assert step > 0.0
        assert np.linalg.norm(got - want) <= 1e-3 * step + 1e-6 * np.linalg.norm(want)
    # the handle follows the refined parameters
    th_h, hd_h, hc_h = (t.cpu().numpy() for t in fac.params())
    assert np.abs(hd_h - R.hdiag.detach().cpu().numpy()).max() == 0.0
    assert np.abs(th_h - R.theta.detach().cpu().numpy()).max() <= 1e-6


def test_adam_refinement_lowers_exact_objective():
    from paper_1507_04396_amd.refine import AngleRefiner
    A = grid_sub_instance()
    ref = oracle.factor(A, k=2, eta=0.5, core=64, cluster=(256, 512), seed=0)
    fac = import_oracle(ref)
    Ad = A.to_scipy().toarray().astype(np.float64)

    def exact(params):
        th, hd, hc = (t.detach().cpu().numpy().astype(np.float64) for t in params)
        D = Ad - om.dense_reconstruction(om.with_angles(ref, th, hd, hc))
        return float((D * D).sum())

    before = exact(fac.params())
    _say("[refine] gpu: 30 Adam steps, 64 probes")
    R = AngleRefiner(fac, *_device_csr(A), lr=1e-3, optimizer="adam")
    hist = R.run(30, 64, seed=7).cpu().numpy()
    after = exact((R.theta, R.hdiag, R.hcore))
    _say(f"[refine] exact objective {before:.6g} -> {after:.6g}; probe losses {hist[0]:.6g} .. "
         f"{hist[-1]:.6g}")
    assert np.all(np.isfinite(hist))
    assert after < before
