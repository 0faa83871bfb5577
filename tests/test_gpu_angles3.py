"""Angles of 3-point rotations (O_t = expm(W(w_t)) O0_t): the GPU angle gradient of mmf_backward
against the oracle's (series form of the derivative of the exponential map) at w = 0 and at
random w, the rotations mmf_set_params forms from w (Rodrigues, FP64) against scipy's expm, and
angle refinement of a k = 3 factorization lowering the probe loss."""
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


@pytest.fixture(scope="module")
def case():
    A = grid_sub_instance()
    ref = oracle.factor(A, k=3, eta=0.5, core=64, cluster=(256, 512), seed=0)
    return A, ref


@pytest.mark.parametrize("scale", [0.0, 0.2])
def test_k3_angle_gradient_and_rotations_match_oracle(case, scale):
    A, ref = case
    fac = import_oracle(ref)
    R = len(ref.rotations)
    rng = np.random.default_rng(11)
    w = (scale * rng.standard_normal((R, 3))).astype(np.float32)
    X = workloads.gaussian_block(A.n, 16, seed=1000)
    Yb = workloads.gaussian_block(A.n, 16, seed=1001)
    if scale > 0:
        fac.set_params(theta=torch.from_numpy(w).cuda())
    moved = om.with_params3(ref, w.astype(np.float64))
    _say(f"[angles3] scale {scale}: apply after the angles")
    y = fac.apply(torch.from_numpy(X).cuda()).cpu().numpy()
    assert rel_err(y, oracle.apply(moved, X.astype(np.float64))) <= 1e-5
    _say(f"[angles3] scale {scale}: backward")
    xb, hdb, hcb, thb = fac.backward(torch.from_numpy(X).cuda(), torch.from_numpy(Yb).cuda())
    assert thb.shape == (R, 3)
    rx, rhd, rhc, rth = oracle.backward(moved, X.astype(np.float64), Yb.astype(np.float64),
                                        theta=w.astype(np.float64))
    assert rel_err(xb.cpu().numpy(), rx) <= 1e-5
    assert rel_err(hdb.cpu().numpy(), rhd) <= 1e-5
    assert rel_err(thb.cpu().numpy(), rth) <= 1e-4
    th, _, _ = fac.params()
    assert np.array_equal(th.cpu().numpy(), w if scale > 0 else np.zeros_like(w))
    fac.close()


def test_k3_angle_refinement_lowers_the_probe_loss():
    from paper_1507_04396_amd.api import Factorization
    from paper_1507_04396_amd.refine import AngleRefiner
    A = workloads.knn_points_matrix(600, 2, 8, 0.01, 5)
    fac = Factorization.from_csr(A, k=3, core=40, cluster=(32, 128), seed=1)
    dev = "cuda"
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.colind.astype(np.int32)).to(dev)
    cv = torch.from_numpy(A.val).to(dev)
    ref_probes = torch.randn(A.n, 256, generator=torch.Generator(device=dev).manual_seed(3),
                             device=dev)
    R = AngleRefiner(fac, rp, ci, cv, lr=1e-3)
    before = R.loss(ref_probes).item()
    R.run(30, 64, seed=1)
    after = R.loss(ref_probes).item()
    _say(f"[angles3] refinement: probe loss {before:.6f} -> {after:.6f}")
    assert after < before
    fac.close()
