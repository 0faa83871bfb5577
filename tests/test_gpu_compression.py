"""Compression curve (the Fig. 3 analogue): the library's FP64 residual equals ||A - U^T H U||_F^2
formed from the GPU product applied to the identity, the best-rank reference matches an
independent FP64 eigensolver, and the error falls as the core grows."""
import sys

import numpy as np
import pytest

import workloads

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


def _dense(csr):
    n = len(csr.rowptr) - 1
    a = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(csr.rowptr))
    a[rows, csr.colind] = csr.val
    return a


@pytest.mark.parametrize("k", [2, 3])
def test_reported_loss_is_the_reconstruction_error(k):
    from paper_1507_04396_amd.api import Factorization
    A = workloads.small_grid((20, 20), sigma=0.5, shift=0.3, seed=2)
    f = Factorization.from_csr(A, k=k, eta=0.5, core=24, cluster=(16, 64), seed=3)
    n = len(A.rowptr) - 1
    eye = torch.eye(n, dtype=torch.float32, device="cuda")
    at = f.apply(eye).double().cpu().numpy()   # column j of A~ = A~ e_j
    loss = f.info()["loss"]
    f.close()
    err2 = float(((_dense(A) - at) ** 2).sum())
    _say(f"[compression] k={k}: reported {loss:.6e}, from the product {err2:.6e}")
    assert abs(err2 - loss) <= 1e-4 * loss


def test_curve_reference_and_trend():
    from paper_1507_04396_amd.compression import compression_curve, eigenvalues_fp64
    A = workloads.knn_points_matrix(1024, 2, 8, 0.01, 4)
    lam = eigenvalues_fp64(A)
    want = np.linalg.eigvalsh(_dense(A))
    want = want[np.argsort(-np.abs(want), kind="stable")]
    assert np.allclose(lam, want, rtol=0, atol=1e-10 * np.abs(want).max())
    recs = compression_curve(A, [64, 256], k=2, cluster=(128, 512), seed=0, lam=lam)
    for r in recs:
        _say(f"[compression] core {r['core']}: pMMF {r['rel_err']:.4f}, best rank "
             f"{r['best_rel_err']:.4f}, ratio {r['ratio']:.3f}")
        tail = want[r["core"]:]
        assert r["best_rel_err"] == pytest.approx(np.sqrt(tail @ tail / (want @ want)), rel=1e-9)
        assert np.isfinite(r["ratio"]) and r["ratio"] > 0
    assert recs[1]["rel_err"] < recs[0]["rel_err"]
