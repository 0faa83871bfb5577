"""The trailing stages of the products as one launch per direction (mmf_set_tail_rows).

The fused launch applies the same rotations with the same arithmetic in the same order as the
per-stage launches (Sec. 2.4), so every product must agree bit for bit with tail rows 0 (every
stage its own launch), whichever stage the fused part starts at; the products of imported oracle
factorizations are checked against the FP64 oracle in test_gpu_parity.py, and here once more with
the fused part starting after the first stage.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from helpers import import_oracle, rel_err

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


CASES = [
    ("grid40x40_k2", lambda: workloads.small_grid((40, 40), sigma=0.5, shift=0.3, seed=7),
     dict(k=2, core=32, cluster=(16, 64), seed=1)),
    ("knn2d_n1200_k3", lambda: workloads.knn_points_matrix(1200, 2, 8, 0.01, 9),
     dict(k=3, core=48, cluster=(30, 90), seed=2)),
    # first active set above the fused launch's 8192 rows: the fused part starts later
    ("grid96x96_k2", lambda: workloads.small_grid((96, 96), sigma=0.5, shift=0.3, seed=8),
     dict(k=2, core=64, cluster=(32, 128), seed=3)),
]


@pytest.mark.parametrize("name,make,params", CASES, ids=[c[0] for c in CASES])
def test_fused_trailing_stages_equal_per_stage_launches(name, make, params):
    from paper_1507_04396_amd.api import Factorization
    A = make()
    _say(f"[tail] {name}: factor n={A.n}")
    fac = Factorization.from_csr(A, **params)
    sizes = [st["size"] for st in fac.stage_info()]
    _say(f"[tail] {name}: stage sizes {sizes}")
    assert len(sizes) >= 3
    # hand-off points: every stage its own launch, the fused part from stage 3 / stage 2 on, and
    # the default (as early as the limits allow)
    thresholds = [0, sizes[2], sizes[1], 8192]
    for nrhs in (1, 5, 64, 130):
        X = torch.from_numpy(workloads.gaussian_block(A.n, nrhs, seed=nrhs)).cuda()
        outs = {}
        for inv in (False, True, "sqrt"):
            ref = None
            for th in thresholds:
                fac.set_tail_rows(th)
                y = fac.apply(X, inverse=inv)
                torch.cuda.synchronize()
                if ref is None:
                    ref = y
                    continue
                _say(f"[tail] {name}: nrhs={nrhs} inverse={inv} rows<={th}")
                assert torch.equal(y, ref), (nrhs, inv, th, (y - ref).abs().max().item())
            outs[inv] = ref
        # A~^{-1} A~ x = x through the fused products
        fac.set_tail_rows(8192)
        z = fac.apply_inverse(fac.apply(X))
        assert rel_err(z.cpu().numpy(), X.cpu().numpy()) <= 1e-4
    fac.close()


def test_fused_trailing_stages_match_oracle_after_a_per_stage_start():
    A = workloads.small_grid((24, 24), sigma=0.5, shift=0.3, seed=5)
    params = dict(k=2, core=24, cluster=(16, 48), seed=6)
    ref = oracle.factor(A, **params)
    fac = import_oracle(ref)
    sizes = [st["size"] for st in ref.stages]
    assert len(sizes) >= 3
    X = workloads.gaussian_block(A.n, 17, seed=2)
    Xd = torch.from_numpy(X).cuda()
    for th in (sizes[1], sizes[2]):
        fac.set_tail_rows(th)
        _say(f"[tail] oracle import: rows<={th}")
        y = fac.apply(Xd).cpu().numpy()
        assert rel_err(y, oracle.apply(ref, X.astype(np.float64))) <= 1e-5
        yi = fac.apply_inverse(Xd).cpu().numpy()
        cond = np.linalg.cond(ref.hcore)
        assert rel_err(yi, oracle.apply_inverse(ref, X.astype(np.float64))) <= max(1e-5,
                                                                                  1e-7 * cond)
    fac.close()


def test_set_tail_rows_rejects_negative():
    from paper_1507_04396_amd.api import Factorization
    from paper_1507_04396_amd import _lib
    A = workloads.small_grid((12, 12), seed=1)
    fac = Factorization.from_csr(A, k=2, core=10, cluster=(8, 30), seed=1)
    with pytest.raises(Exception):
        fac.set_tail_rows(-1)
    assert _lib.load().mmf_set_tail_rows(fac.handle, 0) == 0
    fac.close()
