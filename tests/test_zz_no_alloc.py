"""mmf_apply_noalloc (the product for callers that cannot allocate) against mmf_apply.

Called through the C ABI.  Both calls run the same sweep and core kernels on the same inputs, so
the results must be identical bit for bit; the product is also checked against the FP64 oracle's
factorization product.  Two calls in a row, the second with fewer right-hand sides, then the
refusals: before the handle has a sweep plan, and beyond the scratch array's capacity.
"""
import ctypes
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


def _noalloc(fac, X, Y):
    from paper_1507_04396_amd import _lib
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return _lib.load().mmf_apply_noalloc(fac.handle, X.data_ptr(), Y.data_ptr(), X.shape[1],
                                         X.stride(0), stream)


def test_noalloc_apply_equals_apply_twice_then_refuses():
    from paper_1507_04396_amd._lib import ERRORS as MMF_ERRORS
    A = workloads.small_grid((40, 40), seed=2)
    ref = oracle.factor(A, k=2, core=48, cluster=(32, 96), seed=3)
    _say("[noalloc] import the oracle factorization")
    fac = import_oracle(ref)
    X1 = torch.from_numpy(workloads.gaussian_block(A.n, 24, seed=1)).cuda()
    X2 = torch.from_numpy(workloads.gaussian_block(A.n, 5, seed=2)).cuda()
    Y1 = torch.full_like(X1, float("nan"))
    _say("[noalloc] before the sweep plan exists")
    assert MMF_ERRORS[_noalloc(fac, X1, Y1)] == "MMF_ESTATE"
    _say("[noalloc] mmf_apply, 24 columns")
    R1 = fac.apply(X1)
    torch.cuda.synchronize()
    _say("[noalloc] mmf_apply_noalloc, 24 columns")
    assert _noalloc(fac, X1, Y1) == 0
    torch.cuda.synchronize()
    assert torch.equal(Y1, R1)
    assert rel_err(Y1.cpu().numpy(), oracle.apply(ref, X1.cpu().numpy().astype(np.float64))) <= 1e-5
    _say("[noalloc] second call, 5 columns")
    Y2 = torch.full_like(X2, float("nan"))
    assert _noalloc(fac, X2, Y2) == 0
    R2 = fac.apply(X2)
    torch.cuda.synchronize()
    assert torch.equal(Y2, R2)
    assert rel_err(Y2.cpu().numpy(), oracle.apply(ref, X2.cpu().numpy().astype(np.float64))) <= 1e-5
    # 2 |S_1| nrhs floats beyond 2^24: refused before any kernel runs
    s1 = A.n - ref.stages[0]["rotations"]
    nbig = (1 << 24) // (2 * s1) + 1
    _say(f"[noalloc] {nbig} columns (over capacity)")
    Xb = torch.zeros(A.n, nbig, device="cuda")
    Yb = torch.zeros_like(Xb)
    assert MMF_ERRORS[_noalloc(fac, Xb, Yb)] == "MMF_ECAPACITY"
    torch.cuda.synchronize()
    assert torch.count_nonzero(Yb) == 0
