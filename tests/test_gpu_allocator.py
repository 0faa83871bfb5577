"""mmf_set_allocator through torch's caching allocator: the handle's device memory is taken from
torch (visible in torch.cuda.memory_allocated), the factorization and its products are
bit-identical to the hipMalloc path, and every block goes back to torch when the handle is
destroyed, also after the allocator has been switched back (blocks keep their allocator)."""
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


def test_torch_allocator_same_results_and_all_memory_returned():
    from paper_1507_04396_amd.api import Factorization, use_torch_allocator
    A = workloads.knn_points_matrix(600, 2, 8, 0.01, 5)
    params = dict(k=3, core=40, cluster=(32, 128), seed=1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    X = torch.randn(A.n, 16, generator=gen, device="cuda")
    _say("[alloc] reference factorization (hipMalloc)")
    ref = Factorization.from_csr(A, **params)
    e_ref = ref.export()
    y_ref, yi_ref = ref.apply(X), ref.apply(X, inverse=True)
    ref.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    use_torch_allocator(True)
    try:
        _say("[alloc] factorization through torch's caching allocator")
        f = Factorization.from_csr(A, **params)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - base
        assert held > 0
        e = f.export()
        for key, want in e_ref.items():
            assert np.array_equal(e[key], want), key
        y, yi = f.apply(X), f.apply(X, inverse=True)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref) and torch.equal(yi, yi_ref)
        del y, yi
    finally:
        use_torch_allocator(False)  # later allocations: hipMalloc again
    f.close()
    torch.cuda.synchronize()
    _say(f"[alloc] handle held {held} bytes of torch memory; after destroy "
         f"{torch.cuda.memory_allocated() - base}")
    assert torch.cuda.memory_allocated() == base


def test_kept_blocks_reused_on_same_and_other_stream():
    """The default allocator keeps released blocks: a second factorization on the same stream, one
    on another stream, and one after mmf_trim all reproduce the first bit for bit."""
    from paper_1507_04396_amd.api import Factorization, trim_device_cache
    A = workloads.knn_points_matrix(700, 2, 8, 0.01, 6)
    params = dict(k=2, core=40, cluster=(32, 128), seed=2)
    _say("[alloc] first factorization (fresh blocks)")
    f = Factorization.from_csr(A, **params)
    ref = f.export()
    f.close()
    _say("[alloc] second factorization, same stream (kept blocks)")
    f = Factorization.from_csr(A, **params)
    for key, want in ref.items():
        assert np.array_equal(f.export()[key], want), key
    f.close()
    side = torch.cuda.Stream()
    _say("[alloc] factorization on another stream (kept blocks after a device sync)")
    with torch.cuda.stream(side):
        f = Factorization.from_csr(A, **params)
        got = f.export()
    side.synchronize()
    for key, want in ref.items():
        assert np.array_equal(got[key], want), key
    f.close()
    _say("[alloc] trim, then a factorization on fresh blocks")
    trim_device_cache()
    f = Factorization.from_csr(A, **params)
    for key, want in ref.items():
        assert np.array_equal(f.export()[key], want), key
    f.close()
