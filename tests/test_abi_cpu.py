"""The C-ABI library loads and exports every entry point include/pmmf.h declares; argument
errors are reported before any device work (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmmf.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mmf_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1507_04396_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpmmf.so is not built (python -m paper_1507_04396_amd.build)")
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for want in ["mmf_factor", "mmf_apply", "mmf_apply_inverse", "mmf_backward"]:
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_1507_04396_amd import _lib
    assert sorted(_lib.SIGNATURES) == _declared()


def _factor(lib, n=10, nnz=0, **kw):
    from paper_1507_04396_amd import _lib
    base = dict(k=2, eta=0.5, core_size=2, cluster_min=0, cluster_max=0, seed=0, gram_mode=0,
                flags=0)
    base.update(kw)
    prm = _lib.mmf_params(**base)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    return lib.mmf_factor(n, nnz, dummy, dummy, dummy, ctypes.byref(prm), None, ctypes.byref(h))


@pytest.mark.parametrize("kw", [dict(k=4), dict(eta=0.0), dict(eta=0.7), dict(core_size=0),
                                dict(core_size=11), dict(cluster_min=4, cluster_max=6),
                                dict(cluster_min=1, cluster_max=8), dict(gram_mode=2)])
def test_factor_rejects_bad_params(lib, kw):
    from paper_1507_04396_amd import _lib
    assert _factor(lib, **kw) == -1
    assert lib.mmf_last_error()


def test_factor_rejects_oversized_single_cluster(lib):
    # plain MMF keeps dense c x c cluster state: one cluster of 100000 is refused
    assert _factor(lib, n=100000, core_size=10) == -1
    assert b"limit" in lib.mmf_last_error()


def test_handle_errors(lib):
    from paper_1507_04396_amd import _lib
    inf = _lib.mmf_info()
    assert lib.mmf_get_info(None, ctypes.byref(inf)) == -7
    assert lib.mmf_destroy(None) == -7
    assert lib.mmf_apply(ctypes.c_void_p(12345), None, None, 1, 1, None) == -7


def test_set_allocator_needs_both_functions_or_neither(lib):
    from paper_1507_04396_amd import _lib
    alloc = _lib.ALLOC_FN(lambda nbytes, stream, ctx: None)
    assert lib.mmf_set_allocator(alloc, _lib.RELEASE_FN(), None) == -1
    assert lib.mmf_last_error()
    assert lib.mmf_set_allocator(_lib.ALLOC_FN(), _lib.RELEASE_FN(), None) == 0


def test_trim_with_nothing_kept_is_ok(lib):
    # no block has been released in this process: nothing to free, no device call
    assert lib.mmf_trim() == 0
    assert lib.mmf_last_error() in (b"", None)


def test_cut_clusters_flag_excludes_even_clusters(lib):
    from paper_1507_04396_amd import _lib
    flags = _lib.MMF_EVEN_CLUSTERS | _lib.MMF_CUT_CLUSTERS
    assert _factor(lib, n=32, core_size=4, cluster_min=4, cluster_max=8, flags=flags) == -1
    assert b"exclude" in lib.mmf_last_error()
