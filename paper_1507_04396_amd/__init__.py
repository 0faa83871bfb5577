"""MI355X (gfx950) implementation of the pMMF hot path: factorization, matrix-free apply,
inverse and adjoint, behind the C ABI of include/pmmf.h (libpmmf.so)."""
from ._lib import MMFError, LIB_PATH  # noqa: F401


def __getattr__(name):
    # the torch-facing API is imported lazily so that loading the C library does not need torch
    if name in ("Factorization", "MMFApply", "use_torch_allocator", "trim_device_cache"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
