"""ctypes declarations of the C ABI in include/pmmf.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmmf.so")

MMF_OK = 0
ERRORS = {
    -1: "MMF_EINVAL", -2: "MMF_ENOTSYM", -3: "MMF_ENONFINITE", -4: "MMF_ENOMEM",
    -5: "MMF_EDEVICE", -6: "MMF_ESINGULAR", -7: "MMF_ESTATE", -8: "MMF_ECAPACITY",
}
MMF_CHECK_SYMMETRY = 0x1
MMF_EVEN_CLUSTERS = 0x2
MMF_CUT_CLUSTERS = 0x4
MMF_TWO_ELIMINATIONS = 0x8


class MMFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class mmf_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("eta", ctypes.c_double), ("core_size", ctypes.c_int64),
                ("cluster_min", ctypes.c_int32), ("cluster_max", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("gram_mode", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class mmf_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("core_size", ctypes.c_int64), ("k", ctypes.c_int32),
                ("num_stages", ctypes.c_int32), ("num_rotations", ctypes.c_int64),
                ("max_clusters", ctypes.c_int64), ("loss", ctypes.c_double),
                ("loss_literal", ctypes.c_double), ("fro2_a", ctypes.c_double),
                ("fro2_h", ctypes.c_double), ("trace_a", ctypes.c_double),
                ("trace_h", ctypes.c_double), ("factor_ms", ctypes.c_double)]


class mmf_pcg_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("max_rel_residual", ctypes.c_double), ("solve_ms", ctypes.c_double)]


class mmf_stage_info(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int64), ("rotations", ctypes.c_int64),
                ("clusters", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("max_cluster", ctypes.c_int64), ("max_depth", ctypes.c_int32),
                ("dense_gram", ctypes.c_int32), ("loss", ctypes.c_double),
                ("gram_ms", ctypes.c_double), ("find_ms", ctypes.c_double),
                ("rotate_ms", ctypes.c_double), ("find_bytes", ctypes.c_int64),
                ("bf16_long", ctypes.c_int64), ("bf16_rescored", ctypes.c_int64),
                ("gram_flops", ctypes.c_double), ("gram_useful_flops", ctypes.c_double)]


P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
H = ctypes.c_void_p
# mmf_set_allocator callbacks: alloc(bytes, stream, ctx) -> ptr, release(ptr, stream, ctx)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

SIGNATURES = {
    "mmf_factor": [I64, I64, P, P, P, ctypes.POINTER(mmf_params), P, ctypes.POINTER(H)],
    "mmf_apply": [H, P, P, I64, I64, P],
    "mmf_apply_noalloc": [H, P, P, I64, I64, P],
    "mmf_apply_inverse": [H, P, P, I64, I64, P],
    "mmf_apply_inverse_sqrt": [H, P, P, I64, I64, P],
    "mmf_backward": [H, P, P, P, P, P, P, I64, I64, P],
    "mmf_get_info": [H, ctypes.POINTER(mmf_info)],
    "mmf_get_stage_info": [H, I32, ctypes.POINTER(mmf_stage_info)],
    "mmf_export": [H, P, P, P, P, P, P, P],
    "mmf_import": [I64, I32, I64, I32, P, P, P, P, P, P, P, P, P, P, ctypes.POINTER(H)],
    "mmf_param_ptrs": [H, P, P, P],
    "mmf_get_params": [H, P, P, P, P],
    "mmf_sync_angles": [H, P],
    "mmf_set_params": [H, P, P, P, P],
    "mmf_pcg": [H, I64, P, P, P, P, P, I64, ctypes.c_double, I32, ctypes.c_double, P,
                ctypes.POINTER(mmf_pcg_info)],
    "mmf_pcg_split": [H, I64, P, P, P, P, P, I64, ctypes.c_double, I32, ctypes.c_double, P,
                ctypes.POINTER(mmf_pcg_info)],
    "mmf_spmm": [I64, P, P, P, P, P, I64, I64, P],
    "mmf_graph_capture": [H, I32, P, P, I64, I64, P, ctypes.POINTER(H)],
    "mmf_graph_launch": [H, P],
    "mmf_graph_destroy": [H],
    "mmf_set_tail_rows": [H, I64],
    "mmf_destroy": [H],
    "mmf_set_allocator": [ALLOC_FN, RELEASE_FN, P],
    "mmf_trim": [],
    "mmf_last_error": [],
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libpmmf.so; raises if the library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1507_04396_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "mmf_last_error" else ctypes.c_int
    _lib = lib
    return lib


def check(code: int) -> None:
    if code != MMF_OK:
        msg = load().mmf_last_error()
        raise MMFError(code, msg.decode() if msg else "")
