"""Python surface of the pMMF library: thin wrappers over the C ABI (include/pmmf.h).

Device memory and streams come from PyTorch (ROCm); every step of the factorization and of its
application runs in the HIP kernels of libpmmf.so.  Nothing here computes a part of the method.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import MMFError, check  # noqa: F401


# every callback pair ever installed stays referenced: blocks remember the release function that
# belongs to them, so it must outlive them even after the allocator is switched back
_ALLOCATORS = []


def use_torch_allocator(enable: bool = True) -> None:
    """Route the library's later device allocations through torch's caching allocator
    (mmf_set_allocator); ``enable=False`` restores the library's default allocator for later
    allocations."""
    lib = _lib.load()
    if not enable:
        check(lib.mmf_set_allocator(_lib.ALLOC_FN(), _lib.RELEASE_FN(), None))
        return

    def alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:  # reported by the library as MMF_ENOMEM
            return None

    def release(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    pair = (_lib.ALLOC_FN(alloc), _lib.RELEASE_FN(release))
    _ALLOCATORS.append(pair)
    check(lib.mmf_set_allocator(pair[0], pair[1], None))


def trim_device_cache() -> None:
    """Free the device blocks that the library's default allocator keeps for reuse (mmf_trim)."""
    check(_lib.load().mmf_trim())


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _require_device(t: torch.Tensor, dtype, name: str) -> None:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Factorization:
    """A pMMF factorization A ~ U^T H U held on the GPU (handle-owned)."""

    def __init__(self, handle: ctypes.c_void_p, n: int, k: int, core: int):
        self._h = handle
        self.n = n
        self.k = k
        self.core = core

    # ------------------------------------------------------------------ construction
    @classmethod
    def factor(cls, rowptr: torch.Tensor, colind: torch.Tensor, val: torch.Tensor, *, k: int = 2,
               eta: float = 0.5, core: int = 64, cluster=(0, 0), seed: int = 0,
               check_symmetry: bool = False, even_clusters: bool = False, gram_mode: int = 0,
               cut_clusters: bool = False, elims: int = 1, stream=None) -> "Factorization":
        """mmf_factor on a device CSR (int64 rowptr, int32 colind, float32 val).

        ``cut_clusters`` chooses each stage's cluster boundaries to separate the fewest entries of
        the active matrix (MMF_CUT_CLUSTERS) instead of the seeded sizes; ``elims=2`` retires two
        indices per 3-point rotation (MMF_TWO_ELIMINATIONS)."""
        lib = _lib.load()
        _require_device(rowptr, torch.int64, "rowptr")
        _require_device(colind, torch.int32, "colind")
        _require_device(val, torch.float32, "val")
        n = rowptr.numel() - 1
        prm = _lib.mmf_params(k=k, eta=eta, core_size=core, cluster_min=cluster[0],
                              cluster_max=cluster[1], seed=seed, gram_mode=gram_mode,
                              flags=(_lib.MMF_CHECK_SYMMETRY if check_symmetry else 0)
                              | (_lib.MMF_EVEN_CLUSTERS if even_clusters else 0)
                              | (_lib.MMF_CUT_CLUSTERS if cut_clusters else 0)
                              | (_lib.MMF_TWO_ELIMINATIONS if elims == 2 else 0))
        if elims not in (1, 2):
            raise ValueError("elims must be 1 or 2")
        h = ctypes.c_void_p()
        check(lib.mmf_factor(n, val.numel(), _ptr(rowptr), _ptr(colind), _ptr(val),
                             ctypes.byref(prm), _stream(stream), ctypes.byref(h)))
        return cls(h, n, k, core)

    @classmethod
    def from_csr(cls, csr, device="cuda", **params) -> "Factorization":
        """Factor a host CSR (``workloads.CSR``-like: rowptr, colind, val numpy arrays)."""
        rp = torch.from_numpy(np.ascontiguousarray(csr.rowptr, dtype=np.int64)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(csr.colind, dtype=np.int32)).to(device)
        cv = torch.from_numpy(np.ascontiguousarray(csr.val, dtype=np.float32)).to(device)
        f = cls.factor(rp, ci, cv, **params)
        torch.cuda.current_stream().synchronize()
        return f

    @classmethod
    def import_log(cls, n: int, k: int, core: int, stage_sizes, stage_clusters, cluster_sizes,
                   rot_ids, rot_o, rot_retired, hdiag, core_ids, hcore,
                   stream=None) -> "Factorization":
        """mmf_import from host arrays (mmf_export layout plus stage geometry)."""
        lib = _lib.load()
        ss = np.ascontiguousarray(stage_sizes, dtype=np.int64)
        sc = np.ascontiguousarray(stage_clusters, dtype=np.int64)
        cs = np.ascontiguousarray(cluster_sizes, dtype=np.int64)
        ri = np.ascontiguousarray(rot_ids, dtype=np.int32)
        ro = np.ascontiguousarray(rot_o, dtype=np.float32)
        rr = np.ascontiguousarray(rot_retired, dtype=np.int32)
        hd = np.ascontiguousarray(hdiag, dtype=np.float32)
        ci = np.ascontiguousarray(core_ids, dtype=np.int32)
        hc = np.ascontiguousarray(hcore, dtype=np.float32)
        h = ctypes.c_void_p()
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        check(lib.mmf_import(n, k, core, len(ss), p(ss), p(sc), p(cs), p(ri), p(ro), p(rr),
                             p(hd), p(ci), p(hc), _stream(stream), ctypes.byref(h)))
        return cls(h, n, k, core)

    # ------------------------------------------------------------------ lifecycle
    def close(self) -> None:
        if self._h is not None and self._h.value:
            check(_lib.load().mmf_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise MMFError(-7, "factorization was closed")
        return self._h

    # ------------------------------------------------------------------ introspection
    def info(self) -> dict:
        inf = _lib.mmf_info()
        check(_lib.load().mmf_get_info(self.handle, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _lib.mmf_info._fields_}

    def stage_info(self) -> list:
        out = []
        for p in range(self.info()["num_stages"]):
            si = _lib.mmf_stage_info()
            check(_lib.load().mmf_get_stage_info(self.handle, p, ctypes.byref(si)))
            out.append({f: getattr(si, f) for f, _ in _lib.mmf_stage_info._fields_ if f != "pad"})
        return out

    def export(self) -> dict:
        """Rotation log and H on the host (numpy)."""
        inf = self.info()
        R, k, n, c = inf["num_rotations"], self.k, self.n, self.core
        ids = np.zeros((R, k), np.int32)
        o = np.zeros((R, k, k), np.float32)
        ret = np.zeros(R, np.int32)
        mar = np.zeros(R, np.float32)
        hd = np.zeros(n, np.float32)
        cid = np.zeros(c, np.int32)
        hc = np.zeros((c, c), np.float32)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        check(_lib.load().mmf_export(self.handle, p(ids), p(o), p(ret), p(mar), p(hd), p(cid),
                                     p(hc)))
        return dict(rot_ids=ids, rot_o=o, rot_retired=ret, rot_margin=mar, hdiag=hd,
                    core_ids=cid, hcore=hc)

    # ------------------------------------------------------------------ use
    def _vec_args(self, x: torch.Tensor):
        _require_device(x, torch.float32, "x")
        if x.dim() == 1:
            x = x[:, None]
        if x.shape[0] != self.n:
            raise ValueError("x must have n rows")
        return x, x.shape[1], x.stride(0)

    def apply(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None,
              inverse=False) -> torch.Tensor:
        """Y = U^T H U X, U^T H^-1 U X (inverse=True) or U^T H^-1/2 U X (inverse="sqrt");
        X row-major [n][nrhs]."""
        squeeze = x.dim() == 1
        x2, nrhs, ld = self._vec_args(x.contiguous())
        y = torch.empty_like(x2) if out is None else out
        lib = _lib.load()
        fn = (lib.mmf_apply_inverse_sqrt if inverse == "sqrt"
              else lib.mmf_apply_inverse if inverse else lib.mmf_apply)
        check(fn(self.handle, _ptr(x2), _ptr(y), nrhs, ld, _stream(stream)))
        return y[:, 0] if squeeze else y

    def apply_inverse(self, x: torch.Tensor, out: Optional[torch.Tensor] = None,
                      stream=None) -> torch.Tensor:
        return self.apply(x, out=out, stream=stream, inverse=True)

    def set_tail_rows(self, rows: int) -> None:
        """mmf_set_tail_rows: the products run the trailing stages whose first active set has at
        most ``rows`` rows as one launch per direction (0: every stage as its own launch)."""
        check(_lib.load().mmf_set_tail_rows(self.handle, int(rows)))

    def backward(self, x: torch.Tensor, ybar: torch.Tensor, want=("x", "hdiag", "hcore", "theta"),
                 stream=None):
        """Adjoint of Y = U^T H U X: returns (xbar, hdiag_bar, hcore_bar, theta_bar)."""
        x2, nrhs, ld = self._vec_args(x.contiguous())
        yb = ybar.contiguous()
        if yb.dim() == 1:
            yb = yb[:, None]
        dev = x.device
        R = self.n - self.core
        xb = torch.empty_like(x2) if "x" in want else None
        hdb = torch.empty(self.n, device=dev) if "hdiag" in want else None
        hcb = torch.empty(self.core, self.core, device=dev) if "hcore" in want else None
        na = 3 if self.k == 3 else 1  # angles per rotation
        thb = torch.empty(max(R, 1) * na, device=dev) if "theta" in want else None
        check(_lib.load().mmf_backward(self.handle, _ptr(x2), _ptr(yb), _ptr(xb), _ptr(hdb),
                                       _ptr(hcb), _ptr(thb), nrhs, ld, _stream(stream)))
        if thb is not None:
            thb = thb[:R] if na == 1 else thb[:3 * R].view(R, 3)
        return xb, hdb, hcb, thb

    def pcg(self, rowptr: torch.Tensor, colind: torch.Tensor, val: torch.Tensor,
            b: torch.Tensor, tol: float = 1e-6, max_iter: int = 2000,
            inner_reduction: float = 1e-3, stream=None, split: bool = False):
        """mmf_pcg: solve A X = B with the factorization's inverse as preconditioner
        (``split=True``: mmf_pcg_split, CG on A~^{-1/2} A A~^{-1/2}).

        Returns (X float64 [n][nrhs], info dict)."""
        _require_device(rowptr, torch.int64, "rowptr")
        _require_device(colind, torch.int32, "colind")
        _require_device(val, torch.float32, "val")
        b2 = b.contiguous()
        if b2.dim() == 1:
            b2 = b2[:, None]
        _require_device(b2, torch.float32, "b")
        x = torch.empty(b2.shape, dtype=torch.float64, device=b2.device)
        inf = _lib.mmf_pcg_info()
        fn = _lib.load().mmf_pcg_split if split else _lib.load().mmf_pcg
        check(fn(self.handle, rowptr.numel() - 1, _ptr(rowptr), _ptr(colind), _ptr(val),
                 _ptr(b2), _ptr(x), b2.shape[1], tol, max_iter, inner_reduction,
                 _stream(stream), ctypes.byref(inf)))
        return x, {f: getattr(inf, f) for f, _ in _lib.mmf_pcg_info._fields_ if f != "pad"}

    def capture(self, x: torch.Tensor, y: torch.Tensor, inverse: bool = False,
                stream=None) -> "ProductGraph":
        """mmf_graph_capture: record y = A~ x (or A~^{-1} x) on these buffers as a HIP graph.
        Runs the product once eagerly (y holds it on return)."""
        x2, nrhs, ld = self._vec_args(x)
        _require_device(y, torch.float32, "y")
        if y.shape != x2.shape and not (y.dim() == 1 and x.dim() == 1):
            raise ValueError("y must have the shape of x")
        g = ctypes.c_void_p()
        which = 2 if inverse == "sqrt" else (1 if inverse else 0)
        check(_lib.load().mmf_graph_capture(self.handle, which, _ptr(x2), _ptr(y),
                                            nrhs, ld, _stream(stream), ctypes.byref(g)))
        return ProductGraph(g, self)

    def set_params(self, theta=None, hdiag=None, hcore=None, stream=None) -> None:
        for t, nm in ((theta, "theta"), (hdiag, "hdiag"), (hcore, "hcore")):
            if t is not None:
                _require_device(t, torch.float32, nm)
        check(_lib.load().mmf_set_params(self.handle, _ptr(theta), _ptr(hdiag), _ptr(hcore),
                                         _stream(stream)))

    def params(self, stream=None):
        """Copies of the handle's (theta, hdiag, hcore) as device tensors (mmf_get_params): theta
        is [R] Givens angles (k = 2) or [R][3] angles of the 3-point rotations about the rotations
        as found (k = 3)."""
        R = self.n - self.core
        theta = torch.empty((R,) if self.k == 2 else (R, 3), dtype=torch.float32, device="cuda")
        hdiag = torch.empty(self.n, dtype=torch.float32, device="cuda")
        hcore = torch.empty(self.core, self.core, dtype=torch.float32, device="cuda")
        check(_lib.load().mmf_get_params(self.handle, _ptr(theta), _ptr(hdiag), _ptr(hcore),
                                         _stream(stream)))
        return theta, hdiag, hcore


class ProductGraph:
    """A captured mmf_apply / mmf_apply_inverse (mmf_graph_*); keeps its factorization alive."""

    def __init__(self, g: ctypes.c_void_p, fac: Factorization):
        self._g = g
        self._fac = fac

    def launch(self, stream=None) -> None:
        if self._g is None:
            raise MMFError(-7, "graph was closed")
        check(_lib.load().mmf_graph_launch(self._g, _stream(stream)))

    def close(self) -> None:
        if self._g is not None and self._g.value:
            check(_lib.load().mmf_graph_destroy(self._g))
        self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MMFApply(torch.autograd.Function):
    """y = U(theta)^T H U(theta) x with hand-written backward (mmf_backward)."""

    @staticmethod
    def forward(ctx, x, theta, hdiag, hcore, fac: Factorization):
        # the parameters this product used, kept for the backward: the handle may hold others by
        # then (another forward or set_params on the same factorization)
        params = tuple(t.detach().contiguous().clone() for t in (theta, hdiag, hcore))
        fac.set_params(theta=params[0], hdiag=params[1], hcore=params[2])
        y = fac.apply(x.detach())
        ctx.fac = fac
        ctx.params = params
        ctx.save_for_backward(x)
        return y

    @staticmethod
    def backward(ctx, ybar):
        (x,) = ctx.saved_tensors
        need = ctx.needs_input_grad
        want = tuple(nm for nm, w in zip(("x", "theta", "hdiag", "hcore"), need[:4]) if w)
        th, hd, hc = ctx.params
        ctx.fac.set_params(theta=th, hdiag=hd, hcore=hc)
        xb, hdb, hcb, thb = ctx.fac.backward(x.detach(), ybar.contiguous(), want=want)
        if xb is not None and x.dim() == 1:
            xb = xb[:, 0]
        return xb, thb, hdb, hcb, None
