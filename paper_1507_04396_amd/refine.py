"""Gradient refinement of a factorization's rotation angles and H.

Eq. 1 measures a factorization by ||A - A~||_F^2 with A~ = U^T H U.  For probes x ~ N(0, I),
E ||A x - A~ x||^2 = ||A - A~||_F^2, so the mean over N probes of ||A x_r - A~ x_r||^2 is an
unbiased (Hutchinson) estimate of that objective.  Its gradient in the angles theta and in H comes
from mmf_backward (through MMFApply), A x from mmf_spmm, and the step from a torch optimizer.
Every step hands the new theta to the library, which re-derives each rotation (mmf_set_params)
before the next product: a Givens angle gives (cos, sin); the three angles w of a 3-point rotation
give expm(w_0 G_01 + w_1 G_02 + w_2 G_12) O0, O0 being the rotation the search found.
"""
from __future__ import annotations

from typing import Callable, Optional, Union

import torch

from . import _lib
from ._lib import check
from .api import Factorization, MMFApply, _ptr, _require_device, _stream


def spmm(rowptr: torch.Tensor, colind: torch.Tensor, val: torch.Tensor, x: torch.Tensor,
         out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Y = A X through mmf_spmm (A in device CSR, X row-major float32 [n][nrhs])."""
    _require_device(rowptr, torch.int64, "rowptr")
    _require_device(colind, torch.int32, "colind")
    _require_device(val, torch.float32, "val")
    x2 = x.contiguous()
    if x2.dim() == 1:
        x2 = x2[:, None]
    _require_device(x2, torch.float32, "x")
    n = rowptr.numel() - 1
    if x2.shape[0] != n:
        raise ValueError("x must have n rows")
    y = torch.empty_like(x2) if out is None else out
    check(_lib.load().mmf_spmm(n, _ptr(rowptr), _ptr(colind), _ptr(val), _ptr(x2), _ptr(y),
                               x2.shape[1], x2.stride(0), _stream(stream)))
    return y[:, 0] if x.dim() == 1 else y


class AngleRefiner:
    """Minimises the probe estimate of ||A - U(theta)^T H U(theta)||_F^2 over theta (and H).

    fac: a Factorization of A (k = 2 or 3); (rowptr, colind, val): A in device CSR.  optimizer is
    "adam" (torch.optim.Adam) or "sgd" (torch.optim.SGD); refine_h also moves H's retired
    diagonal and core.  The handle's parameters follow the refined values after every step.
    """

    def __init__(self, fac: Factorization, rowptr: torch.Tensor, colind: torch.Tensor,
                 val: torch.Tensor, lr: float = 1e-3, optimizer: str = "adam",
                 refine_h: bool = True):
        self.fac = fac
        self.A = (rowptr, colind, val)
        theta, hdiag, hcore = fac.params()
        self.theta = theta.clone().requires_grad_(True)
        self.hdiag = hdiag.clone().requires_grad_(refine_h)
        self.hcore = hcore.clone().requires_grad_(refine_h)
        params = [self.theta] + ([self.hdiag, self.hcore] if refine_h else [])
        if optimizer == "adam":
            self.opt = torch.optim.Adam(params, lr=lr)
        elif optimizer == "sgd":
            self.opt = torch.optim.SGD(params, lr=lr)
        else:
            raise ValueError(f"unknown optimizer {optimizer!r}")

    def loss(self, X: torch.Tensor) -> torch.Tensor:
        """(1/N) ||A X - A~ X||_F^2 for probes X [n][N] (differentiable in theta and H)."""
        with torch.no_grad():
            AX = spmm(*self.A, X)
        Y = MMFApply.apply(X, self.theta, self.hdiag, self.hcore, self.fac)
        R = Y - AX
        return (R * R).sum() / X.shape[1]

    def step(self, X: torch.Tensor) -> torch.Tensor:
        """One optimizer step on probes X; returns the loss before the step (device scalar)."""
        self.opt.zero_grad(set_to_none=True)
        L = self.loss(X)
        L.backward()
        self.opt.step()
        self.fac.set_params(theta=self.theta.detach(), hdiag=self.hdiag.detach(),
                            hcore=self.hcore.detach())
        return L.detach()

    def run(self, steps: int, probes: Union[int, Callable[[int], torch.Tensor]],
            seed: int = 0) -> torch.Tensor:
        """`steps` steps, each on fresh probes: `probes` is N (standard normal probes drawn on the
        device from a generator seeded with `seed`) or a function step -> X.  Returns the losses
        before each step (device tensor)."""
        gen = None
        if not callable(probes):
            gen = torch.Generator(device="cuda")
            gen.manual_seed(seed)
        hist = []
        for t in range(steps):
            if gen is not None:
                X = torch.randn(self.fac.n, int(probes), generator=gen, device="cuda")
            else:
                X = probes(t)
            hist.append(self.step(X))
        return torch.stack(hist) if hist else torch.empty(0, device="cuda")
