"""Python front end of the contact solver: projected Gauss-Seidel on a
batch of mixed linear complementarity problems and its adjoint, through the
C ABI (``sim_pgs_*`` in ``include/abadj.h``), with a differentiable wrapper.

  x = pgs(A, b, lo, hi, x0, niter)        # A [B, n, n]; b, lo, hi, x0 [B, n]

Method: the MLCP a = A x + b, lo <= x <= hi of the collision solver
(Sec. 4.1 "Collision resolution", Eq. mlcp), solved by a fixed number of
projected Gauss-Seidel sweeps; the gradient reverses the sweeps with the
adjoint of every operation from the stored sweep vectors (App. C).
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as N
from .sim import _ptr, _stream

_DT = {torch.float32: N.SIM_F32, torch.float64: N.SIM_F64}


def _check(A, b, lo, hi, x0):
    if A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("A must be [batch, n, n]")
    B, n = A.shape[0], A.shape[1]
    for name, v in (("b", b), ("lo", lo), ("hi", hi), ("x0", x0)):
        if v is None:
            continue
        if v.shape != (B, n):
            raise ValueError(f"{name} must be [batch, n] = {(B, n)}")
    for v in (A, b, lo, hi, x0):
        if v is None:
            continue
        if not isinstance(v, torch.Tensor) or v.device.type != "cuda" or v.dtype != A.dtype or not v.is_contiguous():
            raise TypeError("every array must be a contiguous CUDA tensor of A's dtype")
    if A.dtype not in _DT:
        raise TypeError("dtype must be float32 or float64")
    return B, n


def workspace_bytes(batch, n, niter, dtype=torch.float32):
    out = ctypes.c_size_t()
    N.check(N.lib().sim_pgs_workspace_bytes(_DT[dtype], int(batch), int(n), int(niter), ctypes.byref(out)))
    return out.value


def new_workspace(batch, n, niter, dtype=torch.float32, device="cuda"):
    nb = workspace_bytes(batch, n, niter, dtype)
    return torch.empty(max(nb, 1), dtype=torch.uint8, device=device)


def solve(A, b, lo, hi, x0, niter, workspace=None, out=None):
    """niter projected Gauss-Seidel sweeps from x0; with a workspace the
    sweep vectors are kept for adjoint()."""
    B, n = _check(A, b, lo, hi, x0)
    x = torch.empty_like(b) if out is None else out
    ws = workspace
    N.check(N.lib().sim_pgs_solve(_DT[A.dtype], B, n, int(niter), _ptr(A), _ptr(b), _ptr(lo), _ptr(hi), _ptr(x0),
                                  _ptr(x), _ptr(ws), 0 if ws is None else ws.numel(), _stream()))
    return x


def adjoint(A, b, lo, hi, xbar, niter, workspace, out=None):
    """Reverse of solve() from its workspace: returns A_bar, b_bar, lo_bar,
    hi_bar, x0_bar."""
    B, n = _check(A, b, lo, hi, xbar)
    if out is None:
        out = (torch.empty_like(A), torch.empty_like(b), torch.empty_like(b), torch.empty_like(b),
               torch.empty_like(b))
    Ab, bb, lb, hb, x0b = out
    N.check(N.lib().sim_pgs_adjoint(_DT[A.dtype], B, n, int(niter), _ptr(A), _ptr(b), _ptr(lo), _ptr(hi), _ptr(xbar),
                                    _ptr(workspace), workspace.numel(), _ptr(Ab), _ptr(bb), _ptr(lb), _ptr(hb),
                                    _ptr(x0b), _stream()))
    return Ab, bb, lb, hb, x0b


class _PGS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, b, lo, hi, x0, niter):
        A, b, lo, hi, x0 = (t.contiguous() for t in (A, b, lo, hi, x0))
        ws = new_workspace(A.shape[0], A.shape[1], niter, A.dtype, A.device)
        x = solve(A, b, lo, hi, x0, niter, workspace=ws)
        ctx.save_for_backward(A, b, lo, hi)
        ctx.ws, ctx.niter = ws, niter
        return x

    @staticmethod
    def backward(ctx, xbar):
        A, b, lo, hi = ctx.saved_tensors
        Ab, bb, lb, hb, x0b = adjoint(A, b, lo, hi, xbar.contiguous(), ctx.niter, ctx.ws)
        return Ab, bb, lb, hb, x0b, None


def pgs(A, b, lo, hi, x0, niter):
    """Differentiable batched PGS solve (gradients with respect to A, b, lo,
    hi and x0)."""
    return _PGS.apply(A, b, lo, hi, x0, niter)
