"""Differentiable solve: phi = M(c)^+ (rhs - mean(rhs)) behind torch.autograd.

For L(phi) with upstream gradient w = dL/dphi, the operator M = D C G being
symmetric, the adjoint is a second solve with the same hierarchy:
    lam = mean-zero solution of M lam = w - mean(w),
    dL/drhs = lam,
    dL/dc_f = (G lam)_f (G phi)_f     (0 on walls),
the last from dM phi = D dC G phi and D = -G^T.  Both steps run on the GPU
(mp_solve and mp_coef_grad).
"""
from __future__ import annotations

import torch

from .mproj import Context


def _key(ts):
    return tuple((t.data_ptr(), t._version) for t in ts)


def _ensure_coefs(solver: Context, cx, cy, cz):
    k = _key((cx, cy, cz))
    if getattr(solver, "_coef_key", None) != k:
        solver.set_coefs(cx, cy, cz)
        solver._coef_key = k


class MacSolve(torch.autograd.Function):
    """phi = MacSolve.apply(solver, rhs, cx, cy, cz)."""

    @staticmethod
    def forward(ctx, solver, rhs, cx, cy, cz):
        rhs, cx, cy, cz = (t.detach().contiguous() for t in (rhs, cx, cy, cz))
        _ensure_coefs(solver, cx, cy, cz)
        phi, info = solver.solve(rhs)
        ctx.solver = solver
        ctx.info = info
        ctx.save_for_backward(phi, cx, cy, cz)
        return phi

    @staticmethod
    def backward(ctx, w):
        phi, cx, cy, cz = ctx.saved_tensors
        solver = ctx.solver
        _ensure_coefs(solver, cx, cy, cz)
        lam, info = solver.solve(w.detach().contiguous())
        ctx.backward_info = info
        gx, gy, gz = solver.coef_grad(lam, phi)
        return None, lam, gx, gy, gz


def mac_solve(solver, rhs, cx, cy, cz):
    return MacSolve.apply(solver, rhs, cx, cy, cz)
