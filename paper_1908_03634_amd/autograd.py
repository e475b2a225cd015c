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


def _key(solver: Context, ts):
    return (solver.coef_generation,) + tuple((t.data_ptr(), t._version) for t in ts)


def _ensure_coefs(solver: Context, cx, cy, cz):
    """Load (cx, cy, cz) into the solver unless exactly these values are
    loaded already.  The key holds the solver's coefficient generation (bumped
    by every map_base_state and set_coefs, so coefficients replaced by any
    other call are loaded again), and the address and version counter of
    each tensor (an in-place change bumps the version; views and detached
    tensors share it).  The cached tensors are kept alive with the key, so
    no other tensor can take their memory and match it by address."""
    if getattr(solver, "_coef_key", None) != _key(solver, (cx, cy, cz)):
        solver.set_coefs(cx, cy, cz)
        solver._coef_key = _key(solver, (cx, cy, cz))
        solver._coef_refs = (cx, cy, cz)


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
