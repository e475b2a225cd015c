"""Helpers for the GPU tests: move seeded inputs to the device and run the
library on a workloads.Problem."""
import sys

import numpy as np
import torch

from paper_1908_03634_amd import mproj


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev())


def N(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def context_for(p, precision="mixed", **kw):
    return mproj.Context(p.nx, p.ny, p.nz, h=p.h, bc=p.bc, precision=precision, **kw)


def gpu_project(p, precision="mixed", rtol=1e-10, **kw):
    """Map + project on the GPU; returns dict with numpy results and info."""
    ctx = context_for(p, precision, rtol=rtol, **kw)
    cx, cy, cz = ctx.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center)
    ux, uy, uz, S = T(p.ux), T(p.uy), T(p.uz), T(p.S)
    phi, info = ctx.mac_project(ux, uy, uz, S)
    torch.cuda.synchronize()
    out = dict(ctx=ctx, cx=cx, cy=cy, cz=cz, phi=phi, ux=ux, uy=uy, uz=uz, info=info)
    return out


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))
