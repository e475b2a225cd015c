"""Seeded synthetic inputs for the MAC-projection solve.

This module only draws and lays out *inputs*: a 1D base-state table, the cell
density, the unprojected face velocity, the expansion term S and an adjoint
seed w.  It holds none of the projection's arithmetic (no mapping, no face
coefficients, no divergence, no solve), so the oracle and the HIP path can both
be fed from it without sharing any of the method's code.

The inputs stand in for the paper's white-dwarf and hot-bubble workloads (Sec. 4,
whose initial models and microphysics are not available): stratified planar
atmospheres rho0(z) = exp(-z/H) with a 1e2..1e5 top-to-bottom contrast and a
radial star rho0(r) = rho_c (1 + (r/R)^2)^(-5/2).  The density carries a 1e-3
relative perturbation, the face velocity is N(0,1) and S is N(0, (1e-2)^2).

beta0 follows the definition of Sec. 2 (beta0 = rho0(0) exp(int dp0/(Gamma1 p0))):
for an isothermal hydrostatic atmosphere (p0 proportional to rho0) with a
constant Gamma1 = gamma this integral evaluates to beta0 = rho0^(1/gamma) with
rho0(0) = 1, gamma = 5/3.

Layouts (C order, x fastest):
  cell arrays  [nz][ny][nx]
  x faces      [nz][ny][nx + bcx]    (bc = 0 periodic: face i is the low face of
  y faces      [nz][ny + bcy][nx]     cell i, the high face of the last cell is
  z faces      [nz + bcz][ny][nx]     face 0; bc = 1 Neumann: faces 0..n, the
                                      first and last are walls and carry U = 0)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC = 0
NEUMANN = 1
PLANAR = 0
SPHERICAL = 1
SPHERICAL_IRREGULAR = 2
SPHERICAL_QUADRATIC = 3
GAMMA = 5.0 / 3.0

# Seeds: 20190805 + configuration number; the 16^3 finite-difference copy of
# the differentiable configuration adds 100.
SEED_BASE = 20190805


@dataclass
class Problem:
    """One seeded projection problem (all arrays float64, C-contiguous)."""

    name: str
    nx: int
    ny: int
    nz: int
    h: float
    bc: tuple
    geometry: int
    beta0_1d: np.ndarray
    dr: float
    center: tuple
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    S: np.ndarray
    w: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz


def face_shapes(nx, ny, nz, bc):
    """Shapes of the x, y and z face arrays for boundary kinds bc=(bx,by,bz)."""
    bx, by, bz = bc
    return (nz, ny, nx + bx), (nz, ny + by, nx), (nz + bz, ny, nx)


def planar_scale_height(contrast):
    """H such that exp(-z/H) falls by `contrast` between z = 0 and z = 1."""
    return 1.0 / math.log(contrast)


def star_radius_for_contrast(contrast, edge=0.5):
    """R such that (1 + (edge/R)^2)^(-5/2) = 1/contrast."""
    return edge / math.sqrt(contrast ** 0.4 - 1.0)


def _draw_faces(rng, nx, ny, nz, bc):
    sx, sy, sz = face_shapes(nx, ny, nz, bc)
    ux = rng.standard_normal(sx)
    uy = rng.standard_normal(sy)
    uz = rng.standard_normal(sz)
    # Neumann walls carry no normal velocity.
    if bc[0] == NEUMANN:
        ux[:, :, 0] = 0.0
        ux[:, :, -1] = 0.0
    if bc[1] == NEUMANN:
        uy[:, 0, :] = 0.0
        uy[:, -1, :] = 0.0
    if bc[2] == NEUMANN:
        uz[0, :, :] = 0.0
        uz[-1, :, :] = 0.0
    return ux, uy, uz


def _draw_velocity(rng, nx, ny, nz, bc, velocity):
    """Face velocity (MAC projection) or cell-centred velocity (nodal projection)."""
    if velocity == "cells":
        return tuple(rng.standard_normal((nz, ny, nx)) for _ in range(3))
    return _draw_faces(rng, nx, ny, nz, bc)


def planar_problem(n=None, *, nx=None, ny=None, nz=None, contrast=1e4, bc=(PERIODIC, PERIODIC, NEUMANN),
                   seed=SEED_BASE, rho_noise=1e-3, s_sigma=1e-2, u_sigma=1.0, with_w=False, name="planar",
                   velocity="faces"):
    """Plane-parallel atmosphere on the unit-spacing grid h = 1/nz.

    Draw order from numpy's PCG64 `default_rng(seed)`: density noise (cells),
    Ux, Uy, Uz (face shapes, or cell shapes with velocity="cells"), S (cells),
    then w (cells) when requested.
    """
    nx = nx or n
    ny = ny or n
    nz = nz or n
    h = 1.0 / nz
    rng = np.random.default_rng(seed)
    H = planar_scale_height(contrast)
    zc = (np.arange(nz) + 0.5) * h
    rho0 = np.exp(-zc / H)
    beta0_1d = rho0 ** (1.0 / GAMMA)
    xi = rng.standard_normal((nz, ny, nx))
    rho = rho0[:, None, None] * (1.0 + rho_noise * xi)
    del xi
    ux, uy, uz = _draw_velocity(rng, nx, ny, nz, bc, velocity)
    if u_sigma != 1.0:
        ux *= u_sigma
        uy *= u_sigma
        uz *= u_sigma
    S = s_sigma * rng.standard_normal((nz, ny, nx))
    w = rng.standard_normal((nz, ny, nx)) if with_w else None
    return Problem(name=name, nx=nx, ny=ny, nz=nz, h=h, bc=tuple(bc), geometry=PLANAR,
                   beta0_1d=np.ascontiguousarray(beta0_1d), dr=h, center=(0.0, 0.0, 0.0),
                   rho=rho, ux=ux, uy=uy, uz=uz, S=S, w=w,
                   meta=dict(contrast=contrast, H=H, seed=seed, rho_noise=rho_noise, velocity=velocity))


def spherical_n1d(n):
    """Radial table length covering the box corner at dr = h/5, plus two spare cells."""
    return int(math.ceil(5.0 * math.sqrt(3.0) * n / 2.0)) + 2


def spherical_problem(n, *, contrast=1e5, bc=(NEUMANN, NEUMANN, NEUMANN), seed=SEED_BASE,
                      rho_noise=1e-3, s_sigma=1e-2, with_w=False, name="spherical", radial_refine=5,
                      base="linear", velocity="faces"):
    """Full-star box: rho0(r) = (1 + (r/R)^2)^(-5/2) about the box centre.

    base "linear" / "quadratic": the 1D beta0 table lives on r_j = (j + 1/2) dr
    with dr = h/radial_refine (the paper's default uniform spacing is dx/5,
    Sec. 3.1), interpolated linearly or quadratically.  base "irregular": the
    table holds beta0 at the radii h sqrt(0.75 + 2m) of the irregular base
    state (n even; one entry per m).  The cell density is the analytic profile
    at the cell centre times (1 + rho_noise * N(0,1)).  velocity="cells" draws
    a cell-centred velocity (nodal projection) instead of face velocities.
    """
    nx = ny = nz = n
    h = 1.0 / n
    rng = np.random.default_rng(seed)
    R = star_radius_for_contrast(contrast)
    dr = h / radial_refine
    if base == "irregular":
        nm = ((n - 1) ** 2 * 3 - 3) // 8 + 1
        rj = h * np.sqrt(0.75 + 2.0 * np.arange(nm))
        geometry = SPHERICAL_IRREGULAR
    else:
        n1d = spherical_n1d(n) if radial_refine == 5 else int(math.ceil(radial_refine * math.sqrt(3.0) * n / 2.0)) + 2
        rj = (np.arange(n1d) + 0.5) * dr
        geometry = SPHERICAL if base == "linear" else SPHERICAL_QUADRATIC
    beta0_1d = ((1.0 + (rj / R) ** 2) ** -2.5) ** (1.0 / GAMMA)
    center = (0.5, 0.5, 0.5)
    c1 = (np.arange(n) + 0.5) * h - 0.5
    r2 = c1[:, None, None] ** 2 + c1[None, :, None] ** 2 + c1[None, None, :] ** 2
    rho0_cells = (1.0 + r2 / (R * R)) ** -2.5
    del r2
    xi = rng.standard_normal((nz, ny, nx))
    rho = rho0_cells * (1.0 + rho_noise * xi)
    del xi, rho0_cells
    ux, uy, uz = _draw_velocity(rng, nx, ny, nz, bc, velocity)
    S = s_sigma * rng.standard_normal((nz, ny, nx))
    w = rng.standard_normal((nz, ny, nx)) if with_w else None
    return Problem(name=name, nx=nx, ny=ny, nz=nz, h=h, bc=tuple(bc), geometry=geometry,
                   beta0_1d=np.ascontiguousarray(beta0_1d), dr=dr, center=center,
                   rho=rho, ux=ux, uy=uy, uz=uz, S=S, w=w,
                   meta=dict(contrast=contrast, R=R, seed=seed, rho_noise=rho_noise, base=base, velocity=velocity))


# The five workloads: sizes, boundaries and contrasts.
CONFIGS = {
    "c1": dict(kind="planar", n=32, contrast=1e2, precision="fp64"),
    "c2": dict(kind="planar", n=256, contrast=1e4, precision="mixed"),
    "c3": dict(kind="spherical", n=384, contrast=1e5, precision="mixed"),
    "c4": dict(kind="planar", n=128, contrast=1e3, precision="fp64", with_w=True),
    "c5": dict(kind="planar", n=512, contrast=1e5, precision="mixed", with_w=True),
}


def config_problem(name, n=None, seed_offset=0, velocity="faces"):
    """Problem for workload `name` ('c1'..'c5'); `n` overrides the grid size.
    velocity="cells": the same base state and density with a cell-centred
    velocity, the input of the nodal projection (Sec. 3.2 Step 11)."""
    cfg = CONFIGS[name]
    idx = int(name[1:])
    seed = SEED_BASE + idx + seed_offset
    size = n or cfg["n"]
    tag = "" if velocity == "faces" else "-nodal"
    if cfg["kind"] == "planar":
        return planar_problem(size, contrast=cfg["contrast"], seed=seed, with_w=cfg.get("with_w", False),
                              name=f"{name}{tag}-{size}^3", velocity=velocity)
    return spherical_problem(size, contrast=cfg["contrast"], seed=seed, with_w=cfg.get("with_w", False),
                             name=f"{name}{tag}-{size}^3", velocity=velocity)


def fd_copy_problem():
    """16^3 copy of the differentiable workload used for finite differences."""
    return planar_problem(16, contrast=1e3, seed=SEED_BASE + 4 + 100, with_w=True, name="c4-fd-16^3")


def random_coefs(nx, ny, nz, bc, seed, lo=0.5, hi=2.0):
    """Positive random face coefficients in the external face layout (walls 0)."""
    rng = np.random.default_rng(seed)
    sx, sy, sz = face_shapes(nx, ny, nz, bc)
    cx = rng.uniform(lo, hi, sx)
    cy = rng.uniform(lo, hi, sy)
    cz = rng.uniform(lo, hi, sz)
    if bc[0] == NEUMANN:
        cx[:, :, 0] = 0.0
        cx[:, :, -1] = 0.0
    if bc[1] == NEUMANN:
        cy[:, 0, :] = 0.0
        cy[:, -1, :] = 0.0
    if bc[2] == NEUMANN:
        cz[0, :, :] = 0.0
        cz[-1, :, :] = 0.0
    return cx, cy, cz


def random_cells(nx, ny, nz, seed, mean_zero=False):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nz, ny, nx))
    if mean_zero:
        a -= a.mean()
    return a
