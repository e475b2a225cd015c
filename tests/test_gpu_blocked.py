"""Register-blocked finest-level kernels (two x cells and four rows per lane,
z-marching) against the one-cell-per-thread kernels and the oracle.

The blocked smoother and restriction evaluate every cell with the same
arithmetic as the one-cell kernels, so FP64 solves are bitwise equal.  The
blocked FP64 residual sums r^2 in another order, which only moves the last
bits of the norms: FP64 iterates are unaffected (the norms only decide when
to stop), mixed-precision iterates agree bitwise through the first
refinement step (its scale comes from the right-hand side) and to the
tolerance after it."""
import numpy as np
import pytest
import torch

import oracle
from paper_1908_03634_amd import mproj, workloads as W
from tests.gpu_util import N, T, context_for, rel, say

pytestmark = pytest.mark.gpu

BCS = [(0, 0, 1), (1, 1, 1), (0, 0, 0), (1, 0, 1), (0, 1, 0)]
# (nx, ny, nz): one wavefront of columns with a single live row group; ragged
# row groups (ny not a multiple of 16) and plane chunks; several x tiles.
# Strips of 2M cells per lane: M = nx / 128 when the wavefront spans the row
# (1 to 4, x neighbours and a periodic wrap by lane rotation), else tiles
# with halo columns (640: five tiles of pairs; 1024: two tiles of 8 cells).
SHAPES = [(128, 4, 4), (128, 12, 6), (256, 20, 10), (128, 36, 32), (256, 48, 64), (384, 8, 6), (512, 4, 4),
          (640, 8, 4), (1024, 4, 4)]


def _problem(shape, bc, seed):
    nx, ny, nz = shape
    return W.planar_problem(nx=nx, ny=ny, nz=nz, contrast=1e3, bc=bc, seed=seed, rho_noise=0.15)


def _solve(p, precision, blocked, rhs, **kw):
    ctx = context_for(p, precision, blocked=blocked, **kw)
    ctx.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center, want_coefs=False)
    x, info = ctx.solve(T(rhs), allow_not_converged=kw.get("max_outer", 100) < 100)
    out = N(x)
    ctx.close()
    return out, info


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES)
def test_blocked_fp64_solve_is_bitwise_equal(shape, bc):
    say("blocked fp64", shape, bc)
    p = _problem(shape, bc, 4100 + sum(shape))
    rhs = W.random_cells(*shape, 4200 + sum(shape))
    xa, ia = _solve(p, "fp64", True, rhs, rtol=1e-11)
    xb, ib = _solve(p, "fp64", False, rhs, rtol=1e-11)
    assert np.array_equal(xa, xb)
    assert ia["vcycles"] == ib["vcycles"]
    assert ia["rel_resid"] == pytest.approx(ib["rel_resid"], rel=1e-6)
    assert ia["rel_resid"] <= 1e-11


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES)
def test_blocked_mixed_first_step_is_bitwise_equal(shape, bc):
    """One refinement step (restriction, both smoother colours, the zero
    start and the prolongation folded into the post-smoother, all in FP32)."""
    say("blocked mixed step", shape, bc)
    p = _problem(shape, bc, 4300 + sum(shape))
    rhs = W.random_cells(*shape, 4400 + sum(shape))
    xa, _ = _solve(p, "mixed", True, rhs, max_outer=1)
    xb, _ = _solve(p, "mixed", False, rhs, max_outer=1)
    assert np.array_equal(xa, xb)


@pytest.mark.parametrize("bc", [(0, 0, 1), (1, 1, 1)])
@pytest.mark.parametrize("shape", [(128, 36, 32), (256, 48, 64)])
def test_blocked_mixed_solve_matches_oracle(shape, bc):
    say("blocked mixed solve", shape, bc)
    p = _problem(shape, bc, 4500 + sum(shape))
    rhs = W.random_cells(*shape, 4600 + sum(shape))
    xa, ia = _solve(p, "mixed", True, rhs, rtol=1e-11)
    xb, _ = _solve(p, "mixed", False, rhs, rtol=1e-11)
    assert ia["rel_resid"] <= 1e-11
    assert rel(xa, xb) < 1e-9
    g = oracle.Grid(p.nx, p.ny, p.nz, p.h, p.bc)
    beta0 = oracle.fill_beta0(g, p.geometry, p.beta0_1d, p.dr, p.center)
    cx, cy, cz = oracle.face_coefs(g, beta0, p.rho)
    ref, _ = oracle.solve(g, cx, cy, cz, rhs, tol=1e-13)
    assert rel(xa, ref) < 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_blocked_spherical_projection(precision):
    """128^3 spherical star, Neumann walls on every axis, 1e5 contrast: the
    blocked path against the one-cell path and the oracle's projection."""
    say("blocked spherical", precision)
    p = W.spherical_problem(128, contrast=1e5, seed=4700)
    ref = oracle.mac_project(p, tol=1e-12)
    out = {}
    for blocked in (True, False):
        ctx = context_for(p, precision, blocked=blocked, rtol=1e-11)
        ctx.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center, want_coefs=False)
        ux, uy, uz, S = T(p.ux), T(p.uy), T(p.uz), T(p.S)
        phi, info = ctx.mac_project(ux, uy, uz, S)
        out[blocked] = (N(phi), N(ux), info)
        ctx.close()
    (pa, ua, ia), (pb, ub, ib) = out[True], out[False]
    if precision == "fp64":
        assert np.array_equal(pa, pb)
        assert np.array_equal(ua, ub)
    assert ia["rel_resid"] <= 1e-11
    assert ia["div_defect"] <= 2e-11
    assert rel(pa, ref["phi"]) < 1e-8


@pytest.mark.parametrize("nu1,nu2,cycles", [(1, 1, 1), (2, 2, 2), (2, 0, 1), (0, 2, 1), (3, 1, 2)])
def test_blocked_mixed_first_step_smoothing_variants(nu1, nu2, cycles):
    """The refinement update rides on the last smoother pass (plain, or right
    after prolongation when nu2 = 1, or on the second of two V-cycles); with no
    post-smoothing it stays a separate pass."""
    shape, bc = (256, 20, 10), (0, 0, 1)
    say("blocked mixed variants", nu1, nu2, cycles)
    p = _problem(shape, bc, 4800)
    rhs = W.random_cells(*shape, 4801)
    kw = dict(max_outer=1, nu1=nu1, nu2=nu2, cycles_per_outer=cycles)
    xa, _ = _solve(p, "mixed", True, rhs, **kw)
    xb, _ = _solve(p, "mixed", False, rhs, **kw)
    assert np.array_equal(xa, xb)


def test_unaligned_solution_array_uses_one_cell_kernels():
    """A solution array that is only 8-byte aligned cannot take the blocked
    kernels' 16-byte accesses: the one-cell kernels run and the FP64 result
    is bitwise the same."""
    import torch
    shape, bc = (256, 20, 10), (0, 0, 1)
    p = _problem(shape, bc, 4900)
    rhs = W.random_cells(*shape, 4901)
    n = int(np.prod(shape))
    ctx = context_for(p, "fp64", rtol=1e-11)
    ctx.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center, want_coefs=False)
    xa, _ = ctx.solve(T(rhs))
    buf = torch.zeros(n + 1, dtype=torch.float64, device=xa.device)
    xu = buf[1:].view(shape[::-1])
    assert xu.data_ptr() % 16 == 8
    xb, _ = ctx.solve(T(rhs), x=xu)
    assert np.array_equal(N(xa), N(xb))
    ctx.close()


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(128, 12, 6), (128, 36, 32), (256, 20, 10), (256, 48, 64), (384, 12, 10),
                                   (384, 20, 36), (512, 8, 6), (512, 36, 36)])
def test_fused_blocked_sweep_equals_colour_passes(shape, bc):
    """Both colours of a sweep in one out-of-place pass (rows wider than the
    owned ones recomputed, plane chunks started two planes early) equal the two
    in-place colour passes bit for bit, through a refinement step and over a
    full solve: rows of 128 and 256 cells (8 owned rows per workgroup) and of
    384 and 512 cells (6 and 8 cells per lane, 4 owned rows)."""
    say("fused blocked sweep", shape, bc)
    p = _problem(shape, bc, 5000 + sum(shape))
    rhs = W.random_cells(*shape, 5100 + sum(shape))
    for kw in (dict(max_outer=1), dict(rtol=1e-11)):
        xa, ia = _solve(p, "mixed", True, rhs, smoother="fused", **kw)
        xb, ib = _solve(p, "mixed", True, rhs, smoother="per_colour", **kw)
        assert np.array_equal(xa, xb)
        assert ia["vcycles"] == ib["vcycles"]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(256, 64, 32), (512, 16, 16), (1024, 8, 8)])
def test_blocked_face_coefficient_levels(shape, bc):
    """Coarse levels with stored face coefficients also run blocked kernels
    (whole-row strips of 2 and 4 cells, and tiles with halo columns): one
    refinement step equals the one-cell kernels bit for bit, and a full solve
    reaches the tolerance in the same number of cycles."""
    say("blocked face levels", shape, bc)
    p = _problem(shape, bc, 5200 + sum(shape))
    rhs = W.random_cells(*shape, 5300 + sum(shape))
    xa, _ = _solve(p, "mixed", True, rhs, max_outer=1)
    xb, _ = _solve(p, "mixed", False, rhs, max_outer=1)
    assert np.array_equal(xa, xb)
    xa, ia = _solve(p, "mixed", True, rhs, rtol=1e-11)
    xb, ib = _solve(p, "mixed", False, rhs, rtol=1e-11)
    assert ia["vcycles"] == ib["vcycles"] and ia["rel_resid"] <= 1e-11
    assert rel(xa, xb) < 1e-9


@pytest.mark.parametrize("shape,bc", [((128, 64, 32), (0, 0, 1)), ((256, 32, 16), (0, 0, 0)), ((128, 16, 12), (0, 0, 1))])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("split", [False, True])
def test_blocked_projection_kernels(shape, bc, precision, split):
    """Register-blocked right-hand side, velocity correction and defect
    (periodic x and y) against the one-cell kernels (blocked=False): the
    corrected velocity and phi agree to rounding (the partial sums of the
    right-hand side mean are grouped differently), and so does the defect."""
    nx, ny, nz = shape
    say("blocked projection", shape, bc, precision, split)
    p = W.planar_problem(nx=nx, ny=ny, nz=nz, contrast=1e4, bc=bc, seed=9100 + nx + nz)
    outs = []
    for blocked in (True, False):
        ctx = mproj.Context(nx, ny, nz, h=p.h, bc=bc, precision=precision, rtol=1e-12, blocked=blocked)
        ctx.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center, want_coefs=False)
        ux, uy, uz = T(p.ux), T(p.uy), T(p.uz)
        phi, info = ctx.mac_project(ux, uy, uz, T(p.S), split=split,
                                    sbar=torch.zeros(nz, dtype=torch.float64, device="cuda:0") if split else None)
        outs.append((N(phi), N(ux), N(uy), N(uz), info))
        ctx.close()
    a, b = outs
    assert rel(a[0], b[0]) < 1e-10
    for q in (1, 2, 3):
        assert np.abs(a[q] - b[q]).max() <= 1e-10 * np.abs(b[q]).max()
    assert a[4]["rhs_norm"] == pytest.approx(b[4]["rhs_norm"], rel=1e-13)
    assert a[4]["div_defect"] <= 2e-12 and b[4]["div_defect"] <= 2e-12
