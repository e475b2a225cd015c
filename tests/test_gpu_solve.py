"""GPU solves and projections against the FP64 oracle (small and odd grids,
every boundary combination, both precisions), plus error paths."""
import numpy as np
import pytest
import torch

import oracle
from paper_1908_03634_amd import mproj, workloads as W
from tests import pins
from tests.gpu_util import N, T, context_for, gpu_project, rel, say

pytestmark = pytest.mark.gpu

BCS = [(0, 0, 1), (1, 1, 1), (0, 0, 0), (1, 0, 1)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c1_projection_matches_oracle(precision):
    """32^3, periodic x/y, Neumann z, 1e2 contrast: phi within 1e-9 (both sides
    solved to 1e-12), corrected U and the divergence constraint."""
    say("c1", precision)
    p = W.config_problem("c1")
    ref = oracle.mac_project(p, tol=1e-12)
    r = gpu_project(p, precision, rtol=1e-12)
    g = ref["grid"]
    phi = N(r["phi"])
    assert rel(phi, ref["phi"]) < 1e-9
    assert abs(phi.mean()) < 1e-14 * np.abs(phi).max()
    # the oracle's operator on the GPU's phi
    assert oracle.residual_norm(g, ref["cx"], ref["cy"], ref["cz"], ref["rhs"], phi) <= 1.01e-12
    # the corrected velocity equals the oracle's correction applied to the GPU phi
    ux, uy, uz = oracle.velocity_correct(g, ref["cx"], ref["cy"], ref["cz"], ref["beta0_cc"], phi, p.ux, p.uy, p.uz)
    for a, b in ((r["ux"], ux), (r["uy"], uy), (r["uz"], uz)):
        assert np.abs(N(a) - b).max() <= 1e-12 * np.abs(b).max()
    info = r["info"]
    assert info["rel_resid"] <= 1e-12
    assert info["div_defect"] <= 2e-12
    assert info["rhs_mean"] == pytest.approx(ref["mean"], rel=1e-9, abs=1e-14)
    r["ctx"].close()


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(8, 8, 8), (16, 16, 16), (6, 4, 10), (9, 5, 7), (24, 40, 16), (33, 17, 9)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_matches_sparse_lu(bc, shape, precision):
    nx, ny, nz = shape
    say("solve", shape, bc, precision)
    h = 1.0 / nz
    cx, cy, cz = W.random_coefs(nx, ny, nz, bc, 201)
    rhs = W.random_cells(nx, ny, nz, 202)
    ctx = mproj.Context(nx, ny, nz, h=h, bc=bc, precision=precision, rtol=1e-12)
    ctx.set_coefs(T(cx), T(cy), T(cz))
    x, info = ctx.solve(T(rhs))
    x = N(x)
    if nx * ny * nz <= 4096:
        ref = pins.bordered_solve(pins.operator(nx, ny, nz, h, bc, cx, cy, cz), rhs).reshape(x.shape)
    else:
        ref, _ = oracle.solve(oracle.Grid(nx, ny, nz, h, bc), cx, cy, cz, rhs, tol=1e-13)
    assert rel(x, ref) < 1e-9
    assert info["rel_resid"] <= 1e-12
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_spherical_projection_small(precision):
    say("spherical small", precision)
    p = W.spherical_problem(32, seed=303)
    ref = oracle.mac_project(p, tol=1e-12)
    r = gpu_project(p, precision, rtol=1e-12)
    assert rel(N(r["phi"]), ref["phi"]) < 1e-9
    for a, b in ((r["ux"], ref["ux"]), (r["uy"], ref["uy"]), (r["uz"], ref["uz"])):
        assert np.abs(N(a) - b).max() <= 1e-9 * np.abs(b).max()
    r["ctx"].close()


def test_results_are_bitwise_reproducible():
    p = W.config_problem("c1")
    outs = []
    for _ in range(2):
        r = gpu_project(p, "mixed", rtol=1e-10)
        outs.append((N(r["phi"]), N(r["uz"]), r["info"]["rel_resid"]))
        r["ctx"].close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def test_mixed_and_fp64_agree_and_reach_tolerance():
    p = W.planar_problem(64, contrast=1e4, seed=404)
    a = gpu_project(p, "mixed", rtol=1e-10)
    b = gpu_project(p, "fp64", rtol=1e-10)
    say("mixed", a["info"]["outer_iters"], a["info"]["resid_hist"][:4], "fp64", b["info"]["outer_iters"])
    assert a["info"]["rel_resid"] <= 1e-10 and b["info"]["rel_resid"] <= 1e-10
    assert rel(N(a["phi"]), N(b["phi"])) < 1e-7
    a["ctx"].close()
    b["ctx"].close()


def test_warm_start_and_idempotence():
    p = W.planar_problem(32, contrast=1e3, seed=505)
    r = gpu_project(p, "fp64", rtol=1e-12)
    ctx = r["ctx"]
    # projecting the projected velocity again gives phi ~ 0 and leaves U unchanged
    # (its right-hand side is rounding noise, so no relative tolerance is
    # reachable; the stagnation exit is expected)
    ux2, uy2, uz2 = r["ux"].clone(), r["uy"].clone(), r["uz"].clone()
    phi2, info2 = ctx.mac_project(ux2, uy2, uz2, T(p.S), allow_not_converged=True)
    assert np.linalg.norm(N(phi2)) <= 1e-9 * np.linalg.norm(N(r["phi"]))
    assert np.abs(N(uz2) - N(r["uz"])).max() <= 1e-11 * np.abs(N(r["uz"])).max()
    # a converged initial guess needs no further step
    ux3, uy3, uz3 = T(p.ux), T(p.uy), T(p.uz)
    phi3, info3 = ctx.mac_project(ux3, uy3, uz3, T(p.S), phi=r["phi"].clone(), use_initial_guess=True)
    assert info3["outer_iters"] == 0
    ctx.close()


def test_not_converged_reports_and_fills_info():
    p = W.config_problem("c1")
    ctx = context_for(p, "mixed", rtol=1e-12, max_outer=1)
    ctx.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center)
    with pytest.raises(mproj.MprojError) as e:
        ctx.mac_project(T(p.ux), T(p.uy), T(p.uz), T(p.S))
    assert e.value.code == 4
    assert e.value.info["outer_iters"] == 1 and 0 < e.value.info["rel_resid"] < 1
    ctx.close()


def test_nonfinite_source_is_reported():
    p = W.config_problem("c1")
    S = p.S.copy()
    S[3, 3, 3] = np.nan
    ctx = context_for(p, "mixed")
    ctx.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center)
    with pytest.raises(mproj.MprojError) as e:
        ctx.mac_project(T(p.ux), T(p.uy), T(p.uz), T(S))
    assert e.value.code == 5
    ctx.close()


def test_singular_rhs_without_demean():
    n = 8
    cx, cy, cz = W.random_coefs(n, n, n, (0, 0, 1), 7)
    ctx = mproj.Context(n, n, n, precision="fp64", demean=False)
    ctx.set_coefs(T(cx), T(cy), T(cz))
    with pytest.raises(mproj.MprojError) as e:
        ctx.solve(T(np.ones((n, n, n))))
    assert e.value.code == 6
    x, info = ctx.solve(T(W.random_cells(n, n, n, 8, mean_zero=True)))
    assert info["rel_resid"] <= 1e-10
    ctx.close()


def test_zero_rhs_gives_zero():
    n = 16
    ctx = mproj.Context(n, n, n, precision="mixed")
    cx, cy, cz = W.random_coefs(n, n, n, (0, 0, 1), 9)
    ctx.set_coefs(T(cx), T(cy), T(cz))
    x, info = ctx.solve(T(np.zeros((n, n, n))))
    assert not N(x).any() and info["rel_resid"] == 0.0
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape,bc", [((4, 4, 4), (1, 1, 1)), ((4, 4, 4), (0, 0, 1)), ((2, 4, 8), (1, 0, 1)),
                                      ((3, 5, 4), (0, 0, 0)), ((8, 8, 8), (1, 1, 0)), ((16, 8, 8), (0, 1, 0))])
def test_direct_bottom_matches_sparse_lu(precision, shape, bc):
    """Hierarchies that end on a grid of at most 64 cells solve it directly
    through the inverse of L + alpha 1 1^T (single-level grids: the whole
    solve): the answer matches sparse LU and no bottom iteration is counted."""
    nx, ny, nz = shape
    say("direct bottom", shape, bc, precision)
    h = 1.0 / nz
    cx, cy, cz = W.random_coefs(nx, ny, nz, bc, 311)
    rhs = W.random_cells(nx, ny, nz, 312)
    ctx = mproj.Context(nx, ny, nz, h=h, bc=bc, precision=precision, rtol=1e-12)
    ctx.set_coefs(T(cx), T(cy), T(cz))
    x, info = ctx.solve(T(rhs))
    ref = pins.bordered_solve(pins.operator(nx, ny, nz, h, bc, cx, cy, cz), rhs).reshape(nz, ny, nx)
    assert rel(N(x), ref) < 1e-9
    assert info["rel_resid"] <= 1e-12
    assert info["bottom_iters_total"] == 0
    ctx.close()


@pytest.mark.parametrize("precision,coarse_cycle", [("fp64", True), ("fp64", False), ("mixed", True), ("mixed", False)])
@pytest.mark.parametrize("n", [16, 32])
def test_disconnected_bottom_falls_back_to_conjugate_gradients(precision, coarse_cycle, n):
    """Zero x faces on the plane x = 1/2 (walls in x) split every level in
    two, and one cell has no nonzero face: L + alpha 1 1^T is singular on the
    64-cell bottom grid, its inverse is refused and the bottom runs Krylov
    iterations instead, made mean-zero on each connected part (the constants
    on each part are the null space).  The right-hand side is mean-zero on
    each part, so the solve reaches the tolerance; without the per-part
    projection the FP32 V-cycles drift along the second constant."""
    bc = (1, 0, 0)
    cx, cy, cz = W.random_coefs(n, n, n, bc, 321)
    cx[:, :, n // 2] = 0.0
    i, j, k = 2, 3, 5  # isolated cell
    cx[k, j, i] = cx[k, j, i + 1] = 0.0
    cy[k, j, i] = cy[k, (j + 1) % n, i] = 0.0
    cz[k, j, i] = cz[(k + 1) % n, j, i] = 0.0
    rhs = W.random_cells(n, n, n, 322)
    rhs[k, j, i] = 0.0
    for half in (slice(0, n // 2), slice(n // 2, n)):
        m = np.zeros((n, n, n), dtype=bool)
        m[:, :, half] = True
        m[k, j, i] = False
        rhs[m] -= rhs[m].mean()
    say("disconnected bottom", n, precision, coarse_cycle)
    ctx = mproj.Context(n, n, n, h=1.0 / n, bc=bc, precision=precision, rtol=1e-10, coarse_cycle=coarse_cycle)
    ctx.set_coefs(T(cx), T(cy), T(cz))
    x, info = ctx.solve(T(rhs))
    g = oracle.Grid(n, n, n, 1.0 / n, bc)
    assert oracle.residual_norm(g, cx, cy, cz, rhs, N(x)) <= 1e-9
    assert info["bottom_iters_total"] > 0
    ctx.close()


def test_wrong_shapes_are_rejected():
    ctx = mproj.Context(8, 8, 8, precision="fp64")
    with pytest.raises(ValueError):
        ctx.solve(T(np.zeros((8, 8, 9))))
    with pytest.raises(ValueError):
        ctx.solve(T(np.zeros((8, 8, 8))).float())
    ctx.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("shape,bc", [((32, 32, 32), (0, 0, 1)), ((40, 24, 16), (0, 0, 1)), ((48, 48, 48), (1, 1, 1)),
                                      ((128, 64, 64), (0, 0, 1)), ((24, 40, 32), (0, 1, 0)), ((384, 8, 8), (0, 0, 1)),
                                      ((384, 8, 8), (1, 0, 1))])
def test_fused_sweep_is_bitwise_equal_to_per_colour_launches(precision, shape, bc):
    """Both colours in one launch give exactly the bits of one launch per
    colour: the tiled sweep (x_old staged in LDS, red recomputed on a halo
    ring) with smoother="fused", and with "auto" the coarser levels' sweep
    with one red and one black cell per thread (the black cell's other red
    neighbours evaluated again), also on the smallest levels when the coarse
    cycle is off (rows of 96 pairs span two workgroups of the one-launch
    sweep at 384 cells: their x neighbours across the edge are evaluated
    again); the prolongation folded into the first post-smoothing sweep
    either way."""
    nx, ny, nz = shape
    p = W.planar_problem(nz, nx=nx, ny=ny, bc=bc, contrast=1e3, seed=606)

    def run(sm, cc):
        say("smoother", sm, "coarse cycle", cc, shape, bc, precision)
        r = gpu_project(p, precision, rtol=1e-10, smoother=sm, coarse_cycle=cc)
        out = (N(r["phi"]), N(r["uz"]), r["info"]["outer_iters"], r["info"]["resid_hist"])
        r["ctx"].close()
        return out

    for cc in (True, False):
        ref = run("per_colour", cc)
        for sm in ("fused", "auto") if cc else ("auto",):
            out = run(sm, cc)
            assert out[2] == ref[2]
            assert out[3] == ref[3]
            assert np.array_equal(out[0], ref[0])
            assert np.array_equal(out[1], ref[1])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_coarse_cycle_kernel_matches_per_level_launches(precision):
    """The single-workgroup coarse cycle (one-wavefront BiCGStab bottom) against
    one launch per operation on every level: same answer to the tolerance."""
    p = W.planar_problem(64, contrast=1e4, seed=707)
    outs = []
    for cc in (True, False):
        r = gpu_project(p, precision, rtol=1e-12, coarse_cycle=cc)
        outs.append((N(r["phi"]), r["info"]))
        r["ctx"].close()
    say("coarse cycle steps", outs[0][1]["outer_iters"], "per-level steps", outs[1][1]["outer_iters"])
    assert outs[0][1]["rel_resid"] <= 1e-12 and outs[1][1]["rel_resid"] <= 1e-12
    assert rel(outs[0][0], outs[1][0]) < 1e-9
    assert abs(outs[0][1]["outer_iters"] - outs[1][1]["outer_iters"]) <= 1


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("shape,bc", [((64, 64, 64), (0, 0, 1)), ((128, 32, 48), (1, 1, 1)), ((40, 24, 16), (0, 1, 0)),
                                      ((384, 16, 12), (1, 1, 1)), ((512, 12, 10), (0, 0, 1)), ((512, 8, 8), (0, 1, 0)),
                                      ((192, 8, 8), (1, 0, 1)), ((192, 24, 16), (1, 1, 1))])
def test_fused_sweep_bitwise_with_face_coefficients(precision, shape, bc):
    """Caller face coefficients (face mode on every level): the fused sweeps
    ("fused", and "auto" with its one-launch sweep on the coarser levels)
    against one launch per colour."""
    nx, ny, nz = shape
    say("fused vs per-colour, face mode", shape, bc, precision)
    cx, cy, cz = W.random_coefs(nx, ny, nz, bc, 909)
    rhs = W.random_cells(nx, ny, nz, 910)
    outs = []
    for sm in ("per_colour", "fused", "auto"):
        ctx = mproj.Context(nx, ny, nz, h=1.0 / nz, bc=bc, precision=precision, rtol=1e-10, smoother=sm)
        ctx.set_coefs(T(cx), T(cy), T(cz))
        x, info = ctx.solve(T(rhs))
        outs.append((N(x), info["resid_hist"]))
        ctx.close()
    for o in outs[1:]:
        assert o[1] == outs[0][1]
        assert np.array_equal(o[0], outs[0][0])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cell_and_face_coefficient_modes_agree(precision):
    """Mapped coefficients are read as one value per cell on the finest level
    (faces formed on the fly); the same faces passed explicitly give the same
    FP64 operator, so the FP64 path is bitwise equal and the mixed path equal
    to the tolerance."""
    p = W.planar_problem(64, contrast=1e4, seed=808)
    rhs = W.random_cells(64, 64, 64, 811)
    a = context_for(p, precision, rtol=1e-12)
    cx, cy, cz = a.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center)
    xa, ia = a.solve(T(rhs))
    ya = N(a.apply(T(rhs)))
    b = context_for(p, precision, rtol=1e-12)
    b.set_coefs(cx, cy, cz)
    xb, ib = b.solve(T(rhs))
    yb = N(b.apply(T(rhs)))
    assert np.array_equal(ya, yb)
    if precision == "fp64":
        assert np.array_equal(N(xa), N(xb))
    else:
        assert rel(N(xa), N(xb)) < 1e-9
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("rtol", [1e-6, 1e-8, 1e-9, 1e-11])
def test_tolerances_are_reached(precision, rtol):
    """The refinement schedule (predicted cycles per step, a last cycle traded
    for one more finest-level sweep where the prediction leaves room) reaches
    any tolerance: the residual of the GPU phi, evaluated by the oracle's
    operator, is within the requested tolerance, and phi lies within the
    tolerance times a conditioning margin of the oracle's solve at 1e-12."""
    say("tolerance", rtol, precision)
    p = W.planar_problem(64, contrast=1e4, seed=808)
    ref = oracle.mac_project(p, tol=1e-12)
    r = gpu_project(p, precision, rtol=rtol)
    phi = N(r["phi"])
    assert r["info"]["rel_resid"] <= rtol
    assert oracle.residual_norm(ref["grid"], ref["cx"], ref["cy"], ref["cz"], ref["rhs"], phi) <= 1.05 * rtol
    assert rel(phi, ref["phi"]) <= 1e3 * rtol
    r["ctx"].close()


@pytest.mark.parametrize("case", ["nonfinite", "zero", "singular"])
def test_rhs_checks_on_the_blocked_path(case):
    """With the blocked projection kernels in mixed precision (the right-hand
    side kept raw, its mean subtracted by the residual): a non-finite source,
    a zero right-hand side and (demean off) a right-hand side with a mean are
    reported as on the other paths."""
    say("blocked rhs checks", case)
    p = W.planar_problem(nx=128, ny=16, nz=16, contrast=1e3, seed=8100)
    S = p.S.copy()
    kw = {}
    ux, uy, uz = p.ux, p.uy, p.uz
    if case == "nonfinite":
        S[3, 5, 7] = np.inf
    elif case == "zero":
        S = np.zeros_like(S)
        ux, uy, uz = (np.zeros_like(u) for u in (ux, uy, uz))
    else:
        S = S + 1.0
        kw["demean"] = False
    ctx = context_for(p, "mixed", **kw)
    ctx.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center)
    U = [T(u) for u in (ux, uy, uz)]
    if case == "zero":
        phi, info = ctx.mac_project(*U, T(S))
        assert not N(phi).any() and info["rel_resid"] == 0.0 and info["rhs_norm"] == 0.0
        assert all(not N(u).any() for u in U)
    else:
        with pytest.raises(mproj.MprojError) as e:
            ctx.mac_project(*U, T(S))
        assert e.value.code == (5 if case == "nonfinite" else 6)
    # the context still projects a regular right-hand side afterwards
    ref = oracle.mac_project(p, tol=1e-12)
    ctx2 = context_for(p, "mixed", rtol=1e-10)
    ctx2.map_base_state(p.geometry, T(p.beta0_1d), T(p.rho), p.dr, p.center)
    phi2, info2 = ctx2.mac_project(T(p.ux), T(p.uy), T(p.uz), T(p.S))
    assert info2["rel_resid"] <= 1e-10
    assert info2["rhs_mean"] == pytest.approx(ref["mean"], rel=1e-9, abs=1e-14)
    ctx.close()
    ctx2.close()
