"""GPU kernels against the FP64 oracle on identical inputs (small grids that
span several workgroups and ragged tails, every boundary combination)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1908_03634_amd import mproj, workloads as W
from tests.gpu_util import N, T, context_for, gpu_project, rel, say

pytestmark = pytest.mark.gpu

BCS = [(0, 0, 1), (1, 1, 1), (0, 0, 0), (1, 0, 1), (0, 1, 0)]
SHAPES = [(8, 8, 8), (6, 4, 10), (5, 7, 3), (9, 5, 7), (40, 24, 16), (33, 17, 9)]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES)
def test_apply_matches_oracle(bc, shape):
    nx, ny, nz = shape
    say("apply", shape, bc)
    g = oracle.Grid(nx, ny, nz, 1.0 / nz, bc)
    cx, cy, cz = W.random_coefs(nx, ny, nz, bc, 101)
    x = W.random_cells(nx, ny, nz, 102)
    ctx = mproj.Context(nx, ny, nz, h=1.0 / nz, bc=bc, precision="fp64")
    ctx.set_coefs(T(cx), T(cy), T(cz))
    y = N(ctx.apply(T(x)))
    ref = oracle.apply(g, cx, cy, cz, x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    ctx.close()


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES)
def test_coef_grad_matches_oracle(bc, shape):
    nx, ny, nz = shape
    say("coef_grad", shape, bc)
    g = oracle.Grid(nx, ny, nz, 0.25, bc)
    lam = W.random_cells(nx, ny, nz, 111)
    phi = W.random_cells(nx, ny, nz, 112)
    ctx = mproj.Context(nx, ny, nz, h=0.25, bc=bc, precision="fp64")
    got = [N(a) for a in ctx.coef_grad(T(lam), T(phi))]
    ref = oracle.coef_grad(g, lam, phi)
    for a, b in zip(got, ref):
        assert a.shape == b.shape
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    ctx.close()


@pytest.mark.parametrize("bc", [(0, 0, 1), (1, 1, 1), (0, 1, 0)])
@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 5, 7), (40, 24, 16)])
def test_planar_mapping_matches_oracle(bc, shape):
    nx, ny, nz = shape
    say("map planar", shape, bc)
    p = W.planar_problem(nz, nx=nx, ny=ny, bc=bc, contrast=1e4, seed=121)
    r = gpu_project(p, "fp64")
    g = oracle.Grid.of(p)
    b0, (cx, cy, cz) = oracle.map_base_state(g, p.geometry, p.beta0_1d, p.dr, p.center, p.rho)
    for a, b in zip((r["cx"], r["cy"], r["cz"]), (cx, cy, cz)):
        assert np.abs(N(a) - b).max() <= 2e-16 * np.abs(b).max() * 4
    r["ctx"].close()


@pytest.mark.parametrize("n", [8, 16, 22])
def test_spherical_mapping_matches_oracle(n):
    say("map spherical", n)
    p = W.spherical_problem(n, seed=131)
    r = gpu_project(p, "fp64")
    g = oracle.Grid.of(p)
    b0, (cx, cy, cz) = oracle.map_base_state(g, p.geometry, p.beta0_1d, p.dr, p.center, p.rho)
    for a, b in zip((r["cx"], r["cy"], r["cz"]), (cx, cy, cz)):
        assert np.abs(N(a) - b).max() <= 1e-14 * np.abs(b).max()
    r["ctx"].close()


def test_bad_density_is_reported():
    p = W.planar_problem(8, seed=3)
    rho = p.rho.copy()
    rho[2, 3, 4] = -1.0
    ctx = context_for(p, "fp64")
    with pytest.raises(mproj.MprojError) as e:
        ctx.map_base_state(p.geometry, T(p.beta0_1d), T(rho), p.dr, p.center)
    assert e.value.code == 5
    with pytest.raises(mproj.MprojError) as e:
        ctx.mac_project(T(p.ux), T(p.uy), T(p.uz), T(p.S))
    assert e.value.code == 7
    ctx.close()


def test_bad_coefficients_are_reported():
    nx = ny = nz = 8
    cx, cy, cz = W.random_coefs(nx, ny, nz, (0, 0, 1), 5)
    cy[1, 2, 3] = -0.5
    ctx = mproj.Context(nx, ny, nz, precision="fp64")
    with pytest.raises(mproj.MprojError) as e:
        ctx.set_coefs(T(cx), T(cy), T(cz))
    assert e.value.code == 5
    ctx.close()


def test_calls_from_another_stream_are_ordered():
    """A context bound to one stream, called while the caller works on
    another: inputs produced on the caller's stream are read after they are
    written, and the caller's stream sees the outputs of calls that return
    without waiting (operator, coefficient gradient)."""
    nx, ny, nz, bc = 64, 48, 40, (0, 0, 1)
    g = oracle.Grid(nx, ny, nz, 1.0 / nz, bc)
    cx, cy, cz = W.random_coefs(nx, ny, nz, bc, 121)
    x = W.random_cells(nx, ny, nz, 122)
    lam = W.random_cells(nx, ny, nz, 123)
    ctx = mproj.Context(nx, ny, nz, h=1.0 / nz, bc=bc, precision="fp64", stream=torch.cuda.Stream())
    ctx.set_coefs(T(cx), T(cy), T(cz))
    ref_y = oracle.apply(g, cx, cy, cz, x)
    ref_g = oracle.coef_grad(g, lam, x)
    other = torch.cuda.Stream()
    big = torch.ones(1 << 26, dtype=torch.float64, device="cuda:0")
    with torch.cuda.stream(other):
        for _ in range(3):
            xd = T(np.zeros_like(x))
            big.mul_(1.0)  # queue work ahead of the input on the caller's stream
            xd.copy_(T(x))
            y = ctx.apply(xd)
            s_y = y * 1.0  # read on the caller's stream, no explicit wait
            gx, gy, gz = ctx.coef_grad(T(lam), xd)
            s_g = [a * 1.0 for a in (gx, gy, gz)]
        torch.cuda.synchronize()
    assert np.abs(N(s_y) - ref_y).max() <= 1e-13 * np.abs(ref_y).max()
    for a, b in zip(s_g, ref_g):
        assert np.abs(N(a) - b).max() <= 1e-13 * np.abs(b).max()
    ctx.close()
