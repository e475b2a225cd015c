"""Pins of the oracle's planar lateral average and of the velocity-split
source S - Sbar (Appendix A): plane means of fields built here with known
means, zero sums per plane and per radius, and the split projection's
invariants (a right-hand side with zero mean before any de-meaning, and the
split constraint met by the projected velocity)."""
import numpy as np
import pytest

import oracle
from paper_1908_03634_amd import workloads as W
from tests import pins

BCS = [(0, 0, 1), (1, 1, 1), (0, 0, 0), (1, 0, 1)]


def test_plane_average_of_known_plane_means():
    nx, ny, nz = 10, 6, 8
    rng = np.random.default_rng(4)
    f = rng.normal(size=nz)
    a = rng.normal(size=(nz, ny, nx))
    zero_mean = a - a.mean(axis=(1, 2), keepdims=True)
    phi = f[:, None, None] + zero_mean
    assert np.allclose(oracle.plane_average(phi), f, rtol=0, atol=1e-14)
    assert np.array_equal(oracle.plane_average(np.ones((nz, ny, nx))), np.ones(nz))


@pytest.mark.parametrize("geometry,shape", [(0, (10, 6, 8)), (2, (12, 10, 6)), (2, (8, 8, 8))])
def test_split_source_sums_to_zero_on_every_plane_or_radius(geometry, shape):
    nx, ny, nz = shape
    S = W.random_cells(nx, ny, nz, 91)
    s_eff, sbar = oracle.split_source(geometry, S)
    if geometry == 0:
        sums = s_eff.sum(axis=(1, 2))
        assert np.allclose(S - s_eff, np.broadcast_to(sbar[:, None, None], S.shape), rtol=0, atol=1e-15)
    else:
        m = oracle.radius_index(nx, ny, nz)
        sums = np.bincount(m.ravel(), weights=s_eff.ravel(), minlength=len(sbar))
        assert np.allclose(S - s_eff, sbar[m], rtol=0, atol=1e-15)
    assert np.abs(sums).max() <= 1e-13 * np.abs(S).sum()


@pytest.mark.parametrize("bc", BCS)
def test_split_projection_has_a_mean_free_rhs_and_meets_the_split_constraint(bc):
    p = W.planar_problem(nx=8, ny=6, nz=10, contrast=1e3, bc=bc, seed=92)
    r = oracle.mac_project(p, tol=1e-13, split=True)
    g = r["grid"]
    b0 = r["beta0_cc"]
    scale = np.abs(oracle.beta0_divergence(g, b0, p.ux, p.uy, p.uz)).max()
    assert abs(r["mean"]) <= 1e-14 * scale
    # D(beta0 U) of the projected velocity, assembled here from the incidence matrix
    fx = np.zeros_like(r["ux"])
    fy = np.zeros_like(r["uy"])
    fz = np.zeros_like(r["uz"])
    for f, u, ax, per in ((fx, r["ux"], 2, bc[0] == 0), (fy, r["uy"], 1, bc[1] == 0), (fz, r["uz"], 0, bc[2] == 0)):
        if per:
            f[...] = 0.5 * (b0 + np.roll(b0, 1, axis=ax)) * u
        else:
            sl_in = [slice(None)] * 3
            sl_in[ax] = slice(1, -1)
            lo = [slice(None)] * 3
            lo[ax] = slice(0, -1)
            hi = [slice(None)] * 3
            hi[ax] = slice(1, None)
            f[tuple(sl_in)] = 0.5 * (b0[tuple(lo)] + b0[tuple(hi)]) * u[tuple(sl_in)]
    D = pins.divergence_matrix(g.nx, g.ny, g.nz, g.h, g.bc)
    div = (D @ np.concatenate([fx.ravel(), fy.ravel(), fz.ravel()])).reshape(b0.shape)
    assert np.abs(div - b0 * r["S_eff"]).max() <= 1e-9 * scale


def test_split_projection_on_the_irregular_star():
    p = W.spherical_problem(16, base="irregular", seed=93)
    r = oracle.mac_project(p, tol=1e-13, split=True)
    scale = np.abs(oracle.beta0_divergence(r["grid"], r["beta0_cc"], p.ux, p.uy, p.uz)).max()
    assert abs(r["mean"]) <= 1e-14 * scale
    d = oracle.beta0_divergence(r["grid"], r["beta0_cc"], r["ux"], r["uy"], r["uz"])
    assert np.abs(d - r["beta0_cc"] * r["S_eff"]).max() <= 1e-9 * scale
