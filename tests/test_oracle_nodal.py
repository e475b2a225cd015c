"""Pins of the nodal-projection oracle (Sec. 3.2 Step 11, Appendix A; the
discretisation read as trilinear finite elements on the cells).

Every expected value is computed independently of the oracle's arithmetic:
the closed-form symbol of the constant-coefficient operator, element matrices
by Gauss quadrature of pointwise-evaluated basis functions (tests/nodal_pins),
interpolation from the coarse hat functions evaluated at the fine nodes, a
sparse LU of the bordered system, and second-order convergence to an analytic
potential flow.
"""
import numpy as np
import pytest

import oracle
from oracle import nodal as nd
from paper_1908_03634_amd import workloads as W
from tests import nodal_pins as NP

CASES = [((6, 4, 8), (0, 0, 0)), ((5, 6, 4), (1, 0, 1)), ((4, 4, 6), (1, 1, 1)), ((6, 8, 4), (0, 1, 0))]


def _grid(shape, bc):
    nx, ny, nz = shape
    return oracle.Grid(nx, ny, nz, 1.0 / nz, bc)


def _rand(shape, seed, lo=None, hi=None):
    rng = np.random.default_rng(seed)
    if lo is not None:
        return rng.uniform(lo, hi, shape)
    return rng.standard_normal(shape)


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 10, 4), (12, 4, 6)])
def test_symbol_of_the_constant_coefficient_operator(shape):
    """sigma = 1, periodic: Fourier modes are eigenvectors with eigenvalue
    -(S_x M_y M_z + M_x S_y M_z + M_x M_y S_z) / h^2, S(t) = 2 - 2cos t and
    M(t) = (4 + 2cos t)/6 the symbols of the 1D stiffness and mass matrices."""
    nx, ny, nz = shape
    g = oracle.Grid(nx, ny, nz, 0.37, (0, 0, 0))
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    S = lambda t: 2.0 - 2.0 * np.cos(t)  # noqa: E731
    M = lambda t: (4.0 + 2.0 * np.cos(t)) / 6.0  # noqa: E731
    for mx, my, mz in [(1, 0, 0), (1, 2, 1), (nx // 2, ny // 2, nz // 2), (2, 1, 3)]:
        tx, ty, tz = 2 * np.pi * mx / nx, 2 * np.pi * my / ny, 2 * np.pi * mz / nz
        phi = np.cos(tx * i + ty * j + tz * k + 0.3)
        lam = (S(tx) * M(ty) * M(tz) + M(tx) * S(ty) * M(tz) + M(tx) * M(ty) * S(tz)) / g.h**2
        got = nd.apply(g, np.ones((nz, ny, nx)), phi)
        assert np.abs(got + lam * phi).max() <= 1e-12 * max(lam, 1.0 / g.h**2)


@pytest.mark.parametrize("shape,bc", CASES)
def test_operator_equals_the_quadrature_assembly(shape, bc):
    g = _grid(shape, bc)
    nx, ny, nz = shape
    sigma = _rand((nz, ny, nx), 1, 0.2, 5.0)
    M = NP.operator(nx, ny, nz, g.h, bc, sigma)
    for seed in (2, 3):
        phi = _rand(nd.node_shape(g), seed)
        ref = (M @ phi.ravel()).reshape(phi.shape)
        assert np.abs(nd.apply(g, sigma, phi) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("shape,bc", CASES)
def test_operator_is_symmetric_negative_with_constant_null_space(shape, bc):
    g = _grid(shape, bc)
    nx, ny, nz = shape
    sigma = _rand((nz, ny, nx), 4, 0.2, 5.0)
    u, v = _rand(nd.node_shape(g), 5), _rand(nd.node_shape(g), 6)
    uMv = nd.node_dot(g, u, nd.apply(g, sigma, v))
    vMu = nd.node_dot(g, v, nd.apply(g, sigma, u))
    assert abs(uMv - vMu) <= 1e-12 * abs(uMv)
    assert nd.node_dot(g, u, nd.apply(g, sigma, u)) < 0.0
    assert np.abs(nd.apply(g, sigma, np.full(nd.node_shape(g), 2.5))).max() <= 1e-12 / g.h**2


@pytest.mark.parametrize("shape,bc", CASES)
def test_divergence_gradient_and_load_equal_the_quadrature(shape, bc):
    g = _grid(shape, bc)
    nx, ny, nz = shape
    V = [_rand((nz, ny, nx), 10 + d) for d in range(3)]
    D = NP.divergence(nx, ny, nz, g.h, bc)
    ref = (D @ np.concatenate([v.ravel() for v in V])).reshape(nd.node_shape(g))
    assert np.abs(nd.divergence(g, *V) - ref).max() <= 1e-12 * np.abs(ref).max()
    phi = _rand(nd.node_shape(g), 13)
    G = NP.gradient(nx, ny, nz, g.h, bc)
    gref = (G @ phi.ravel()).reshape(3, nz, ny, nx)
    for a, b in zip(nd.gradient(g, phi), gref):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(gref).max()
    f = _rand((nz, ny, nx), 14)
    L = NP.load(nx, ny, nz, g.h, bc)
    lref = (L @ f.ravel()).reshape(nd.node_shape(g))
    assert np.abs(nd.load(g, f) - lref).max() <= 1e-13 * np.abs(lref).max()


@pytest.mark.parametrize("shape,bc", CASES)
def test_divergence_is_minus_the_gradient_transpose(shape, bc):
    """Summation by parts: sum_n (DV)_n phi_n = -sum_e V_e . (G phi)_e."""
    g = _grid(shape, bc)
    nx, ny, nz = shape
    V = [_rand((nz, ny, nx), 20 + d) for d in range(3)]
    phi = _rand(nd.node_shape(g), 23)
    lhs = float((nd.divergence(g, *V) * phi).sum())
    rhs = -sum(float((v * gphi).sum()) for v, gphi in zip(V, nd.gradient(g, phi)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_gradient_of_a_linear_function_is_its_slope():
    g = oracle.Grid(5, 4, 6, 0.2, (1, 1, 1))
    k, j, i = np.meshgrid(*(np.arange(m) for m in nd.node_shape(g)), indexing="ij")
    phi = 0.3 + 1.5 * i * g.h - 2.0 * j * g.h + 0.25 * k * g.h
    gx, gy, gz = nd.gradient(g, phi)
    assert np.allclose(gx, 1.5, atol=1e-13) and np.allclose(gy, -2.0, atol=1e-13)
    assert np.allclose(gz, 0.25, atol=1e-13)


@pytest.mark.parametrize("shape,bc", [((8, 8, 8), (0, 0, 0)), ((8, 4, 6), (1, 0, 1)), ((4, 6, 8), (1, 1, 1))])
def test_transfers_are_interpolation_and_its_scaled_transpose(shape, bc):
    g = _grid(shape, bc)
    nx, ny, nz = shape
    P = NP.interpolation(nx, ny, nz, bc).toarray()
    cshape = NP.node_shape(nx // 2, ny // 2, nz // 2, bc)
    ec = _rand(cshape, 30)
    base = _rand(nd.node_shape(g), 31)
    got = nd.prolong_add(g, ec, base)
    assert np.abs(got - base - (P @ ec.ravel()).reshape(base.shape)).max() <= 1e-14 * np.abs(got).max()
    rf = _rand(nd.node_shape(g), 32)
    assert np.abs(nd.restrict(g, rf) - (P.T @ rf.ravel() / 8.0).reshape(cshape)).max() <= 1e-14 * np.abs(rf).max()


def test_prolongation_is_exact_for_trilinear_functions():
    g = oracle.Grid(8, 6, 4, 0.25, (1, 1, 1))
    f = lambda x, y, z: 1.0 + 2.0 * x - y + 0.5 * z + 3.0 * x * y - x * y * z  # noqa: E731
    cz, cy, cx = NP.node_shape(4, 3, 2, (1, 1, 1))
    K, J, I = np.meshgrid(np.arange(cz), np.arange(cy), np.arange(cx), indexing="ij")
    ec = f(2.0 * I, 2.0 * J, 2.0 * K)
    k, j, i = np.meshgrid(*(np.arange(m) for m in nd.node_shape(g)), indexing="ij")
    got = nd.prolong_add(g, ec, np.zeros(nd.node_shape(g)))
    assert np.allclose(got, f(1.0 * i, 1.0 * j, 1.0 * k), rtol=1e-14, atol=1e-13)


def test_sigma_coarsening_is_the_mean_of_the_children():
    s = _rand((6, 4, 8), 40, 0.5, 2.0)
    ref = s.reshape(3, 2, 2, 2, 4, 2).mean(axis=(1, 3, 5))
    assert np.allclose(nd.sigma_coarsen(s), ref, rtol=1e-15, atol=0)


def test_right_hand_side_is_the_weak_form_and_sums_to_zero():
    p = W.planar_problem(nx=6, ny=4, nz=8, contrast=1e3, bc=(0, 1, 1), seed=50, velocity="cells")
    g = oracle.Grid.of(p)
    b0 = oracle.fill_beta0(g, p.geometry, p.beta0_1d, p.dr, p.center)
    R, m = nd.rhs(g, b0, p.ux, p.uy, p.uz, p.S)
    assert m == pytest.approx(float((b0 * p.S).mean()), rel=1e-13)
    D = NP.divergence(g.nx, g.ny, g.nz, g.h, g.bc)
    L = NP.load(g.nx, g.ny, g.nz, g.h, g.bc)
    V = np.concatenate([(b0 * u).ravel() for u in (p.ux, p.uy, p.uz)])
    ref = (D @ V - L @ (b0 * p.S - m).ravel()).reshape(R.shape)
    assert np.abs(R - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(R.sum()) <= 1e-12 * np.abs(R).sum()


@pytest.mark.parametrize("shape,bc", [((4, 4, 4), (0, 0, 0)), ((6, 4, 5), (1, 0, 1)), ((16, 16, 16), (0, 0, 1)),
                                      ((16, 8, 12), (1, 1, 1))])
def test_solve_matches_a_sparse_lu_of_the_bordered_system(shape, bc):
    nx, ny, nz = shape
    g = _grid(shape, bc)
    sigma = _rand((nz, ny, nx), 60, 0.1, 10.0)
    R = _rand(nd.node_shape(g), 61)
    phi, info = nd.solve(g, sigma, R, tol=1e-13)
    assert info["converged"]
    ref = NP.solve_gauged(NP.operator(nx, ny, nz, g.h, bc, sigma), R.ravel()).reshape(R.shape)
    assert np.abs(phi - ref).max() <= 1e-10 * np.abs(ref).max()
    assert abs(phi.mean()) <= 1e-13 * np.abs(phi).max()


def test_smooth_flow_is_projected_at_second_order():
    """rho = beta0 = 1, S = 0, U = grad psi sampled at the cell centres (psi a
    periodic trigonometric potential): phi -> psi and the projected U -> 0
    as h^2."""
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        g = oracle.Grid(n, n, n, h, (0, 0, 0))
        c = (np.arange(n) + 0.5) * h
        z, y, x = np.meshgrid(c, c, c, indexing="ij")
        tp = 2 * np.pi
        ux = tp * np.cos(tp * x) * np.sin(tp * y) * np.cos(tp * z)
        uy = tp * np.sin(tp * x) * np.cos(tp * y) * np.cos(tp * z)
        uz = -tp * np.sin(tp * x) * np.sin(tp * y) * np.sin(tp * z)
        ones = np.ones((n, n, n))
        R, _ = nd.rhs(g, ones, ux, uy, uz, np.zeros((n, n, n)))
        phi, info = nd.solve(g, ones, R, tol=1e-13)
        nodes = np.arange(n) * h
        Z, Y, X = np.meshgrid(nodes, nodes, nodes, indexing="ij")
        psi = np.sin(tp * X) * np.sin(tp * Y) * np.cos(tp * Z)
        vx, vy, vz = nd.correct(g, ones, ones, phi, ux, uy, uz)
        errs.append((np.abs(phi - (psi - psi.mean())).max(), max(np.abs(v).max() for v in (vx, vy, vz))))
    (e1, u1), (e2, u2) = errs
    assert e1 < 0.05 and u1 < 0.5
    assert e1 / e2 > 3.5 and u1 / u2 > 3.5


def test_projection_of_a_workload_reaches_the_tolerance():
    p = W.planar_problem(16, contrast=1e4, seed=70, velocity="cells")
    r = nd.project(p, tol=1e-12)
    assert r["info"]["converged"] and r["info"]["rel_resid"] <= 1e-12
    assert nd.residual_norm(r["grid"], r["sigma"], r["R"], r["phi"]) <= 1.01e-12
    # the correction removes sigma/beta0 G phi from U
    gx, gy, gz = nd.gradient(r["grid"], r["phi"])
    w = r["sigma"] / r["beta0"]
    for new, old, gr in ((r["ux"], p.ux, gx), (r["uy"], p.uy, gy), (r["uz"], p.uz, gz)):
        assert np.allclose(old - new, w * gr, rtol=1e-12, atol=1e-14)


def test_pressure_update_reproduces_the_applied_correction():
    """pi = s phi: (sigma/beta0) G(pi) / s is U_dagger - U_new cell by cell,
    and the increment form adds a multiple of the old pi."""
    p = W.planar_problem(12, contrast=1e3, seed=71, velocity="cells")
    r = nd.project(p, tol=1e-12)
    s = 1.0 / 3.0e-3
    pi = nd.update_pi(r["phi"], s)
    gx, gy, gz = nd.gradient(r["grid"], pi)
    w = r["sigma"] / r["beta0"] / s
    for new, old, gr in ((r["ux"], p.ux, gx), (r["uy"], p.uy, gy), (r["uz"], p.uz, gz)):
        assert np.allclose(old - new, w * gr, rtol=1e-11, atol=1e-13)
    old = np.random.default_rng(3).standard_normal(pi.shape)
    inc = nd.update_pi(r["phi"], s, pi=old, a=1.0)
    assert np.allclose(inc, old + pi, rtol=1e-15, atol=1e-15 * np.abs(pi).max())
