"""Pins of the oracle's lateral Average onto a uniform radial base state
(Sec. 3.1: the averages over the radii h sqrt(0.75 + 2m) quadratically
interpolated onto r_j = (j + 1/2) dr), of the velocity-split source of a
uniform spherical base state, and of the full velocity U = U~ + w0 e_r of the
split (Appendix A).

Radii, reached sets and averages are rebuilt here from the cell coordinates
with integer arithmetic and numpy (bincount, unique, polyfit), independently
of the oracle's loops."""
import numpy as np
import pytest

import oracle
from paper_1908_03634_amd import workloads as W


def _offsets(n):
    """Odd offsets 2i + 1 - n of the cell centres from the middle node, in
    units of h / 2."""
    return 2 * np.arange(n) + 1 - n


def _cells(nx, ny, nz, h):
    """(m, r) of every cell: the integer radius index and the distance of the
    cell centre from the middle node, from the coordinates."""
    a, b, c = _offsets(nx), _offsets(ny), _offsets(nz)
    q = c[:, None, None] ** 2 + b[None, :, None] ** 2 + a[None, None, :] ** 2
    assert np.all((q - 3) % 8 == 0)
    m = (q - 3) // 8
    x = a * 0.5 * h
    y = b * 0.5 * h
    z = c * 0.5 * h
    r = np.sqrt(z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2)
    return m, r


def _reached(nx, ny, nz, h, phi):
    """Reached radii (increasing) and the plain average of phi over each."""
    m, _ = _cells(nx, ny, nz, h)
    cnt = np.bincount(m.ravel())
    tot = np.bincount(m.ravel(), weights=phi.ravel())
    idx = np.nonzero(cnt)[0]
    return h * np.sqrt(0.75 + 2.0 * idx), tot[idx] / cnt[idx]


# cubes reach every radius up to the inscribed sphere; flat boxes leave many
# radii of their corner regions unreached
SHAPES = [(16, 16, 16), (14, 10, 6), (12, 8, 20), (24, 4, 4)]


@pytest.mark.parametrize("shape", SHAPES)
def test_uniform_average_reproduces_quadratic_profiles(shape):
    """phi = f(r) quadratic in r: every radius average is f there, so the
    parabola through any three of them is f itself; below the first and
    beyond the last reached radius the end averages are held."""
    nx, ny, nz = shape
    h = 1.0 / max(shape)
    dr = h / 5
    _, r = _cells(nx, ny, nz, h)
    f = lambda x: 2.0 - 3.0 * x + 5.0 * x * x  # noqa: E731
    n1d = int(np.ceil(r.max() / dr)) + 3
    avg = oracle.average_uniform(f(r), h, n1d, dr)
    rj = (np.arange(n1d) + 0.5) * dr
    R, _ = _reached(nx, ny, nz, h, f(r))
    inside = (rj >= R[0]) & (rj <= R[-1])
    assert np.allclose(avg[inside], f(rj[inside]), rtol=1e-12, atol=0)
    assert np.all(avg[rj < R[0]] == avg[np.argmax(rj >= R[0]) - 1])
    assert np.allclose(avg[rj < R[0]], f(R[0]), rtol=1e-13)
    assert np.allclose(avg[rj > R[-1]], f(R[-1]), rtol=1e-13)


@pytest.mark.parametrize("shape", SHAPES)
def test_uniform_average_takes_the_three_reached_radii_around_the_nearest(shape):
    """A cubic profile (the parabola is then only an approximation, so the
    stencil matters) and a rough field: for every table radius, the parabola
    fitted (numpy polyfit) through the reached radius nearest to it and its
    reached neighbours, shifted inward at the ends."""
    nx, ny, nz = shape
    h = 1.0 / max(shape)
    dr = h / 5
    _, r = _cells(nx, ny, nz, h)
    rng = np.random.default_rng(sum(shape))
    for phi in (1.0 + r**3 - 4.0 * r**2, rng.standard_normal(r.shape)):
        n1d = int(np.ceil(r.max() / dr)) + 3
        avg = oracle.average_uniform(phi, h, n1d, dr)
        R, A = _reached(nx, ny, nz, h, phi)
        for j in range(n1d):
            x = (j + 0.5) * dr
            if x <= R[0] or x >= R[-1]:
                continue
            d = np.abs(R - x)
            q = int(np.argmin(d))  # the first of equally near radii: the lower one
            s = min(max(q - 1, 0), len(R) - 3)
            cf = np.polyfit(R[s:s + 3] - x, A[s:s + 3], 2)
            assert avg[j] == pytest.approx(cf[-1], rel=1e-9, abs=1e-9 * np.abs(A).max())


def test_uniform_average_of_shell_values_and_a_single_bump():
    """A field constant on each reached radius (any values) is reproduced at
    the reached radii that coincide with table radii; a bump on one cell
    changes only the table entries whose stencil contains its radius."""
    nx = ny = nz = 8
    h = 1.0 / 8
    m, r = _cells(nx, ny, nz, h)
    base = np.zeros(r.shape)
    n1d = 60
    dr = h / 5
    a0 = oracle.average_uniform(base, h, n1d, dr)
    assert np.array_equal(a0, np.zeros(n1d))
    bump = base.copy()
    bump[3, 4, 5] = 1.0
    a1 = oracle.average_uniform(bump, h, n1d, dr)
    R, _ = _reached(nx, ny, nz, h, base)
    mb = m[3, 4, 5]
    rb = h * np.sqrt(0.75 + 2.0 * mb)
    p = int(np.nonzero(np.isclose(R, rb))[0][0])
    lo, hi = R[max(p - 2, 0)], R[min(p + 2, len(R) - 1)]
    rj = (np.arange(n1d) + 0.5) * dr
    touched = np.nonzero(a1 != 0.0)[0]
    assert len(touched) > 0
    assert np.all((rj[touched] > lo) & (rj[touched] < hi))


@pytest.mark.parametrize("geometry", [1, 3])
def test_uniform_split_source(geometry):
    """S = f(r) quadratic: with the quadratic fill S - Sbar vanishes wherever
    the fill's three table points lie inside the reached radii; with the
    linear fill it is the interpolation error, at most dr^2 max|f''| / 8."""
    n = 16
    h = 1.0 / n
    dr = h / 5
    _, r = _cells(n, n, n, h)
    f = lambda x: 1.0 + 2.0 * x - 6.0 * x * x  # noqa: E731
    n1d = W.spherical_n1d(n)
    s_eff, sbar = oracle.split_source(geometry, f(r), h=h, n1d=n1d, dr=dr)
    rj = (np.arange(n1d) + 0.5) * dr
    R, _ = _reached(n, n, n, h, f(r))
    inside = (rj >= R[0]) & (rj <= R[-1])
    assert np.allclose(sbar[inside], f(rj[inside]), rtol=1e-12, atol=0)
    ok = (r >= h) & (r <= R[-1] - 2 * dr)
    if geometry == 3:
        assert np.abs(s_eff[ok]).max() <= 1e-12
    else:
        err = np.abs(s_eff[ok]).max()
        assert 0.0 < err <= dr * dr * 12.0 / 8.0 * (1 + 1e-9)


def _planar_split_with_w0(bc):
    p = W.planar_problem(nx=8, ny=6, nz=12, contrast=1e3, bc=bc, seed=93)
    res = oracle.mac_project(p, tol=1e-13, split=True)
    g = res["grid"]
    nz, h = p.nz, p.h
    re = np.arange(nz + 1) * h
    rc = (np.arange(nz) + 0.5) * h
    sbar = res["sbar"]
    # psi (the dp0/dt term) chosen so that the integrated source vanishes at the top
    psi0 = float((p.beta0_1d * sbar).sum() / p.beta0_1d.sum())
    psi = np.full(nz, psi0)
    w0 = oracle.w0(0, rc, re, p.beta0_1d, sbar, psi)
    U = oracle.add_w0(g, 0, w0, None, None, res["ux"], res["uy"], res["uz"])
    return p, res, w0, psi, U


@pytest.mark.parametrize("bc", [(0, 0, 1), (1, 1, 1)])
def test_planar_full_velocity_meets_the_constraint(bc):
    """U = U~ + w0 e_z: D(beta0 U) = beta0 (S - psi) cell by cell (the split
    projection to 1e-13 and w0 integrated with a psi that closes the top wall)."""
    p, res, w0, psi, (ux, uy, uz) = _planar_split_with_w0(bc)
    g = res["grid"]
    assert abs(w0[-1]) <= 1e-12 * np.abs(w0).max()
    d = oracle.beta0_divergence(g, res["beta0_cc"], ux, uy, uz)
    want = res["beta0_cc"] * (p.S - psi[:, None, None])
    scale = np.abs(oracle.beta0_divergence(g, res["beta0_cc"], p.ux, p.uy, p.uz)).max()
    assert np.abs(d - want).max() <= 1e-10 * scale
    # only the interior z faces change, by w0 of their edge
    assert np.array_equal(ux, res["ux"]) and np.array_equal(uy, res["uy"])
    dz = uz - res["uz"]
    assert np.array_equal(dz[0], np.zeros_like(dz[0])) and np.array_equal(dz[-1], np.zeros_like(dz[-1]))
    assert np.allclose(dz[1:-1], np.broadcast_to(w0[1:-1, None, None], dz[1:-1].shape), rtol=0, atol=1e-15)


def _sphere_faces(n, h, center):
    """Face-centre coordinates relative to `center`, per axis, for walls on
    every side (faces 0..n along the face axis)."""
    f = np.arange(n + 1) * h
    c = (np.arange(n) + 0.5) * h
    out = []
    for axis in range(3):  # x, y, z faces in (z, y, x) index order
        zz = (f if axis == 2 else c) - center[2]
        yy = (f if axis == 1 else c) - center[1]
        xx = (f if axis == 0 else c) - center[0]
        Z, Y, X = np.meshgrid(zz, yy, xx, indexing="ij")
        out.append((X, Y, Z))
    return out


def test_spherical_w0_faces_for_a_linear_w0_are_exact():
    """Constant beta0 and source s: w0 = s r / 3 on the edges, so the face
    velocity is s (x_f - centre)_d / 3 and D(beta0 U) = beta0 s exactly in
    every cell away from the walls."""
    n = 12
    h = 1.0 / n
    center = (0.5, 0.5, 0.5)
    g = oracle.Grid(n, n, n, h, (1, 1, 1))
    dr = h / 5
    n1d = W.spherical_n1d(n)
    re = np.arange(n1d + 1) * dr
    rc = (np.arange(n1d) + 0.5) * dr
    s = 0.8
    w0 = oracle.w0(1, rc, re, np.full(n1d, 2.0), np.full(n1d, s))
    assert np.allclose(w0, s * re / 3.0, rtol=1e-13, atol=1e-16)
    zx, zy, zz = g.faces()
    ux, uy, uz = oracle.add_w0(g, 1, w0, re, center, zx, zy, zz)
    faces = _sphere_faces(n, h, center)
    for u, (X, Y, Z), axis in ((ux, faces[0], 0), (uy, faces[1], 1), (uz, faces[2], 2)):
        comp = (X, Y, Z)[axis]
        want = s * comp / 3.0
        inner = [slice(None)] * 3
        inner[2 - axis] = slice(1, -1)
        assert np.allclose(u[tuple(inner)], want[tuple(inner)], rtol=1e-12, atol=1e-15)
        wall = [slice(None)] * 3
        wall[2 - axis] = [0, -1]
        assert np.array_equal(u[tuple(wall)], np.zeros_like(u[tuple(wall)]))
    b0 = np.full(g.shape, 2.0)
    d = oracle.beta0_divergence(g, b0, ux, uy, uz)
    assert np.allclose(d[1:-1, 1:-1, 1:-1], 2.0 * s, rtol=1e-12, atol=0)


def test_spherical_w0_faces_interpolate_between_edges():
    """w0 = r^2 on the edges: each face carries w0(r_f) e_r . n_f with w0 linear
    between the edges (error at most dr^2 / 4 against r_f^2), the end value
    held beyond the last edge."""
    n = 10
    h = 1.0 / n
    center = (0.5, 0.5, 0.5)
    g = oracle.Grid(n, n, n, h, (1, 1, 1))
    dr = h / 5
    ne = 30  # edges up to 0.58: the corners lie beyond the last edge
    re = np.arange(ne) * dr
    zx, zy, zz = g.faces()
    ux, uy, uz = oracle.add_w0(g, 1, re**2, re, center, zx, zy, zz)
    faces = _sphere_faces(n, h, center)
    for u, (X, Y, Z), axis in ((ux, faces[0], 0), (uy, faces[1], 1), (uz, faces[2], 2)):
        R = np.sqrt(X**2 + Y**2 + Z**2)
        comp = (X, Y, Z)[axis]
        wr = np.where(R >= re[-1], re[-1] ** 2, R**2)
        want = np.where(R > 0, wr * comp / np.where(R > 0, R, 1.0), 0.0)
        inner = [slice(None)] * 3
        inner[2 - axis] = slice(1, -1)
        err = np.abs(u - want)[tuple(inner)]
        assert err.max() <= dr * dr / 4.0


def test_spherical_full_velocity_converges_at_second_order():
    """beta0 = exp(-r) on the table, a smooth source: D(beta0_f w0 e_r) -
    beta0 (Sbar - psi) on cells between radii 0.1 and 0.4 falls about four
    times per halving of h (w0 integrated on the uniform edges r = e dr)."""
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        dr = h / 5
        n1d = W.spherical_n1d(n)
        re = np.arange(n1d + 1) * dr
        rc = (np.arange(n1d) + 0.5) * dr
        b1 = np.exp(-rc)
        src = np.cos(3.0 * rc)
        w0 = oracle.w0(1, rc, re, b1, src)
        g = oracle.Grid(n, n, n, h, (1, 1, 1))
        center = (0.5, 0.5, 0.5)
        b0 = oracle.fill_beta0(g, 1, b1, dr, center)
        zx, zy, zz = g.faces()
        ux, uy, uz = oracle.add_w0(g, 1, w0, re, center, zx, zy, zz)
        d = oracle.beta0_divergence(g, b0, ux, uy, uz)
        _, r = _cells(n, n, n, h)
        want = b0 * np.cos(3.0 * r)
        sel = (r > 0.1) & (r < 0.4)
        errs.append(np.abs(d - want)[sel].max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
