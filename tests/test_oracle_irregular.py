"""Pins of the oracle's irregular radial base state (Sec. 3.1): the radius
index of each cell, the lateral Average over the irregular radii, the fill by
index, and the quadratic fill of a uniformly spaced table.

Each check is independent of the oracle's own arithmetic: cell radii from the
cell-centre coordinates computed here, counts by brute force over the cells,
values the paper prints, functions of r whose averages and interpolants are
known exactly."""
import os

import numpy as np
import pytest

import oracle
from paper_1908_03634_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.txt")


def golden():
    vals = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if "=" in line:
            k, v = (s.strip() for s in line.split("="))
            vals[k] = float(v)
    return vals


def radii_over_h(nx, ny, nz):
    """|x - centre| / h of every cell centre, centre at the middle node."""
    x = np.arange(nx) + 0.5 - nx / 2
    y = np.arange(ny) + 0.5 - ny / 2
    z = np.arange(nz) + 0.5 - nz / 2
    return np.sqrt(z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2)


SHAPES = [(8, 8, 8), (12, 10, 6), (16, 16, 16), (6, 14, 10)]


@pytest.mark.parametrize("shape", SHAPES)
def test_radius_index_is_the_papers_radius_set(shape):
    """Every cell centre sits at h sqrt(0.75 + 2m) with the oracle's m."""
    nx, ny, nz = shape
    g = golden()
    m = oracle.radius_index(nx, ny, nz)
    r2 = radii_over_h(nx, ny, nz) ** 2
    assert np.abs(r2 - (g["radius_offset"] + g["radius_step"] * m)).max() < 1e-9
    assert oracle.radius_count(nx, ny, nz) == m.max() + 1


def test_radius_count_matches_the_paper():
    """Sec. 4.1: 24,384 averaging radii at 256^3 and 883,584 at 1536^3 (m_max)."""
    g = golden()
    assert oracle.radius_count(256, 256, 256) - 1 == g["radius_count_256"]
    assert oracle.radius_count(1536, 1536, 1536) - 1 == g["radius_count_1536"]
    assert oracle.radius_count(7, 8, 8) == 0


@pytest.mark.parametrize("shape", SHAPES)
def test_average_counts_cells_per_radius(shape):
    """Brute force: the number of cells whose centre is at each radius."""
    nx, ny, nz = shape
    _, cnt = oracle.average_irregular(np.ones((nz, ny, nx)))
    r2 = np.rint(radii_over_h(nx, ny, nz) ** 2 * 4).astype(np.int64)  # 4 r^2 / h^2 = 8m + 3
    brute = np.zeros(len(cnt))
    for v in r2.ravel():
        brute[(v - 3) // 8] += 1
    assert np.array_equal(cnt, brute)
    assert cnt.sum() == nx * ny * nz


@pytest.mark.parametrize("shape", SHAPES)
def test_average_of_a_radial_function_is_its_value_at_the_radius(shape):
    nx, ny, nz = shape
    r = radii_over_h(nx, ny, nz)
    f = lambda s: np.exp(-0.3 * s) + 0.1 * s**2  # noqa: E731
    avg, cnt = oracle.average_irregular(f(r))
    m = np.arange(len(avg))
    rm = np.sqrt(0.75 + 2 * m)
    on = cnt > 0
    assert np.allclose(avg[on], f(rm[on]), rtol=1e-13, atol=0)
    assert np.all(avg[~on] == 0.0)


def test_average_conserves_the_sum_and_ignores_other_radii():
    nx, ny, nz = 12, 10, 6
    phi = W.random_cells(nx, ny, nz, 77)
    avg, cnt = oracle.average_irregular(phi)
    assert abs((avg * cnt).sum() - phi.sum()) <= 1e-12 * np.abs(phi).sum()
    # a value placed on one cell moves only that cell's radius
    m = oracle.radius_index(nx, ny, nz)
    bump = phi.copy()
    bump[3, 4, 5] += 1.0
    avg2, _ = oracle.average_irregular(bump)
    changed = np.nonzero(avg2 != avg)[0]
    assert list(changed) == [m[3, 4, 5]]
    assert avg2[m[3, 4, 5]] - avg[m[3, 4, 5]] == pytest.approx(1.0 / cnt[m[3, 4, 5]], rel=1e-12)


@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 10, 6)])
def test_fill_by_radius_index_and_average_round_trip(shape):
    """The irregular fill needs no interpolation: filling a table and averaging
    it back returns the table on every radius a cell reaches."""
    nx, ny, nz = shape
    h = 1.0 / nz
    nm = oracle.radius_count(nx, ny, nz)
    tab = 1.0 + np.cos(0.37 * np.arange(nm))
    g = oracle.Grid(nx, ny, nz, h, (1, 1, 1))
    cells = oracle.fill_beta0(g, 2, tab, 0.0, (0.5, 0.5, 0.5))
    m = oracle.radius_index(nx, ny, nz)
    assert np.array_equal(cells, tab[m])
    avg, cnt = oracle.average_irregular(cells)
    assert np.allclose(avg[cnt > 0], tab[cnt > 0], rtol=1e-14, atol=0)
    with pytest.raises(ValueError):
        oracle.fill_beta0(g, 2, tab[:-1], 0.0, (0.5, 0.5, 0.5))


def test_quadratic_fill_reproduces_quadratic_profiles_and_holds_ends():
    n, h = 16, 1.0 / 16
    dr = h / 5
    n1d = W.spherical_n1d(n)
    rj = (np.arange(n1d) + 0.5) * dr
    g = oracle.Grid(n, n, n, h, (1, 1, 1))
    r = radii_over_h(n, n, n) * h
    q = lambda s: 0.7 - 2.0 * s + 5.0 * s**2  # noqa: E731
    b = oracle.fill_beta0(g, 3, q(rj), dr, (0.5, 0.5, 0.5))
    inside = (r / dr - 0.5 > 0) & (r / dr - 0.5 < n1d - 1)
    assert np.allclose(b[inside], q(r[inside]), rtol=1e-12, atol=0)
    # a linear table gives the linear fill
    lin = oracle.fill_beta0(g, 1, 2.0 + 3.0 * rj, dr, (0.5, 0.5, 0.5))
    qlin = oracle.fill_beta0(g, 3, 2.0 + 3.0 * rj, dr, (0.5, 0.5, 0.5))
    assert np.allclose(lin, qlin, rtol=1e-13, atol=0)
    # beyond the table the end values are held
    short = q(rj[:40])
    bs = oracle.fill_beta0(g, 3, short, dr, (0.5, 0.5, 0.5))
    far = r / dr - 0.5 >= 39
    assert np.all(bs[far] == short[-1])
