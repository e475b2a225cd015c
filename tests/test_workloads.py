"""The seeded input generators: determinism, layouts and the stated contrasts."""
import hashlib

import numpy as np
import pytest

from paper_1908_03634_amd import workloads as W


def _digest(p):
    h = hashlib.sha256()
    for a in (p.beta0_1d, p.rho, p.ux, p.uy, p.uz, p.S):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_same_seed_same_bytes():
    a = W.config_problem("c1")
    b = W.config_problem("c1")
    assert _digest(a) == _digest(b)
    c = W.config_problem("c1", seed_offset=1)
    assert _digest(a) != _digest(c)


@pytest.mark.parametrize("bc", [(0, 0, 1), (1, 1, 1), (0, 0, 0)])
def test_face_layout_and_walls(bc):
    p = W.planar_problem(8, nx=6, ny=5, bc=bc, seed=1)
    sx, sy, sz = W.face_shapes(6, 5, 8, bc)
    assert p.ux.shape == sx and p.uy.shape == sy and p.uz.shape == sz
    if bc[0]:
        assert not p.ux[:, :, 0].any() and not p.ux[:, :, -1].any()
    if bc[2]:
        assert not p.uz[0].any() and not p.uz[-1].any()
    assert p.rho.shape == (8, 5, 6) and (p.rho > 0).all()


def test_planar_contrast_and_seed_convention():
    p = W.config_problem("c1")
    assert p.meta["seed"] == 20190806
    H = p.meta["H"]
    assert np.exp(-1.0 / H) == pytest.approx(1e-2, rel=1e-12)
    assert p.bc == (0, 0, 1) and p.nx == 32


def test_spherical_contrast_to_box_face():
    p = W.spherical_problem(16, seed=2)
    R = p.meta["R"]
    assert (1 + (0.5 / R) ** 2) ** -2.5 == pytest.approx(1e-5, rel=1e-12)
    assert len(p.beta0_1d) == W.spherical_n1d(16)
    # the radial table reaches beyond the box corner
    assert (len(p.beta0_1d) - 1) * p.dr > np.sqrt(3) * 0.5


def test_noise_statistics():
    p = W.planar_problem(32, seed=5)
    assert abs(p.S.std() - 1e-2) < 1e-3
    assert abs(p.ux.std() - 1.0) < 0.05
