"""FP64 CPU oracle for the MAC-projection solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path (the
HIP library and its Python binding) never does, and shares no code with it.

The arithmetic lives in `mproj_oracle.c` (plain C, FP64, OpenMP over z planes);
the nodal projection of Sec. 3.2 Step 11 is in `nodal_oracle.c` / `nodal.py`;
this module builds it with gcc and wraps it for numpy arrays.  Each wrapper
names the passage of the paper it follows; see the C file's header for the
discretisation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mproj_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile the oracle (and the nodal-projection oracle) with gcc (FP64, -O2, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    from . import nodal

    nodal.build(force=force)
    return _LIB


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int
_F = ctypes.c_double
_GRID = [_I, _I, _I, _F, _I, _I, _I]


def _declare(lib):
    lib.or_cell_radius.argtypes = _GRID + [_D, _D]
    lib.or_fill_beta0.argtypes = _GRID + [_I, _D, _I, _F, _D, _D]
    lib.or_fill_beta0.restype = _I
    lib.or_face_coefs.argtypes = _GRID + [_D, _D, _D, _D, _D]
    lib.or_gradient.argtypes = _GRID + [_D, _D, _D, _D]
    lib.or_divergence.argtypes = _GRID + [_D, _D, _D, _D]
    lib.or_apply.argtypes = _GRID + [_D, _D, _D, _D, _D]
    lib.or_beta0_divergence.argtypes = _GRID + [_D, _D, _D, _D, _D]
    lib.or_mac_rhs.argtypes = _GRID + [_D, _D, _D, _D, _D, _D]
    lib.or_mac_rhs.restype = _F
    lib.or_velocity_correct.argtypes = _GRID + [_D, _D, _D, _D, _D, _D, _D, _D]
    lib.or_coef_grad.argtypes = _GRID + [_D, _D, _D, _D, _D]
    lib.or_solve.argtypes = _GRID + [_D, _D, _D, _D, _D, _F, _I, _I, _I, ctypes.POINTER(_I), _D]
    lib.or_solve.restype = _I
    lib.or_sum.argtypes = [_I, _I, _I, _D]
    lib.or_sum.restype = _F
    lib.or_dot.argtypes = [_I, _I, _I, _D, _D]
    lib.or_dot.restype = _F
    lib.or_num_threads.restype = _I
    lib.or_plane_average.argtypes = [_I, _I, _I, _D, _D]
    lib.or_split_source.argtypes = [_I, _I, _I, _I, _D, _D, _D]
    lib.or_split_source.restype = _I
    lib.or_average_uniform.argtypes = [_I, _I, _I, _F, _D, _I, _F, _D]
    lib.or_average_uniform.restype = _I
    lib.or_split_source_uniform.argtypes = [_I, _I, _I, _F, _I, _I, _F, _D, _D, _D]
    lib.or_split_source_uniform.restype = _I
    lib.or_add_w0.argtypes = _GRID + [_I, _D, _D, ctypes.c_long, _D, _D, _D, _D]
    lib.or_add_w0.restype = _I
    lib.or_radius_count.argtypes = [_I, _I, _I]
    lib.or_radius_count.restype = ctypes.c_long
    lib.or_radius_index.argtypes = [_I, _I, _I, ctypes.POINTER(ctypes.c_long)]
    lib.or_radius_index.restype = _I
    lib.or_average_irregular.argtypes = [_I, _I, _I, _D, ctypes.c_long, _D, _D]
    lib.or_average_irregular.restype = _I
    lib.or_irregular_radii.argtypes = [ctypes.c_long, _F, _D, _D]
    lib.or_irregular_radii.restype = None
    lib.or_enforce_hse.argtypes = [ctypes.c_long, _D, _D, _D, _F, _F, _D]
    lib.or_enforce_hse.restype = ctypes.c_long
    lib.or_beta0_from_p0.argtypes = [ctypes.c_long, _F, _D, _D, _D]
    lib.or_beta0_from_p0.restype = None
    lib.or_w0.argtypes = [_I, ctypes.c_long, _D, _D, _D, _D, _D, _D]
    lib.or_w0.restype = _I
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


class use_library:
    """Context manager that routes every wrapper in this module through another
    build of the oracle source (the mutation tests compile planted mistakes
    into copies of it)."""

    def __init__(self, path):
        self.lib = _declare(ctypes.CDLL(path))

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = self.lib
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def compile_variant(src_text, out_path):
    """Compile a (modified) copy of the oracle source to `out_path`."""
    c_path = out_path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", out_path, c_path, "-lm"])
    return out_path


def source_text():
    with open(_SRC) as f:
        return f.read()


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous, "oracle arrays must be C-contiguous float64"
    return a.ctypes.data_as(_D)


class Grid:
    """Uniform cell-centred grid: nx, ny, nz cells of spacing h; bc per axis
    (0 periodic, 1 Neumann wall)."""

    def __init__(self, nx, ny, nz, h, bc):
        self.nx, self.ny, self.nz, self.h = int(nx), int(ny), int(nz), float(h)
        self.bc = tuple(int(b) for b in bc)

    @classmethod
    def of(cls, prob):
        return cls(prob.nx, prob.ny, prob.nz, prob.h, prob.bc)

    def args(self):
        return [self.nx, self.ny, self.nz, self.h, *self.bc]

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def face_shapes(self):
        bx, by, bz = self.bc
        n = (self.nz, self.ny, self.nx)
        return (n[0], n[1], n[2] + bx), (n[0], n[1] + by, n[2]), (n[0] + bz, n[1], n[2])

    def cells(self):
        return np.zeros(self.shape)

    def faces(self):
        return tuple(np.zeros(s) for s in self.face_shapes())


def num_threads():
    return _load().or_num_threads()


def cell_radius(g, center):
    """Distance of each cell centre from `center` (radius used by fill, Sec. 3.1)."""
    r = g.cells()
    c = np.ascontiguousarray(center, dtype=np.float64)
    _load().or_cell_radius(*g.args(), _p(c), _p(r))
    return r


def fill_beta0(g, geometry, beta0_1d, dr, center):
    """Fill module of Sec. 3.1: direct injection (planar, table per z cell),
    interpolation in r on (j+1/2) dr (spherical: 1 linear, 3 quadratic), or
    lookup by the radius index m (2, irregular base state; centre at the
    middle node of the box)."""
    out = g.cells()
    b = np.ascontiguousarray(beta0_1d, dtype=np.float64)
    c = np.ascontiguousarray(center, dtype=np.float64)
    st = _load().or_fill_beta0(*g.args(), int(geometry), _p(b), len(b), float(dr), _p(c), _p(out))
    if st:
        raise ValueError("bad base-state table for this geometry")
    return out


def radius_count(nx, ny, nz):
    """Number of radii h sqrt(0.75 + 2m) of the irregular base state (0 when an
    extent is odd)."""
    return int(_load().or_radius_count(nx, ny, nz))


def radius_index(nx, ny, nz):
    """Radius index m of every cell (cell layout, int64)."""
    out = np.zeros((nz, ny, nx), dtype=np.int64)
    st = _load().or_radius_index(nx, ny, nz, out.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
    if st:
        raise ValueError("the irregular base state needs even extents")
    return out


def average_irregular(phi):
    """Lateral average over the irregular radii (Sec. 3.1): (avg, count) per m."""
    nz, ny, nx = phi.shape
    nm = radius_count(nx, ny, nz)
    a = np.ascontiguousarray(phi, dtype=np.float64)
    avg = np.zeros(nm)
    cnt = np.zeros(nm)
    st = _load().or_average_irregular(nx, ny, nz, _p(a), nm, _p(avg), _p(cnt))
    if st:
        raise ValueError("the irregular base state needs even extents")
    return avg, cnt


def plane_average(phi):
    """Lateral average of a planar atmosphere: mean of each horizontal plane."""
    nz, ny, nx = phi.shape
    a = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros(nz)
    _load().or_plane_average(nx, ny, nz, _p(a), _p(out))
    return out


def average_uniform(phi, h, n1d, dr):
    """Lateral average onto the uniform base state r_j = (j + 1/2) dr (Sec. 3.1):
    the averages over the irregular radii, quadratically interpolated (the
    three reached radii around the nearest one; end values held)."""
    nz, ny, nx = phi.shape
    a = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros(int(n1d))
    if _load().or_average_uniform(nx, ny, nz, float(h), _p(a), int(n1d), float(dr), _p(out)):
        raise ValueError("the uniform Average needs even extents and dr > 0")
    return out


def split_source(geometry, S, h=None, n1d=None, dr=None):
    """(S - Sbar on the cells, Sbar): the source of the velocity-split
    constraint div(beta0 U~) = beta0 (S - Sbar) of Appendix A, Sbar the
    lateral average: per plane (geometry 0), per irregular radius (2), or on
    the uniform table of n1d entries at spacing dr filled back linearly (1) or
    quadratically (3) (h the cell size; the star centred on the middle node)."""
    nz, ny, nx = S.shape
    a = np.ascontiguousarray(S, dtype=np.float64)
    out = np.zeros_like(a)
    if geometry in (1, 3):
        sbar = np.zeros(int(n1d))
        if _load().or_split_source_uniform(nx, ny, nz, float(h), int(geometry), int(n1d), float(dr), _p(a), _p(out),
                                           _p(sbar)):
            raise ValueError("the uniform split source needs even extents and dr > 0")
        return out, sbar
    sbar = np.zeros(nz if geometry == 0 else max(radius_count(nx, ny, nz), 1))
    if _load().or_split_source(nx, ny, nz, int(geometry), _p(a), _p(out), _p(sbar)):
        raise ValueError("the split source needs a planar or spherical base state")
    return out, sbar


def add_w0(g, geometry, w0_edges, re, center, ux, uy, uz):
    """U = U~ + w0 e_r on the faces (Appendix A): planar (geometry 0) adds
    w0[k] to the interior z faces; spherical adds w0(r_f) e_r . n_f on every
    non-wall face, w0 linear between the edges re.  Returns copies."""
    ux, uy, uz = (np.array(a, dtype=np.float64, order="C") for a in (ux, uy, uz))
    w = np.ascontiguousarray(w0_edges, dtype=np.float64)
    e = np.ascontiguousarray(re if re is not None else np.zeros(len(w)), dtype=np.float64)
    c = np.ascontiguousarray(center if center is not None else (0.0, 0.0, 0.0), dtype=np.float64)
    if _load().or_add_w0(*g.args(), int(geometry), _p(w), _p(e), len(w), _p(c), _p(ux), _p(uy), _p(uz)):
        raise ValueError("w0 on faces: planar needs Neumann z and nz + 1 edge values")
    return ux, uy, uz


def irregular_radii(nm, h):
    """(centres, edges) of the irregular base state: h sqrt(0.75 + 2m) and
    h sqrt(2m - 0.25) (edge 0 at the centre of the star)."""
    rc, re = np.zeros(nm), np.zeros(nm + 1)
    _load().or_irregular_radii(int(nm), float(h), _p(rc), _p(re))
    return rc, re


def enforce_hse(rc, rho0, g_edge, p0_base, rho_cutoff=0.0):
    """Enforce HSE (Sec. 3.2): p0 from rho0, trapezoidal across the centres
    rc, held constant from the cutoff density outward.  Returns (p0, cutoff index)."""
    rc, rho0, g_edge = (np.ascontiguousarray(a, dtype=np.float64) for a in (rc, rho0, g_edge))
    n = len(rc)
    assert len(rho0) == n and len(g_edge) == n + 1
    p0 = np.zeros(n)
    jc = _load().or_enforce_hse(n, _p(rc), _p(rho0), _p(g_edge), float(p0_base), float(rho_cutoff), _p(p0))
    return p0, int(jc)


def beta0_from_p0(rho0_centre, p0, gamma1):
    """beta0 = rho0(0) exp(int dp0 / (Gamma1 p0)) (Sec. 2) on the base-state centres."""
    p0, gamma1 = (np.ascontiguousarray(a, dtype=np.float64) for a in (p0, gamma1))
    out = np.zeros(len(p0))
    _load().or_beta0_from_p0(len(p0), float(rho0_centre), _p(p0), _p(gamma1), _p(out))
    return out


def w0(geometry, rc, re, beta0, sbar, psi=None):
    """Base-state velocity w0 on the n + 1 edges re from div(beta0 w0 e_r) =
    beta0 (Sbar - psi) (Appendix A), centres rc; geometry 0 planar, 1 spherical."""
    rc, re, beta0, sbar = (np.ascontiguousarray(a, dtype=np.float64) for a in (rc, re, beta0, sbar))
    n = len(beta0)
    assert len(rc) == n and len(re) == n + 1 and len(sbar) == n
    ps = None if psi is None else np.ascontiguousarray(psi, dtype=np.float64)
    out = np.zeros(n + 1)
    if _load().or_w0(int(geometry), n, _p(rc), _p(re), _p(beta0), _p(sbar), _p(ps) if ps is not None else None,
                     _p(out)):
        raise ValueError("w0 needs geometry 0 (planar) or 1 (spherical)")
    return out


def face_coefs(g, beta0_cc, rho):
    """beta0/rho at faces: harmonic mean of the two cells; walls 0 (momentum
    equation of Sec. 2 carries beta0/rho in front of the pressure gradient)."""
    cx, cy, cz = g.faces()
    _load().or_face_coefs(*g.args(), _p(beta0_cc), _p(rho), _p(cx), _p(cy), _p(cz))
    return cx, cy, cz


def map_base_state(g, geometry, beta0_1d, dr, center, rho):
    """beta0 on cells and the three face-coefficient arrays."""
    b = fill_beta0(g, geometry, beta0_1d, dr, center)
    return b, face_coefs(g, b, rho)


def gradient(g, phi):
    gx, gy, gz = g.faces()
    _load().or_gradient(*g.args(), _p(phi), _p(gx), _p(gy), _p(gz))
    return gx, gy, gz


def divergence(g, fx, fy, fz):
    out = g.cells()
    _load().or_divergence(*g.args(), _p(fx), _p(fy), _p(fz), _p(out))
    return out


def apply(g, cx, cy, cz, phi):
    """M phi = D(C G phi)."""
    out = g.cells()
    _load().or_apply(*g.args(), _p(cx), _p(cy), _p(cz), _p(phi), _p(out))
    return out


def beta0_divergence(g, beta0_cc, ux, uy, uz):
    """D(beta0_f U) with beta0_f the mean of the two cells."""
    out = g.cells()
    _load().or_beta0_divergence(*g.args(), _p(beta0_cc), _p(ux), _p(uy), _p(uz), _p(out))
    return out


def mac_rhs(g, beta0_cc, ux, uy, uz, S):
    """rhs = D(beta0 U) - beta0 S made mean-zero (constraints div1/div2 of
    Sec. 3.2 with the dp0/dt term folded into S).  Returns (rhs, removed mean)."""
    out = g.cells()
    m = _load().or_mac_rhs(*g.args(), _p(beta0_cc), _p(ux), _p(uy), _p(uz), _p(S), _p(out))
    return out, m


def solve(g, cx, cy, cz, rhs, tol=1e-12, maxcycles=200, nu1=2, nu2=2, phi0=None):
    """Mean-zero phi with M phi = rhs - mean(rhs), to ||r||/||rhs|| <= tol."""
    phi = g.cells() if phi0 is None else np.array(phi0, dtype=np.float64, order="C")
    cyc = _I(0)
    rel = _F(0.0)
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    st = _load().or_solve(*g.args(), _p(cx), _p(cy), _p(cz), _p(rhs), _p(phi), float(tol), int(maxcycles),
                          int(nu1), int(nu2), ctypes.byref(cyc), ctypes.byref(rel))
    return phi, dict(converged=(st == 0), cycles=cyc.value, rel_resid=rel.value)


def velocity_correct(g, cx, cy, cz, beta0_cc, phi, ux, uy, uz):
    """U - (c_f/beta0_f) G phi (Appendix A: remove the gradient part).  Returns copies."""
    ux, uy, uz = (np.array(a, dtype=np.float64, order="C") for a in (ux, uy, uz))
    _load().or_velocity_correct(*g.args(), _p(cx), _p(cy), _p(cz), _p(beta0_cc), _p(phi), _p(ux), _p(uy), _p(uz))
    return ux, uy, uz


def coef_grad(g, lam, phi):
    """(G lam)_f (G phi)_f: gradient of <w, phi> with respect to c_f when lam
    solves M lam = w - mean(w)."""
    gx, gy, gz = g.faces()
    _load().or_coef_grad(*g.args(), _p(lam), _p(phi), _p(gx), _p(gy), _p(gz))
    return gx, gy, gz


def residual_norm(g, cx, cy, cz, rhs, phi):
    """||rhs - M phi||_2 / ||rhs||_2 in FP64 (rhs taken as given)."""
    r = rhs - apply(g, cx, cy, cz, phi)
    lib = _load()
    r = np.ascontiguousarray(r)
    rhs = np.ascontiguousarray(rhs)
    return float(np.sqrt(lib.or_dot(g.nx, g.ny, g.nz, _p(r), _p(r)) / lib.or_dot(g.nx, g.ny, g.nz, _p(rhs), _p(rhs))))


def mac_project(prob, tol=1e-12, maxcycles=200, split=False):
    """Whole projection on a workloads.Problem: map, rhs, solve, correct.
    split: project onto div(beta0 U~) = beta0 (S - Sbar) (Appendix A) instead
    of div(beta0 U) = beta0 S.  Returns a dict of every intermediate."""
    g = Grid.of(prob)
    beta0_cc, (cx, cy, cz) = map_base_state(g, prob.geometry, prob.beta0_1d, prob.dr, prob.center, prob.rho)
    S = prob.S
    sbar = None
    if split:
        S, sbar = split_source(prob.geometry, prob.S, h=prob.h, n1d=len(prob.beta0_1d), dr=prob.dr)
    rhs, m = mac_rhs(g, beta0_cc, prob.ux, prob.uy, prob.uz, S)
    phi, info = solve(g, cx, cy, cz, rhs, tol=tol, maxcycles=maxcycles)
    ux, uy, uz = velocity_correct(g, cx, cy, cz, beta0_cc, phi, prob.ux, prob.uy, prob.uz)
    return dict(grid=g, beta0_cc=beta0_cc, cx=cx, cy=cy, cz=cz, rhs=rhs, mean=m, phi=phi, info=info,
                ux=ux, uy=uy, uz=uz, S_eff=S, sbar=sbar)
