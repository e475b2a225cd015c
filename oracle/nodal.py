"""FP64 CPU oracle for the nodal projection (Sec. 3.2 Step 11, Appendix A).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module; the product path never
does, and shares no code with it.

The arithmetic lives in `nodal_oracle.c` (plain C, FP64, OpenMP over z
planes): trilinear finite elements on the cells for the node-based phi, the
divergence of a cell-centred velocity at the nodes, the cell-average gradient
of phi, and a multigrid solve of the node system.  See the C file's header for
the discretisation and the reading of the paper it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nodal_oracle.c")
_LIB = os.path.join(_HERE, "libnodal_oracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int
_F = ctypes.c_double
_GRID = [_I, _I, _I, _F, _I, _I, _I]


def build(force=True):
    """Compile the nodal oracle with gcc (FP64, -O2, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _declare(lib):
    lib.nd_apply.argtypes = _GRID + [_D, _D, _D]
    lib.nd_divergence.argtypes = _GRID + [_D, _D, _D, _D]
    lib.nd_gradient.argtypes = _GRID + [_D, _D, _D, _D]
    lib.nd_load.argtypes = _GRID + [_D, _D]
    lib.nd_rhs.argtypes = _GRID + [_D, _D, _D, _D, _D, _D]
    lib.nd_rhs.restype = _F
    lib.nd_correct.argtypes = _GRID + [_D, _D, _D, _D, _D, _D]
    lib.nd_prolong_add.argtypes = _GRID + [_D, _D]
    lib.nd_restrict.argtypes = _GRID + [_D, _D]
    lib.nd_sigma_coarsen.argtypes = [_I, _I, _I, _D, _D]
    lib.nd_solve.argtypes = _GRID + [_D, _D, _D, _F, _I, _I, _I, ctypes.POINTER(_I), _D]
    lib.nd_solve.restype = _I
    lib.nd_node_dot.argtypes = [_I, _I, _I, _I, _I, _I, _D, _D]
    lib.nd_node_dot.restype = _F
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
    """Route every wrapper here through another build of the source (the
    mutation tests compile planted mistakes into copies of it)."""

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


def source_text():
    with open(_SRC) as f:
        return f.read()


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous, "oracle arrays must be C-contiguous float64"
    return a.ctypes.data_as(_D)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def node_shape(g):
    """Node array shape (nz+bz, ny+by, nx+bx) of a cell grid g (oracle.Grid)."""
    bx, by, bz = g.bc
    return (g.nz + bz, g.ny + by, g.nx + bx)


def nodes(g):
    return np.zeros(node_shape(g))


def apply(g, sigma, phi):
    """M phi: the finite-element form of div(sigma grad phi) at the nodes."""
    out = nodes(g)
    _load().nd_apply(*g.args(), _p(_c(sigma)), _p(_c(phi)), _p(out))
    return out


def divergence(g, vx, vy, vz):
    """Nodal divergence of a cell-centred vector field."""
    out = nodes(g)
    _load().nd_divergence(*g.args(), _p(_c(vx)), _p(_c(vy)), _p(_c(vz)), _p(out))
    return out


def gradient(g, phi):
    """Cell average of grad phi_h on every cell: (gx, gy, gz)."""
    gx, gy, gz = g.cells(), g.cells(), g.cells()
    _load().nd_gradient(*g.args(), _p(_c(phi)), _p(gx), _p(gy), _p(gz))
    return gx, gy, gz


def load(g, f):
    """Finite-element load of a cell-constant source at the nodes."""
    out = nodes(g)
    _load().nd_load(*g.args(), _p(_c(f)), _p(out))
    return out


def rhs(g, beta0, ux, uy, uz, S):
    """R = D(beta0 U) - L(beta0 S - m), m the cell mean of beta0 S.  Returns (R, m)."""
    out = nodes(g)
    m = _load().nd_rhs(*g.args(), _p(_c(beta0)), _p(_c(ux)), _p(_c(uy)), _p(_c(uz)), _p(_c(S)), _p(out))
    return out, m


def correct(g, sigma, beta0, phi, ux, uy, uz):
    """U - (sigma / beta0) G phi on every cell.  Returns copies."""
    ux, uy, uz = (np.array(a, dtype=np.float64, order="C") for a in (ux, uy, uz))
    _load().nd_correct(*g.args(), _p(_c(sigma)), _p(_c(beta0)), _p(_c(phi)), _p(ux), _p(uy), _p(uz))
    return ux, uy, uz


def prolong_add(g, ec, phi):
    """phi + P ec, P trilinear interpolation from the grid coarsened by 2."""
    out = np.array(phi, dtype=np.float64, order="C")
    _load().nd_prolong_add(*g.args(), _p(_c(ec)), _p(out))
    return out


def restrict(g, rf):
    """(1/8) P^T rf on the grid coarsened by 2."""
    bx, by, bz = g.bc
    out = np.zeros((g.nz // 2 + bz, g.ny // 2 + by, g.nx // 2 + bx))
    _load().nd_restrict(*g.args(), _p(_c(rf)), _p(out))
    return out


def sigma_coarsen(sigma):
    nz, ny, nx = sigma.shape
    out = np.zeros((nz // 2, ny // 2, nx // 2))
    _load().nd_sigma_coarsen(nx, ny, nz, _p(_c(sigma)), _p(out))
    return out


def node_dot(g, a, b):
    return float(_load().nd_node_dot(g.nx, g.ny, g.nz, *g.bc, _p(_c(a)), _p(_c(b))))


def solve(g, sigma, R, tol=1e-12, maxcycles=200, nu1=2, nu2=2, phi0=None):
    """phi with M phi = R - mean(R) and zero node mean, to ||r|| / ||R|| <= tol."""
    phi = nodes(g) if phi0 is None else np.array(phi0, dtype=np.float64, order="C")
    cyc = _I(0)
    rel = _F(0.0)
    st = _load().nd_solve(*g.args(), _p(_c(sigma)), _p(_c(R)), _p(phi), float(tol), int(maxcycles), int(nu1),
                          int(nu2), ctypes.byref(cyc), ctypes.byref(rel))
    if st == 2:
        raise ValueError("the nodal solve needs at least 2 cells per axis")
    return phi, dict(converged=(st == 0), cycles=cyc.value, rel_resid=rel.value)


def residual_norm(g, sigma, R, phi):
    """||R - M phi||_2 / ||R||_2 over the nodes, in FP64."""
    r = np.ascontiguousarray(R - apply(g, sigma, phi))
    return float(np.sqrt(node_dot(g, r, r) / node_dot(g, R, R)))


def project(prob, tol=1e-12, maxcycles=200):
    """Nodal projection of a workloads.NodalProblem (cell-centred ux, uy, uz):
    map beta0 by the fill of Sec. 3.1, sigma = beta0 / rho, right-hand side,
    solve, correction.  Returns a dict of every intermediate."""
    import oracle

    g = oracle.Grid.of(prob)
    beta0 = oracle.fill_beta0(g, prob.geometry, prob.beta0_1d, prob.dr, prob.center)
    sigma = beta0 / prob.rho
    R, m = rhs(g, beta0, prob.ux, prob.uy, prob.uz, prob.S)
    phi, info = solve(g, sigma, R, tol=tol, maxcycles=maxcycles)
    ux, uy, uz = correct(g, sigma, beta0, phi, prob.ux, prob.uy, prob.uz)
    return dict(grid=g, beta0=beta0, sigma=sigma, R=R, mean=m, phi=phi, info=info, ux=ux, uy=uy, uz=uz)


def update_pi(phi, s, pi=None, a=0.0):
    """Perturbational pressure from the nodal scalar (Sec. 3.2 Step 11; Appendix A
    says the gradient of that scalar updates pi): pi <- a pi + s phi on every
    node, s the caller's time-step scaling.  With a = 0, (sigma/beta0) G(pi)/s
    is the correction `correct` applies."""
    phi = np.asarray(phi, dtype=np.float64)
    if pi is None:
        return s * phi
    return a * np.asarray(pi, dtype=np.float64) + s * phi
