"""Python binding of libmproj (the C ABI in include/mproj.h).

Argument marshalling only: tensors are checked (device, dtype, shape,
contiguity) and their device pointers handed to the library, which runs every
step on the GPU.  There is no CPU fallback; a missing library raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmproj.so")

MP_OK = 0
STATUS = {
    0: "MP_OK",
    1: "MP_ERR_ARG",
    2: "MP_ERR_DEVICE",
    3: "MP_ERR_NOMEM",
    4: "MP_ERR_NOT_CONVERGED",
    5: "MP_ERR_NONFINITE",
    6: "MP_ERR_SINGULAR_RHS",
    7: "MP_ERR_STATE",
}
MP_ERR_NOT_CONVERGED = 4
PERIODIC, NEUMANN = 0, 1
PLANAR, SPHERICAL, SPHERICAL_IRREGULAR, SPHERICAL_QUADRATIC = 0, 1, 2, 3
FP64, MIXED = 0, 1


class MprojError(RuntimeError):
    def __init__(self, code, msg, info=None):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.msg = msg
        self.info = info


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("h", ctypes.c_double),
        ("bc", ctypes.c_int * 3),
        ("precision", ctypes.c_int),
        ("rtol", ctypes.c_double),
        ("max_outer", ctypes.c_int),
        ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
        ("cycles_per_outer", ctypes.c_int),
        ("bottom_rtol", ctypes.c_double),
        ("bottom_max_iter", ctypes.c_int),
        ("demean", ctypes.c_int),
        ("kernel_timing", ctypes.c_int),
        ("smoother", ctypes.c_int),
        ("coarse_cycle", ctypes.c_int),
        ("blocked", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("device", ctypes.c_int),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_int),
        ("vcycles", ctypes.c_int),
        ("bottom_iters_total", ctypes.c_int),
        ("levels", ctypes.c_int),
        ("rel_resid", ctypes.c_double),
        ("div_defect", ctypes.c_double),
        ("rhs_norm", ctypes.c_double),
        ("rhs_mean", ctypes.c_double),
        ("resid_hist", ctypes.c_double * 64),
        ("ms_setup", ctypes.c_double),
        ("ms_rhs", ctypes.c_double), ("ms_solve", ctypes.c_double), ("ms_correct", ctypes.c_double),
        ("smooth_ms_total", ctypes.c_double),
        ("smooth_launches", ctypes.c_int),
        ("smooth_bytes", ctypes.c_double),
        ("smooth_form", ctypes.c_int),
        ("flags", ctypes.c_int),
    ]

    def as_dict(self):
        n = min(max(self.outer_iters + 1, 0), 64)
        return dict(outer_iters=self.outer_iters, vcycles=self.vcycles, levels=self.levels,
                    bottom_iters_total=self.bottom_iters_total, ms_setup=self.ms_setup,
                    rel_resid=self.rel_resid, div_defect=self.div_defect, rhs_norm=self.rhs_norm,
                    rhs_mean=self.rhs_mean, resid_hist=list(self.resid_hist[:n]), ms_rhs=self.ms_rhs,
                    ms_solve=self.ms_solve, ms_correct=self.ms_correct, smooth_ms_total=self.smooth_ms_total,
                    smooth_launches=self.smooth_launches, smooth_bytes=self.smooth_bytes,
                    smooth_form=self.smooth_form, flags=self.flags)


# Every exported symbol of include/mproj.h.
EXPORTS = ["mp_config_default", "mp_init", "mp_map_base_state", "mp_set_coefs", "mp_mac_project", "mp_solve",
           "mp_mac_project_split", "mp_radius_count", "mp_average", "mp_set_kernel_timing", "mp_apply", "mp_coef_grad",
           "mp_nodal_shape", "mp_nodal_project", "mp_nodal_apply", "mp_nodal_pi", "mp_base_radii", "mp_enforce_hse",
           "mp_beta0_from_p0", "mp_w0", "mp_enforce_hse_noalloc", "mp_average_uniform", "mp_add_w0", "mp_free",
           "mp_last_error", "mp_version"]

_lib = None


def load_library(path=None):
    """Load libmproj.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libmproj.so not found at {p}: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    lib.mp_config_default.argtypes = [ctypes.POINTER(Config), I, I, I]
    lib.mp_config_default.restype = None
    lib.mp_init.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(P)]
    lib.mp_init.restype = I
    lib.mp_map_base_state.argtypes = [P, I, P, I, D, ctypes.POINTER(D), P, P, P, P]
    lib.mp_map_base_state.restype = I
    lib.mp_set_coefs.argtypes = [P, P, P, P]
    lib.mp_set_coefs.restype = I
    lib.mp_mac_project.argtypes = [P, P, P, P, P, P, I, ctypes.POINTER(Info)]
    lib.mp_mac_project.restype = I
    lib.mp_solve.argtypes = [P, P, P, I, ctypes.POINTER(Info)]
    lib.mp_solve.restype = I
    lib.mp_mac_project_split.argtypes = [P, P, P, P, P, P, I, P, ctypes.POINTER(Info)]
    lib.mp_mac_project_split.restype = I
    lib.mp_radius_count.argtypes = [P, ctypes.POINTER(ctypes.c_longlong)]
    lib.mp_radius_count.restype = I
    lib.mp_average.argtypes = [P, P, P, P]
    lib.mp_average.restype = I
    lib.mp_average_uniform.argtypes = [P, P, I, D, P]
    lib.mp_average_uniform.restype = I
    lib.mp_add_w0.argtypes = [P, P, P, ctypes.c_longlong, P, P, P]
    lib.mp_add_w0.restype = I
    lib.mp_set_kernel_timing.argtypes = [P, I]
    lib.mp_set_kernel_timing.restype = I
    lib.mp_apply.argtypes = [P, P, P]
    lib.mp_apply.restype = I
    lib.mp_coef_grad.argtypes = [P, P, P, P, P, P]
    lib.mp_coef_grad.restype = I
    lib.mp_nodal_shape.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.mp_nodal_shape.restype = I
    lib.mp_nodal_project.argtypes = [P, P, P, P, P, P, I, ctypes.POINTER(Info)]
    lib.mp_nodal_project.restype = I
    lib.mp_nodal_apply.argtypes = [P, P, P]
    lib.mp_nodal_apply.restype = I
    lib.mp_nodal_pi.argtypes = [P, P, D, D, P]
    lib.mp_nodal_pi.restype = I
    L = ctypes.c_longlong
    lib.mp_base_radii.argtypes = [P, P, P]
    lib.mp_base_radii.restype = I
    lib.mp_enforce_hse.argtypes = [P, L, P, P, P, D, D, P, ctypes.POINTER(L)]
    lib.mp_enforce_hse.restype = I
    lib.mp_enforce_hse_noalloc.argtypes = [P, L, P, P, P, D, D, P, P]
    lib.mp_enforce_hse_noalloc.restype = I
    lib.mp_beta0_from_p0.argtypes = [P, L, D, P, P, P]
    lib.mp_beta0_from_p0.restype = I
    lib.mp_w0.argtypes = [P, I, L, P, P, P, P, P, P]
    lib.mp_w0.restype = I
    lib.mp_free.argtypes = [P]
    lib.mp_free.restype = I
    lib.mp_last_error.argtypes = [P]
    lib.mp_last_error.restype = ctypes.c_char_p
    lib.mp_version.argtypes = []
    lib.mp_version.restype = ctypes.c_char_p
    if path is None:
        _lib = lib
    return lib


def face_shapes(nx, ny, nz, bc):
    bx, by, bz = bc
    return (nz, ny, nx + bx), (nz, ny + by, nx), (nz + bz, ny, nx)


class Context:
    """One solver context: grid, boundary kinds, precision and the multigrid
    hierarchy on one device and stream."""

    def __init__(self, nx, ny, nz, h=None, bc=(PERIODIC, PERIODIC, NEUMANN), precision="mixed", rtol=1e-10,
                 max_outer=100, nu1=2, nu2=2, cycles_per_outer=0, bottom_rtol=1e-8, bottom_max_iter=400,
                 demean=True, kernel_timing=False, smoother="auto", coarse_cycle=True, blocked=True, device=None, stream=None):
        self.lib = load_library()
        self._args = []
        self.coef_generation = 0  # bumped whenever the library's coefficients change
        if not torch.cuda.is_available():
            raise MprojError(2, "no GPU visible to torch")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        cfg = Config()
        self.lib.mp_config_default(ctypes.byref(cfg), nx, ny, nz)
        cfg.h = float(h) if h is not None else 1.0 / nz
        for a in range(3):
            cfg.bc[a] = int(bc[a])
        cfg.precision = {"mixed": MIXED, "fp64": FP64}[precision]
        cfg.rtol = rtol
        cfg.max_outer = max_outer
        cfg.nu1, cfg.nu2 = nu1, nu2
        cfg.cycles_per_outer = cycles_per_outer
        cfg.bottom_rtol = bottom_rtol
        cfg.bottom_max_iter = bottom_max_iter
        cfg.demean = 1 if demean else 0
        cfg.kernel_timing = 1 if kernel_timing else 0
        cfg.smoother = {"auto": 0, "per_colour": 1, "fused": 2}[smoother]
        cfg.coarse_cycle = 1 if coarse_cycle else 0
        cfg.blocked = 1 if blocked else 0
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = st
        cfg.stream = ctypes.c_void_p(st.cuda_stream)
        cfg.device = self.device.index
        self.cfg = cfg
        self.nx, self.ny, self.nz, self.h, self.bc = nx, ny, nz, cfg.h, tuple(int(b) for b in bc)
        self.precision = precision
        handle = ctypes.c_void_p()
        code = self.lib.mp_init(ctypes.byref(cfg), ctypes.byref(handle))
        if code != MP_OK:
            raise MprojError(code, "mp_init failed")
        self._h = handle

    # -- helpers ---------------------------------------------------------
    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def face_shapes(self):
        return face_shapes(self.nx, self.ny, self.nz, self.bc)

    def _ptr(self, t, shape, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        self._args.append(t)
        return ctypes.c_void_p(t.data_ptr())

    def _run(self, fn, *args):
        """Call the library on this context with the tensors marshalled since
        the last call, in stream order with the caller's current stream: when
        that is not the context's stream, the context's stream first waits
        for the work queued on the caller's (which produced the inputs), the
        caller's stream then waits for the context's (so that it sees the
        outputs), and each tensor is recorded as used on the context's stream
        (the caching allocator does not hand its memory out again before
        that work ends)."""
        ts, self._args = self._args, []
        cur = torch.cuda.current_stream(self.device)
        cross = cur.cuda_stream != self.stream.cuda_stream
        if cross:
            self.stream.wait_stream(cur)
            for t in ts:
                t.record_stream(self.stream)
        try:
            return fn(self._h, *args)
        finally:
            if cross:
                cur.wait_stream(self.stream)

    def _check(self, code, what, info=None):
        if code != MP_OK:
            msg = self.lib.mp_last_error(self._h).decode()
            raise MprojError(code, f"{what}: {msg}", info)

    def empty_cells(self):
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    def empty_faces(self):
        return tuple(torch.empty(s, dtype=torch.float64, device=self.device) for s in self.face_shapes())

    # -- API -------------------------------------------------------------
    def map_base_state(self, geometry, beta0_1d, rho, dr=0.0, center=None, out=None, want_coefs=True):
        """Fill beta0 (planar injection; spherical linear or quadratic
        interpolation; irregular spherical base state indexed by radius) and
        build the face coefficients; returns (cx, cy, cz) or None."""
        n1d = int(beta0_1d.shape[0])
        tab = self._ptr(beta0_1d, (n1d,), "beta0_1d")
        rp = self._ptr(rho, self.shape, "rho")
        faces = None
        if want_coefs:
            faces = out if out is not None else self.empty_faces()
            ptrs = [self._ptr(f, s, "coef") for f, s in zip(faces, self.face_shapes())]
        else:
            ptrs = [None, None, None]
        c = (ctypes.c_double * 3)(*(center if center is not None else (0.0, 0.0, 0.0)))
        code = self._run(self.lib.mp_map_base_state, int(geometry), tab, n1d, float(dr), c, rp, *ptrs)
        self.coef_generation += 1
        self._check(code, "mp_map_base_state")
        return faces

    def set_coefs(self, cx, cy, cz):
        ps = [self._ptr(f, s, n) for f, s, n in zip((cx, cy, cz), self.face_shapes(), ("cx", "cy", "cz"))]
        code = self._run(self.lib.mp_set_coefs, *ps)
        self.coef_generation += 1
        self._check(code, "mp_set_coefs")

    def mac_project(self, ux, uy, uz, S, phi=None, use_initial_guess=False, allow_not_converged=False,
                    split=False, sbar=None):
        """Project (ux, uy, uz) in place; returns (phi, info dict).  split:
        velocity-split constraint div(beta0 U~) = beta0 (S - Sbar), Sbar (the
        lateral average of S) written to `sbar` when given."""
        sx, sy, sz = self.face_shapes()
        pu = [self._ptr(ux, sx, "ux"), self._ptr(uy, sy, "uy"), self._ptr(uz, sz, "uz")]
        ps = self._ptr(S, self.shape, "S")
        if phi is None:
            phi = self.empty_cells()
            use_initial_guess = False
        pp = self._ptr(phi, self.shape, "phi")
        info = Info()
        if split:
            pb = self._ptr(sbar, None, "sbar") if sbar is not None else None
            code = self._run(self.lib.mp_mac_project_split, *pu, ps, pp, int(bool(use_initial_guess)), pb,
                                                 ctypes.byref(info))
        else:
            code = self._run(self.lib.mp_mac_project, *pu, ps, pp, int(bool(use_initial_guess)), ctypes.byref(info))
        d = info.as_dict()
        if not (allow_not_converged and code == MP_ERR_NOT_CONVERGED):
            self._check(code, "mp_mac_project_split" if split else "mp_mac_project", d)
        d["status"] = code
        return phi, d

    def solve(self, rhs, x=None, use_initial_guess=False, allow_not_converged=False):
        """Mean-zero x with div(c grad x) = rhs (mean of rhs removed)."""
        pr = self._ptr(rhs, self.shape, "rhs")
        if x is None:
            x = self.empty_cells()
            use_initial_guess = False
        px = self._ptr(x, self.shape, "x")
        info = Info()
        code = self._run(self.lib.mp_solve, pr, px, int(bool(use_initial_guess)), ctypes.byref(info))
        d = info.as_dict()
        if not (allow_not_converged and code == MP_ERR_NOT_CONVERGED):
            self._check(code, "mp_solve", d)
        d["status"] = code
        return x, d

    def radius_count(self):
        """Number of radii h sqrt(0.75 + 2m) of the irregular base state."""
        nm = ctypes.c_longlong()
        self._check(self.lib.mp_radius_count(self._h, ctypes.byref(nm)), "mp_radius_count")
        return int(nm.value)

    def average(self, phi, out=None, count=True):
        """Lateral average of a cell field over the irregular radii:
        returns (avg, count) (count None when not asked for)."""
        nm = self.radius_count()
        pp = self._ptr(phi, self.shape, "phi")
        avg = out if out is not None else torch.empty(nm, dtype=torch.float64, device=self.device)
        cnt = torch.empty(nm, dtype=torch.float64, device=self.device) if count else None
        pa = self._ptr(avg, (nm,), "avg")
        pc = self._ptr(cnt, (nm,), "count") if count else None
        self._check(self._run(self.lib.mp_average, pp, pa, pc), "mp_average")
        return avg, cnt

    def average_uniform(self, phi, n1d, dr, out=None):
        """Lateral average onto the uniform base state r_j = (j + 1/2) dr
        (radius averages interpolated quadratically)."""
        avg = out if out is not None else torch.empty(int(n1d), dtype=torch.float64, device=self.device)
        self._check(self._run(self.lib.mp_average_uniform, self._ptr(phi, self.shape, "phi"), int(n1d), float(dr),
                              self._ptr(avg, (int(n1d),), "avg")), "mp_average_uniform")
        return avg

    def add_w0(self, w0, ux, uy, uz, re=None):
        """U += w0 e_r on the faces (in place): planar, w0 on the nz + 1 z
        edges; spherical, w0 on the edges re (linear between them)."""
        ne = int(w0.shape[0])
        sx, sy, sz = self.face_shapes()
        pr = self._ptr(re, (ne,), "re") if re is not None else None
        code = self._run(self.lib.mp_add_w0, self._ptr(w0, (ne,), "w0"), pr, ne, self._ptr(ux, sx, "ux"),
                         self._ptr(uy, sy, "uy"), self._ptr(uz, sz, "uz"))
        self._check(code, "mp_add_w0")
        return ux, uy, uz

    def set_kernel_timing(self, on):
        """Time the finest-level smoother launches of the following calls."""
        self._check(self.lib.mp_set_kernel_timing(self._h, 1 if on else 0), "mp_set_kernel_timing")

    def apply(self, x, out=None):
        """M x = div(c grad x) with the FP64 finest-level coefficients."""
        y = out if out is not None else self.empty_cells()
        self._check(self._run(self.lib.mp_apply, self._ptr(x, self.shape, "x"), self._ptr(y, self.shape, "y")),
                    "mp_apply")
        return y

    def coef_grad(self, lam, phi, out=None):
        """(G lam)(G phi) on every face (walls 0)."""
        g = out if out is not None else self.empty_faces()
        ps = [self._ptr(f, s, "g") for f, s in zip(g, self.face_shapes())]
        self._check(self._run(self.lib.mp_coef_grad, self._ptr(lam, self.shape, "lam"),
                                          self._ptr(phi, self.shape, "phi"), *ps), "mp_coef_grad")
        return g

    # -- nodal projection (Sec. 3.2 Step 11) -------------------------------
    @property
    def node_shape(self):
        """Node array shape (z, y, x): n per periodic axis, n + 1 per Neumann axis."""
        mx, my, mz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.mp_nodal_shape(self._h, ctypes.byref(mx), ctypes.byref(my), ctypes.byref(mz)),
                    "mp_nodal_shape")
        return (mz.value, my.value, mx.value)

    def empty_nodes(self):
        return torch.empty(self.node_shape, dtype=torch.float64, device=self.device)

    def nodal_project(self, ux, uy, uz, S, phi=None, use_initial_guess=False, allow_not_converged=False):
        """Nodal projection of the cell-centred velocity (ux, uy, uz), in
        place, with phi on the nodes; returns (phi, info dict)."""
        pu = [self._ptr(u, self.shape, n) for u, n in ((ux, "ux"), (uy, "uy"), (uz, "uz"))]
        ps = self._ptr(S, self.shape, "S")
        if phi is None:
            phi = self.empty_nodes()
            use_initial_guess = False
        pp = self._ptr(phi, self.node_shape, "phi")
        info = Info()
        code = self._run(self.lib.mp_nodal_project, *pu, ps, pp, int(bool(use_initial_guess)), ctypes.byref(info))
        d = info.as_dict()
        if not (allow_not_converged and code == MP_ERR_NOT_CONVERGED):
            self._check(code, "mp_nodal_project", d)
        d["status"] = code
        return phi, d

    def nodal_apply(self, x, out=None):
        """M x on the nodes (finite-element div(sigma grad x)), FP64."""
        y = out if out is not None else self.empty_nodes()
        ns = self.node_shape
        self._check(self._run(self.lib.mp_nodal_apply, self._ptr(x, ns, "x"), self._ptr(y, ns, "y")), "mp_nodal_apply")
        return y

    def nodal_pi(self, phi, s, pi=None, a=0.0):
        """pi <- a pi + s phi on the nodes (the perturbational pressure from
        the nodal projection's scalar; a = 0 writes a new pi)."""
        ns = self.node_shape
        if pi is None:
            pi = self.empty_nodes()
            a = 0.0
        self._check(self._run(self.lib.mp_nodal_pi, self._ptr(phi, ns, "phi"), float(a), float(s), self._ptr(pi, ns, "pi")),
                    "mp_nodal_pi")
        return pi

    # -- one-dimensional base state ----------------------------------------
    def _vec(self, n):
        return torch.empty(n, dtype=torch.float64, device=self.device)

    def base_radii(self):
        """(centres, edges) of the irregular base state of this grid."""
        nm = self.radius_count()
        rc, re = self._vec(nm), self._vec(nm + 1)
        self._check(self._run(self.lib.mp_base_radii, self._ptr(rc, (nm,), "rc"), self._ptr(re, (nm + 1,), "re")),
                    "mp_base_radii")
        return rc, re

    def enforce_hse(self, rc, rho0, g_edge, p0_base, rho_cutoff=0.0, out=None):
        """Enforce HSE: returns (p0, cutoff index)."""
        n = int(rc.shape[0])
        p0 = out if out is not None else self._vec(n)
        jc = ctypes.c_longlong()
        code = self._run(self.lib.mp_enforce_hse, n, self._ptr(rc, (n,), "rc"), self._ptr(rho0, (n,), "rho0"),
                                       self._ptr(g_edge, (n + 1,), "g_edge"), float(p0_base), float(rho_cutoff),
                                       self._ptr(p0, (n,), "p0"), ctypes.byref(jc))
        self._check(code, "mp_enforce_hse")
        return p0, int(jc.value)

    def beta0_from_p0(self, rho0_centre, p0, gamma1, out=None):
        """beta0 = rho0(0) exp(int dp0 / (Gamma1 p0)) on the base state."""
        n = int(p0.shape[0])
        b = out if out is not None else self._vec(n)
        self._check(self._run(self.lib.mp_beta0_from_p0, n, float(rho0_centre), self._ptr(p0, (n,), "p0"),
                                              self._ptr(gamma1, (n,), "gamma1"), self._ptr(b, (n,), "beta0")),
                    "mp_beta0_from_p0")
        return b

    def w0(self, geometry, rc, re, beta0, sbar, psi=None, out=None):
        """Base-state velocity on the n + 1 edges (Appendix A)."""
        n = int(rc.shape[0])
        w = out if out is not None else self._vec(n + 1)
        pp = self._ptr(psi, (n,), "psi") if psi is not None else None
        self._check(self._run(self.lib.mp_w0, int(geometry), n, self._ptr(rc, (n,), "rc"),
                                   self._ptr(re, (n + 1,), "re"), self._ptr(beta0, (n,), "beta0"),
                                   self._ptr(sbar, (n,), "sbar"), pp, self._ptr(w, (n + 1,), "w0")), "mp_w0")
        return w

    def close(self):
        if getattr(self, "_h", None):
            self.lib.mp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False


def enforce_hse_noalloc(rc, rho0, g_edge, p0_base, rho_cutoff, p0, cutoff_index=None, stream=None):
    """mp_enforce_hse_noalloc: Enforce HSE without a context and without any
    device allocation (the library's static scratch); p0 (out) and
    cutoff_index (a one-element int64 tensor, out, or None) are device
    tensors on the current device.  Returns without waiting; runs on
    `stream` (default: torch's current stream)."""
    lib = load_library()
    n = int(rc.shape[0])
    dev = rc.device
    for t, shape, name in ((rc, (n,), "rc"), (rho0, (n,), "rho0"), (g_edge, (n + 1,), "g_edge"), (p0, (n,), "p0")):
        if t.device != dev or t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape {shape} on {dev}")
    if cutoff_index is not None and (cutoff_index.dtype != torch.int64 or cutoff_index.numel() != 1
                                     or cutoff_index.device != dev):
        raise ValueError("cutoff_index must be a one-element int64 tensor on the same device")
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    code = lib.mp_enforce_hse_noalloc(ctypes.c_void_p(st.cuda_stream), n, ctypes.c_void_p(rc.data_ptr()),
                                      ctypes.c_void_p(rho0.data_ptr()), ctypes.c_void_p(g_edge.data_ptr()),
                                      float(p0_base), float(rho_cutoff), ctypes.c_void_p(p0.data_ptr()),
                                      ctypes.c_void_p(cutoff_index.data_ptr()) if cutoff_index is not None else None)
    if code != MP_OK:
        raise MprojError(code, f"mp_enforce_hse_noalloc: {lib.mp_last_error(None).decode()}")
    return p0


def version():
    return load_library().mp_version().decode()
