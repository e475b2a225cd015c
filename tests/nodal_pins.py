"""Independent finite-element reference for the nodal-projection pins.

The oracle forms its element integrals from closed-form 1D integrals.  Here
the same definitions (trilinear hat functions on the cells, Sec. 3.2 Step 11
read as a finite-element projection) are evaluated another way: the basis
functions and their gradients are evaluated pointwise and integrated by
2-point Gauss quadrature per axis (exact for these polynomials), the
interpolation operator comes from evaluating the coarse hat functions at the
fine node positions, and everything is assembled into scipy sparse matrices.
"""
import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

GAUSS = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))


def _hat(a, t):
    return 1.0 - t if a == 0 else t


def _dhat(a):
    return -1.0 if a == 0 else 1.0


def corners():
    return [(A & 1, (A >> 1) & 1, (A >> 2) & 1) for A in range(8)]


def element_integrals(h):
    """(K, Gi, Ni) on a cube of side h: K[A, B] = int grad N_A . grad N_B,
    Gi[A, d] = int dN_A/dx_d, Ni[A] = int N_A, by Gauss quadrature."""
    K = np.zeros((8, 8))
    Gi = np.zeros((8, 3))
    Ni = np.zeros(8)
    w = h**3 / 8.0
    cs = corners()
    for t in itertools.product(GAUSS, GAUSS, GAUSS):  # (tx, ty, tz)
        N = np.array([_hat(c[0], t[0]) * _hat(c[1], t[1]) * _hat(c[2], t[2]) for c in cs])
        dN = np.array([[_dhat(c[0]) / h * _hat(c[1], t[1]) * _hat(c[2], t[2]),
                        _hat(c[0], t[0]) * _dhat(c[1]) / h * _hat(c[2], t[2]),
                        _hat(c[0], t[0]) * _hat(c[1], t[1]) * _dhat(c[2]) / h] for c in cs])
        K += w * dN @ dN.T
        Gi += w * dN
        Ni += w * N
    return K, Gi, Ni


def node_shape(nx, ny, nz, bc):
    return (nz + bc[2], ny + bc[1], nx + bc[0])


def cell_nodes(nx, ny, nz, bc):
    """(ncell, 8) flat node index of each cell corner (corner bits x, y, z)."""
    mz, my, mx = node_shape(nx, ny, nz, bc)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((nx * ny * nz, 8), dtype=np.int64)
    for A, (a, b, c) in enumerate(corners()):
        ii = (i + a) % mx
        jj = (j + b) % my
        kk = (k + c) % mz
        out[:, A] = ((kk * my + jj) * mx + ii).ravel()
    return out


def operator(nx, ny, nz, h, bc, sigma):
    """M = -(1/h^3) sum_e sigma_e K_e assembled over the nodes (sparse)."""
    K, _, _ = element_integrals(h)
    cn = cell_nodes(nx, ny, nz, bc)
    s = np.asarray(sigma).ravel()
    rows = np.repeat(cn, 8, axis=1).ravel()
    cols = np.tile(cn, (1, 8)).ravel()
    vals = (s[:, None] * K.ravel()[None, :]).ravel() * (-1.0 / h**3)
    n = int(np.prod(node_shape(nx, ny, nz, bc)))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def divergence(nx, ny, nz, h, bc):
    """D: 3 cell arrays (x, y, z stacked) -> nodes, (DV)_n = -(1/h^3) sum_e V_e . int grad N_n."""
    _, Gi, _ = element_integrals(h)
    cn = cell_nodes(nx, ny, nz, bc)
    nc = nx * ny * nz
    n = int(np.prod(node_shape(nx, ny, nz, bc)))
    rows, cols, vals = [], [], []
    for d in range(3):
        for A in range(8):
            rows.append(cn[:, A])
            cols.append(d * nc + np.arange(nc))
            vals.append(np.full(nc, -Gi[A, d] / h**3))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, 3 * nc))


def gradient(nx, ny, nz, h, bc):
    """G: nodes -> 3 cell arrays stacked, the cell average of grad phi_h."""
    _, Gi, _ = element_integrals(h)
    cn = cell_nodes(nx, ny, nz, bc)
    nc = nx * ny * nz
    n = int(np.prod(node_shape(nx, ny, nz, bc)))
    rows, cols, vals = [], [], []
    for d in range(3):
        for A in range(8):
            rows.append(d * nc + np.arange(nc))
            cols.append(cn[:, A])
            vals.append(np.full(nc, Gi[A, d] / h**3))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * nc, n))


def load(nx, ny, nz, h, bc):
    """L: cells -> nodes, (1/h^3) sum_e f_e int N_n."""
    _, _, Ni = element_integrals(h)
    cn = cell_nodes(nx, ny, nz, bc)
    nc = nx * ny * nz
    n = int(np.prod(node_shape(nx, ny, nz, bc)))
    rows = cn.T.ravel()
    cols = np.tile(np.arange(nc), 8)
    vals = np.repeat(Ni / h**3, nc)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def interpolation(nx, ny, nz, bc):
    """P: coarse nodes (grid coarsened by 2) -> fine nodes, the coarse hat
    functions evaluated at the fine node positions (unit fine spacing)."""
    fz, fy, fx = node_shape(nx, ny, nz, bc)
    cz, cy, cx = node_shape(nx // 2, ny // 2, nz // 2, bc)

    def axis(nf_nodes, nc_nodes, ncell, b):
        W = np.zeros((nf_nodes, nc_nodes))
        for i in range(nf_nodes):
            for I in range(nc_nodes):
                d = abs(i - 2 * I)
                if not b:
                    d = min(d, ncell - d)
                W[i, I] = max(0.0, 1.0 - d / 2.0)
        return W

    Wx = axis(fx, cx, nx, bc[0])
    Wy = axis(fy, cy, ny, bc[1])
    Wz = axis(fz, cz, nz, bc[2])
    return sp.csr_matrix(np.kron(Wz, np.kron(Wy, Wx)))


def solve_gauged(M, R):
    """phi with M phi = R - mean(R), mean(phi) = 0, by a sparse LU of the
    bordered system [M 1; 1^T 0]."""
    n = M.shape[0]
    one = np.ones((n, 1))
    B = sp.bmat([[M, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]], format="csc")
    rhs = np.concatenate([R - R.mean(), [0.0]])
    return spla.spsolve(B, rhs)[:n]
