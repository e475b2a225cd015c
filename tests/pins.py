"""Independent constructions that pin the oracle (and, through it, the GPU path).

None of this reuses the oracle's code.  The operator is assembled here as a
sparse product of incidence matrices (M = D C G built from the face/cell
connectivity, with D = -G^T checked separately), and the solution is obtained
with library routines the oracle does not use: sparse LU on a bordered system,
FFT x tridiagonal elimination for coefficients that vary only in z, and
FFT/DCT diagonalisation for a constant coefficient.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _axis_faces(n, b):
    """(face index, left cell, right cell, has_two_sides) along one axis."""
    nf = n + b
    f = np.arange(nf)
    if b:
        L = f - 1
        R = f.copy()
        two = (f > 0) & (f < n)
        L = np.where(two, L, 0)
        R = np.where(two, R, 0)
    else:
        L = (f - 1) % n
        R = f % n
        two = np.ones(nf, bool)
    return f, L, R, two


def incidence(nx, ny, nz, h, bc):
    """Sparse G (faces x cells) for the x, y, z face arrays stacked in that
    order (each in C order of its own [z][y][x] shape).  Rows of wall faces are
    empty."""
    bx, by, bz = bc
    cid = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    off = 0
    # x faces, shape (nz, ny, nx + bx)
    f, L, R, two = _axis_faces(nx, bx)
    K, J, F = np.meshgrid(np.arange(nz), np.arange(ny), f, indexing="ij")
    fid = off + np.arange(K.size).reshape(K.shape)
    m = two[F]
    rows += [fid[m], fid[m]]
    cols += [cid[K[m], J[m], R[F[m]]], cid[K[m], J[m], L[F[m]]]]
    vals += [np.full(m.sum(), 1.0 / h), np.full(m.sum(), -1.0 / h)]
    off += K.size
    # y faces, shape (nz, ny + by, nx)
    f, L, R, two = _axis_faces(ny, by)
    K, F, I = np.meshgrid(np.arange(nz), f, np.arange(nx), indexing="ij")
    fid = off + np.arange(K.size).reshape(K.shape)
    m = two[F]
    rows += [fid[m], fid[m]]
    cols += [cid[K[m], R[F[m]], I[m]], cid[K[m], L[F[m]], I[m]]]
    vals += [np.full(m.sum(), 1.0 / h), np.full(m.sum(), -1.0 / h)]
    off += K.size
    # z faces, shape (nz + bz, ny, nx)
    f, L, R, two = _axis_faces(nz, bz)
    F, J, I = np.meshgrid(f, np.arange(ny), np.arange(nx), indexing="ij")
    fid = off + np.arange(F.size).reshape(F.shape)
    m = two[F]
    rows += [fid[m], fid[m]]
    cols += [cid[R[F[m]], J[m], I[m]], cid[L[F[m]], J[m], I[m]]]
    vals += [np.full(m.sum(), 1.0 / h), np.full(m.sum(), -1.0 / h)]
    off += F.size
    G = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(off, nx * ny * nz)).tocsr()
    return G


def divergence_matrix(nx, ny, nz, h, bc):
    """Sparse D (cells x faces) built from each cell's own low and high faces
    (wall faces contribute nothing)."""
    bx, by, bz = bc
    n = nx * ny * nz
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cell = (K * ny + J) * nx + I
    rows, cols, vals = [], [], []
    sizes = [nz * ny * (nx + bx), nz * (ny + by) * nx, (nz + bz) * ny * nx]
    offs = [0, sizes[0], sizes[0] + sizes[1]]

    def add(fid, sign, keep):
        rows.append(cell[keep].ravel())
        cols.append(fid[keep].ravel())
        vals.append(np.full(int(keep.sum()), sign / h))

    # x
    lo = I
    hi = I + 1 if bx else (I + 1) % nx
    fid_lo = offs[0] + (K * ny + J) * (nx + bx) + lo
    fid_hi = offs[0] + (K * ny + J) * (nx + bx) + hi
    add(fid_hi, +1.0, ~((hi == nx) & (bx == 1)))
    add(fid_lo, -1.0, ~((lo == 0) & (bx == 1)))
    # y
    lo = J
    hi = J + 1 if by else (J + 1) % ny
    fid_lo = offs[1] + (K * (ny + by) + lo) * nx + I
    fid_hi = offs[1] + (K * (ny + by) + hi) * nx + I
    add(fid_hi, +1.0, ~((hi == ny) & (by == 1)))
    add(fid_lo, -1.0, ~((lo == 0) & (by == 1)))
    # z
    lo = K
    hi = K + 1 if bz else (K + 1) % nz
    fid_lo = offs[2] + (lo * ny + J) * nx + I
    fid_hi = offs[2] + (hi * ny + J) * nx + I
    add(fid_hi, +1.0, ~((hi == nz) & (bz == 1)))
    add(fid_lo, -1.0, ~((lo == 0) & (bz == 1)))
    D = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, sum(sizes))).tocsr()
    return D


def operator(nx, ny, nz, h, bc, cx, cy, cz):
    """M = D C G as a sparse matrix."""
    G = incidence(nx, ny, nz, h, bc)
    D = divergence_matrix(nx, ny, nz, h, bc)
    c = np.concatenate([cx.ravel(), cy.ravel(), cz.ravel()])
    return (D @ sp.diags(c) @ G).tocsr()


def bordered_solve(M, rhs):
    """Mean-zero phi with M phi = rhs - mean(rhs) by sparse LU of
    [[M, 1], [1^T, 0]]."""
    n = M.shape[0]
    one = sp.csr_matrix(np.ones((n, 1)))
    B = sp.bmat([[M, one], [one.T, None]], format="csc")
    b = np.concatenate([rhs.ravel() - rhs.mean(), [0.0]])
    x = spla.spsolve(B, b)
    return x[:n]


def fft_tridiag_solve(nx, ny, nz, h, c_cell_z, c_face_z, rhs):
    """Exact solve of M phi = rhs for periodic x/y, Neumann z, with x and y
    face coefficients equal to c_cell_z[k] on plane k and z face coefficients
    c_face_z[f] (f = 0..nz, walls 0).  Fourier in x/y makes M tridiagonal in z:
        (1/h^2)[c_{k+1/2}(p_{k+1}-p_k) - c_{k-1/2}(p_k-p_{k-1})] - c_k lam p_k = r_k
    with lam = (4/h^2)(sin^2(pi kx/nx) + sin^2(pi ky/ny)).  The (0,0) mode is
    singular and is solved with a border row fixing its mean to zero."""
    rh = sfft.rfftn(rhs, axes=(1, 2))  # (nz, ny, nx//2+1)
    kx = np.arange(nx // 2 + 1)
    ky = np.arange(ny)
    lam = (4.0 / h ** 2) * (np.sin(np.pi * ky / ny)[:, None] ** 2 + np.sin(np.pi * kx / nx)[None, :] ** 2)
    cf = np.asarray(c_face_z, dtype=np.float64)
    cc = np.asarray(c_cell_z, dtype=np.float64)
    lower = cf[:-1][1:] / h ** 2  # coefficient of p_{k-1} for k = 1..nz-1
    upper = cf[1:][:-1] / h ** 2  # coefficient of p_{k+1} for k = 0..nz-2
    diag0 = -(cf[:-1] + cf[1:]) / h ** 2  # (nz,)
    # Thomas elimination over z for every (ky, kx) at once.
    d = diag0[:, None, None] - cc[:, None, None] * lam[None, :, :]
    d = d.astype(np.complex128)
    r = rh.copy()
    d[:, 0, 0] = 1.0  # placeholder; (0,0) is handled separately below
    cp = np.zeros_like(d)
    for k in range(nz):
        a = lower[k - 1] if k > 0 else 0.0
        if k > 0:
            denom = d[k] - a * cp[k - 1]
            r[k] = (r[k] - a * r[k - 1]) / denom
            cp[k] = (upper[k] / denom) if k < nz - 1 else 0.0
        else:
            r[k] = r[k] / d[k]
            cp[k] = upper[k] / d[k] if nz > 1 else 0.0
    for k in range(nz - 2, -1, -1):
        r[k] = r[k] - cp[k] * r[k + 1]
    # (0,0) mode: singular 1D Neumann problem with a border.
    A = np.diag(diag0) + np.diag(upper, 1) + np.diag(lower, -1)
    Bm = np.zeros((nz + 1, nz + 1))
    Bm[:nz, :nz] = A
    Bm[:nz, nz] = 1.0
    Bm[nz, :nz] = 1.0
    b00 = np.concatenate([rh[:, 0, 0].real, [0.0]])
    r[:, 0, 0] = np.linalg.solve(Bm, b00)[:nz]
    phi = sfft.irfftn(r, s=(ny, nx), axes=(1, 2))
    return phi - phi.mean()


def const_coef_solve(nx, ny, nz, h, bc, rhs):
    """Exact solve of M phi = rhs for c = 1 everywhere (walls 0) by
    diagonalisation: Fourier along periodic axes (eigenvalue
    (4/h^2) sin^2(pi k/n)) and DCT-II along Neumann axes (eigenvalue
    (4/h^2) sin^2(pi k/(2n)))."""
    shape = (nz, ny, nx)
    a = rhs - rhs.mean()
    lam = np.zeros(shape)
    out = a.astype(np.complex128)
    # forward transforms axis by axis (array axes 0=z, 1=y, 2=x)
    bcs = {2: bc[0], 1: bc[1], 0: bc[2]}
    for ax in (0, 1, 2):
        n = shape[ax]
        k = np.arange(n)
        if bcs[ax] == 1:
            out = sfft.dct(out.real, type=2, axis=ax, norm="ortho") + 1j * sfft.dct(out.imag, type=2, axis=ax,
                                                                                        norm="ortho")
            ev = (4.0 / h ** 2) * np.sin(np.pi * k / (2 * n)) ** 2
        else:
            out = sfft.fft(out, axis=ax)
            ev = (4.0 / h ** 2) * np.sin(np.pi * k / n) ** 2
        s = [1, 1, 1]
        s[ax] = n
        lam = lam + ev.reshape(s)
    lam[0, 0, 0] = 1.0
    out = -out / lam
    out[0, 0, 0] = 0.0
    for ax in (0, 1, 2):
        if bcs[ax] == 1:
            out = sfft.idct(out.real, type=2, axis=ax, norm="ortho") + 1j * sfft.idct(out.imag, type=2, axis=ax,
                                                                                          norm="ortho")
        else:
            out = sfft.ifft(out, axis=ax)
    phi = out.real
    return phi - phi.mean()
