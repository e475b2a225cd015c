// k_mg.hip -- gfx950 multigrid kernels launched one per operation: one colour
// of red-black Gauss-Seidel (the reference the fused sweep is checked
// against, and the fallback for odd periodic extents), residual + 8-cell
// restriction, piecewise-constant prolongation, the workgroup BiCGStab
// bottom solve for coarsest grids too large for one wavefront, and the FP64
// finest-level operator, residual and update of the iterative refinement.
//
// The stencils are bandwidth-bound (about 20 flops per 24-48 bytes), so no
// matrix cores are involved.  Launches are 3D (x fastest, 64 lanes along x)
// so no thread divides a 64-bit index; the FP64 residual marches along z
// keeping the z-neighbours of its column in registers.
#include "mp_device.h"
#include "mp_kernels.h"
#include "mp_launch.h"

#include <math.h>

namespace mp {

// ------------------------------------------------------------------ smoother

template <typename T, bool CELL>
__global__ __launch_bounds__(256) void k_rbgs(Dims d, T* __restrict__ x, const T* __restrict__ b, Coef<T> C, T h2,
                                              int colour, int zero_init)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (p >= (d.nx + 1) / 2 || j >= d.ny || k >= d.nz) return;
    rbgs_cell<T, CELL>(d, x, b, C, h2, colour, zero_init, p, j, k);
}

template <typename T>
void launch_rbgs(const Dims& d, T* phi, const T* rhs, const Coef<T>& c, T h2, int colour, int zero_init,
                 hipStream_t s)
{
    const Shape3 sh = cells3((d.nx + 1) / 2, d.ny, d.nz);
    if (c.cell)
        hipLaunchKernelGGL((k_rbgs<T, true>), sh.grid, sh.block, 0, s, d, phi, rhs, c, h2, colour, zero_init);
    else
        hipLaunchKernelGGL((k_rbgs<T, false>), sh.grid, sh.block, 0, s, d, phi, rhs, c, h2, colour, zero_init);
}

// The two colour passes that follow a prolongation, with the prolongation
// folded in (ec: coarse correction; piecewise constant, parent of (i,j,k) is
// (i/2, j/2, k/2)).  ALL (first colour): every value read, neighbours and
// own, is x + e of its parent, the values the separate prolongation would
// have stored; the other colour is left as stored.  Otherwise (second
// colour): the neighbours, just updated, are read as stored and the cell's
// own value as x + e.  Together they equal launch_prolong followed by two
// plain passes, bit for bit.
__device__ __forceinline__ long long parent_of(const Dims& d, int i, int j, int k)
{
    return ((long long)(k >> 1) * (d.ny >> 1) + (j >> 1)) * (d.nx >> 1) + (i >> 1);
}

template <typename T, bool CELL, bool ALL>
__global__ __launch_bounds__(256) void k_rbgs_e(Dims d, T* __restrict__ x, const T* __restrict__ b, Coef<T> C, T h2,
                                                int colour, const T* __restrict__ ec)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (p >= (d.nx + 1) / 2 || j >= d.ny || k >= d.nz) return;
    const int i = 2 * p + ((j + k + colour) & 1);
    if (i >= d.nx) return;
    const long long q = ((long long)k * d.ny + j) * d.nx + i;
    const Nbr nb = neighbours(d, q, i, j, k);
    T c0, c1, c2, c3, c4, c5;
    coef6<T, CELL>(C, d, q, nb, i, j, k, c0, c1, c2, c3, c4, c5);
    const T own = x[q] + ec[parent_of(d, i, j, k)];
    if constexpr (ALL) {
        // neighbour coordinates (a wall neighbour is the cell itself)
        const int im = i > 0 ? i - 1 : (d.px ? d.nx - 1 : i), ip = i < d.nx - 1 ? i + 1 : (d.px ? 0 : i);
        const int jm = j > 0 ? j - 1 : (d.py ? d.ny - 1 : j), jp = j < d.ny - 1 ? j + 1 : (d.py ? 0 : j);
        const int km = k > 0 ? k - 1 : (d.pz ? d.nz - 1 : k), kp = k < d.nz - 1 ? k + 1 : (d.pz ? 0 : k);
        const T xm = x[nb.xm] + ec[parent_of(d, im, j, k)], xp = x[nb.xp] + ec[parent_of(d, ip, j, k)];
        const T ym = x[nb.ym] + ec[parent_of(d, i, jm, k)], yp = x[nb.yp] + ec[parent_of(d, i, jp, k)];
        const T zm = x[nb.zm] + ec[parent_of(d, i, j, km)], zp = x[nb.zp] + ec[parent_of(d, i, j, kp)];
        x[q] = gs_value<T>(c0, c1, c2, c3, c4, c5, xm, xp, ym, yp, zm, zp, b[q], h2, own);
    } else {
        x[q] = gs_value<T>(c0, c1, c2, c3, c4, c5, x[nb.xm], x[nb.xp], x[nb.ym], x[nb.yp], x[nb.zm], x[nb.zp], b[q],
                           h2, own);
    }
}

template <typename T>
void launch_rbgs_e(const Dims& d, T* phi, const T* rhs, const Coef<T>& c, T h2, int colour, int first,
                   const T* ec, hipStream_t s)
{
    const Shape3 sh = cells3((d.nx + 1) / 2, d.ny, d.nz);
    if (c.cell) {
        if (first)
            hipLaunchKernelGGL((k_rbgs_e<T, true, true>), sh.grid, sh.block, 0, s, d, phi, rhs, c, h2, colour, ec);
        else
            hipLaunchKernelGGL((k_rbgs_e<T, true, false>), sh.grid, sh.block, 0, s, d, phi, rhs, c, h2, colour, ec);
    } else {
        if (first)
            hipLaunchKernelGGL((k_rbgs_e<T, false, true>), sh.grid, sh.block, 0, s, d, phi, rhs, c, h2, colour, ec);
        else
            hipLaunchKernelGGL((k_rbgs_e<T, false, false>), sh.grid, sh.block, 0, s, d, phi, rhs, c, h2, colour, ec);
    }
}

// Both colours of a sweep in one launch, out of place, for levels with stored
// faces and even extents, where a launch costs more than its cells: thread
// (p, j, k) owns cells 2p and 2p+1 of row j of plane k, one red and one black.
// It updates the red cell from old values and publishes it in LDS; after one
// barrier it updates the black cell from the new red values of its six
// neighbours, which are the red cells of the neighbouring threads (the pair
// p -/+ 1 along x, the same p on the rows and planes beside it): taken from
// LDS inside the workgroup, evaluated again from old values at its edges.  A
// red value depends on old values only, so the repeated evaluation gives the
// bits of the colour pass.  Old values (MODE): FS_ZERO 0 (first sweep from a
// zero iterate), FS_PLAIN x as stored, FS_PROLONG x + e of the parent cell
// (first sweep after prolongation).  Every cell takes the operands of
// rbgs_cell / k_rbgs_e: a black cell's neighbour behind a wall is its value as
// the colour pass finds it stored (x, without e).
template <typename T, int MODE>
struct RbPair {
    Dims d;
    const T* __restrict__ xo;
    const T* __restrict__ b;
    const T* __restrict__ cx;
    const T* __restrict__ cy;
    const T* __restrict__ cz;
    const T* __restrict__ ec;
    T h2;

    __device__ __forceinline__ int parent(int i, int j, int k) const
    {
        return ((k >> 1) * (d.ny >> 1) + (j >> 1)) * (d.nx >> 1) + (i >> 1);
    }
    __device__ __forceinline__ T old_at(int q, int i, int j, int k) const
    {
        if constexpr (MODE == FS_ZERO) return T(0);
        else if constexpr (MODE == FS_PLAIN) return xo[q];
        else return xo[q] + ec[parent(i, j, k)];
    }
    // face coefficients of cell q in stencil order (coef6, face mode)
    __device__ __forceinline__ void coefs(int q, const Nb32& nb, T (&c)[6]) const
    {
        const T xh = cx[nb.xp], yh = cy[nb.yp], zh = cz[nb.zp];
        c[0] = cx[q];
        c[1] = nb.hx ? xh : T(0);
        c[2] = cy[q];
        c[3] = nb.hy ? yh : T(0);
        c[4] = cz[q];
        c[5] = nb.hz ? zh : T(0);
    }
    // new value of red cell (i, j, k) (coordinates inside the grid)
    __device__ __forceinline__ T red(int i, int j, int k) const
    {
        const int q = (k * d.ny + j) * d.nx + i;
        const Nb32 nb = nb32(d, q, i, j, k);
        T c[6];
        coefs(q, nb, c);
        T v[6], own;
        if constexpr (MODE == FS_ZERO) {
            own = v[0] = v[1] = v[2] = v[3] = v[4] = v[5] = T(0);
        } else {
            // neighbour coordinates (a wall neighbour is the cell itself)
            const int im = i > 0 ? i - 1 : (d.px ? d.nx - 1 : i), ip = i < d.nx - 1 ? i + 1 : (d.px ? 0 : i);
            const int jm = j > 0 ? j - 1 : (d.py ? d.ny - 1 : j), jp = j < d.ny - 1 ? j + 1 : (d.py ? 0 : j);
            const int km = k > 0 ? k - 1 : (d.pz ? d.nz - 1 : k), kp = k < d.nz - 1 ? k + 1 : (d.pz ? 0 : k);
            own = old_at(q, i, j, k);
            v[0] = old_at(nb.xm, im, j, k);
            v[1] = old_at(nb.xp, ip, j, k);
            v[2] = old_at(nb.ym, i, jm, k);
            v[3] = old_at(nb.yp, i, jp, k);
            v[4] = old_at(nb.zm, i, j, km);
            v[5] = old_at(nb.zp, i, j, kp);
        }
        return gs_value<T>(c[0], c[1], c[2], c[3], c[4], c[5], v[0], v[1], v[2], v[3], v[4], v[5], b[q], h2, own);
    }
};

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_rb_pair(Dims d, const T* __restrict__ xo, T* __restrict__ xn,
                                                 const T* __restrict__ b, const T* __restrict__ cx,
                                                 const T* __restrict__ cy, const T* __restrict__ cz, T h2,
                                                 const T* __restrict__ ec)
{
    __shared__ T sred[256];
    const int bx = (int)blockDim.x, by = (int)blockDim.y, bz = (int)blockDim.z;
    const int p0 = (int)blockIdx.x * bx, j0 = (int)blockIdx.y * by, k0 = (int)blockIdx.z * bz;
    const int p = p0 + (int)threadIdx.x, j = j0 + (int)threadIdx.y, k = k0 + (int)threadIdx.z;
    const bool live = p < d.nx / 2 && j < d.ny && k < d.nz;
    const RbPair<T, MODE> s{d, xo, b, cx, cy, cz, ec, h2};
    const int par = (j + k) & 1;  // the red cell is 2p + par
    const int ir = 2 * p + par, ib = 2 * p + 1 - par;
    const T rv = live ? s.red(ir, j, k) : T(0);
    sred[((int)threadIdx.z * by + (int)threadIdx.y) * bx + (int)threadIdx.x] = rv;
    __syncthreads();
    if (!live) return;
    // the red cell of pair (pn, jn, kn): from LDS when that thread is in this
    // workgroup, else evaluated here
    auto red_of = [&](int pn, int jn, int kn) -> T {
        const int u = pn - p0, v = jn - j0, w = kn - k0;
        if (u >= 0 && u < bx && v >= 0 && v < by && w >= 0 && w < bz) return sred[(w * by + v) * bx + u];
        return s.red(2 * pn + ((jn + kn) & 1), jn, kn);
    };
    const int row = (k * d.ny + j) * d.nx;
    const int q = row + ib;
    const Nb32 nb = nb32(d, q, ib, j, k);
    // the black cell as the second colour pass finds it stored
    const T stored = MODE == FS_ZERO ? T(0) : xo[q];
    // one x neighbour is the pair's red cell; the other is the red cell of
    // the pair beside it (-1: behind a wall)
    const int np = d.nx / 2;
    const int po = par ? (p > 0 ? p - 1 : (d.px ? np - 1 : -1)) : (p < np - 1 ? p + 1 : (d.px ? 0 : -1));
    const int jm = j > 0 ? j - 1 : (d.py ? d.ny - 1 : -1), jp = j < d.ny - 1 ? j + 1 : (d.py ? 0 : -1);
    const int km = k > 0 ? k - 1 : (d.pz ? d.nz - 1 : -1), kp = k < d.nz - 1 ? k + 1 : (d.pz ? 0 : -1);
    const T vo = po >= 0 ? red_of(po, j, k) : stored;
    const T ym = jm >= 0 ? red_of(p, jm, k) : stored;
    const T yp = jp >= 0 ? red_of(p, jp, k) : stored;
    const T zm = km >= 0 ? red_of(p, j, km) : stored;
    const T zp = kp >= 0 ? red_of(p, j, kp) : stored;
    T c[6];
    s.coefs(q, nb, c);
    const T xm = par ? vo : rv, xp = par ? rv : vo;
    const T bv = gs_value<T>(c[0], c[1], c[2], c[3], c[4], c[5], xm, xp, ym, yp, zm, zp, b[q], h2,
                             s.old_at(q, ib, j, k));
    xn[row + ir] = rv;
    xn[q] = bv;
}

bool rb_pair_supported(const Dims& d)
{
    return d.nx % 2 == 0 && d.ny % 2 == 0 && d.nz % 2 == 0 && d.n() < (1LL << 31);
}

// Workgroup of whole rows of pairs (up to 64 pairs wide) by a few rows and
// planes, so that most red neighbours of a black cell lie inside it.
template <typename T>
void launch_rb_pair(const Dims& d, const T* xo, T* xn, const T* b, const Coef<T>& c, T h2, int mode, const T* ec,
                    hipStream_t s)
{
    const int np = d.nx / 2;
    const int bx = pow2_at_least(np, 64);
    const int rem = 256 / bx;
    const int bz = pow2_at_least(d.nz, rem >= 16 ? 4 : rem >= 4 ? 2 : 1);
    const int by = pow2_at_least(d.ny, rem / bz);
    const dim3 block(bx, by, bz);
    const dim3 grid((np + bx - 1) / bx, (d.ny + by - 1) / by, (d.nz + bz - 1) / bz);
    if (mode == FS_ZERO)
        hipLaunchKernelGGL((k_rb_pair<T, FS_ZERO>), grid, block, 0, s, d, xo, xn, b, c.x, c.y, c.z, h2, ec);
    else if (mode == FS_PROLONG)
        hipLaunchKernelGGL((k_rb_pair<T, FS_PROLONG>), grid, block, 0, s, d, xo, xn, b, c.x, c.y, c.z, h2, ec);
    else
        hipLaunchKernelGGL((k_rb_pair<T, FS_PLAIN>), grid, block, 0, s, d, xo, xn, b, c.x, c.y, c.z, h2, ec);
}

// --------------------------------------------------------- transfer operators

template <typename T, bool CELL>
__global__ __launch_bounds__(256) void k_resid_restrict(Dims d, const T* __restrict__ x, const T* __restrict__ b,
                                                        Coef<T> C, T inv_h2, T* __restrict__ bc)
{
    const int nxc = d.nx / 2, nyc = d.ny / 2, nzc = d.nz / 2;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= nxc || J >= nyc || K >= nzc) return;
    bc[((long long)K * nyc + J) * nxc + I] = restrict_cell<T, CELL>(d, x, b, C, inv_h2, I, J, K);
}

template <typename T>
void launch_resid_restrict(const Dims& fine, const T* phi, const T* rhs, const Coef<T>& c, T inv_h2, T* coarse_rhs,
                           hipStream_t s)
{
    const Shape3 sh = cells3(fine.nx / 2, fine.ny / 2, fine.nz / 2);
    if (c.cell)
        hipLaunchKernelGGL((k_resid_restrict<T, true>), sh.grid, sh.block, 0, s, fine, phi, rhs, c, inv_h2,
                           coarse_rhs);
    else
        hipLaunchKernelGGL((k_resid_restrict<T, false>), sh.grid, sh.block, 0, s, fine, phi, rhs, c, inv_h2,
                           coarse_rhs);
}

// Fine x += coarse e of the parent cell.
template <typename T>
__global__ __launch_bounds__(256) void k_prolong(Dims d, T* __restrict__ x, const T* __restrict__ e)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= d.nx || j >= d.ny || k >= d.nz) return;
    const int nxc = d.nx / 2, nyc = d.ny / 2;
    x[((long long)k * d.ny + j) * d.nx + i] += e[((long long)(k >> 1) * nyc + (j >> 1)) * nxc + (i >> 1)];
}

template <typename T>
void launch_prolong(const Dims& fine, T* phi, const T* coarse_phi, hipStream_t s)
{
    const Shape3 sh = cells3(fine.nx, fine.ny, fine.nz);
    hipLaunchKernelGGL((k_prolong<T>), sh.grid, sh.block, 0, s, fine, phi, coarse_phi);
}

// ------------------------------------------------------------ bottom solve

// Block minimum; every thread receives the same value (sh as for block_sum).
__device__ __forceinline__ double block_min(double v, double* sh)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double m = sh[0];
    for (int i = 1; i < nw; i++) m = fmin(m, sh[i]);
    return m;
}

// The six face coefficients of cell q (stencil order), FP64.
template <typename T>
__device__ __forceinline__ void face6(const T* cx, const T* cy, const T* cz, long long q, const Nbr& nb, double (&c)[6])
{
    c[0] = (double)cx[q];
    c[1] = (double)ld_or0(cx, nb.cxp);
    c[2] = (double)cy[q];
    c[3] = (double)ld_or0(cy, nb.cyp);
    c[4] = (double)cz[q];
    c[5] = (double)ld_or0(cz, nb.czp);
}

// BiCGStab in FP64 for A x = b on the coarsest grid, run by one workgroup
// (used when that grid holds more cells than one wavefront solves in
// registers).  The constants on each connected part of the grid (cells
// joined through nonzero faces) span the null space, so b is made mean-zero
// part by part first and the result is returned so (with every cell coupled:
// the plain mean removal, in the same operations).  With use_x0 the
// iteration starts from the x passed in and stops at rtol times the initial
// residual; otherwise it starts from zero.  An unconverged solve returns the
// iterate of the smallest residual.  work holds 9 n doubles.
template <typename T>
__global__ __launch_bounds__(1024) void k_bottom(Dims d, const T* __restrict__ bin, T* __restrict__ xout,
                                                 const T* __restrict__ cx, const T* __restrict__ cy,
                                                 const T* __restrict__ cz, double h2, double rtol, int maxit,
                                                 int use_x0, double* __restrict__ work, double* __restrict__ iters,
                                                 const double* __restrict__ skip_if_direct)
{
    __shared__ double sh[16];
    if (skip_if_direct && skip_if_direct[0] == 1.0) return;
    const int n = (int)d.n();
    const int tid = threadIdx.x, nt = blockDim.x;
    double* x = work;
    double* r = work + n;
    double* rh = work + 2 * n;
    double* p = work + 3 * n;
    double* v = work + 4 * n;
    double* s = work + 5 * n;
    double* tv = work + 6 * n;
    double* xb = work + 7 * n;
    double* lab = work + 8 * n;  // connected-part label: smallest cell index of the part
    const double inv_h2 = 1.0 / h2;

    // labels by minimum-label propagation (in place: the fixed point, each
    // part's smallest index, does not depend on the order of the updates)
    for (int q = tid; q < n; q += nt) lab[q] = (double)q;
    for (;;) {
        __syncthreads();
        double changed = 0.0;
        for (int q = tid; q < n; q += nt) {
            int i, j, k;
            cell_ijk(d, q, i, j, k);
            const Nbr nb = neighbours(d, q, i, j, k);
            double c[6];
            face6<T>(cx, cy, cz, q, nb, c);
            const long long nq[6] = {nb.xm, nb.xp, nb.ym, nb.yp, nb.zm, nb.zp};
            double m = lab[q];
#pragma unroll
            for (int f = 0; f < 6; f++)
                if (c[f] != 0.0) m = fmin(m, lab[nq[f]]);
            if (m < lab[q]) {
                lab[q] = m;
                changed = 1.0;
            }
        }
        if (block_sum(changed, sh) == 0.0) break;
    }
    // pm[q] = mean of y over the part of cell q (pm may not alias y)
    auto part_means = [&](const double* y, bool from_bin, double* pm) {
        double lo = (double)n;
        for (int q = tid; q < n; q += nt) lo = fmin(lo, lab[q]);
        double cur = block_min(lo, sh);
        while (cur < (double)n) {
            double sum = 0.0, cnt = 0.0, nxt = (double)n;
            for (int q = tid; q < n; q += nt) {
                if (lab[q] == cur) {
                    sum += from_bin ? (double)bin[q] : y[q];
                    cnt += 1.0;
                } else if (lab[q] > cur) {
                    nxt = fmin(nxt, lab[q]);
                }
            }
            const double m = block_sum(sum, sh) / block_sum(cnt, sh);
            for (int q = tid; q < n; q += nt)
                if (lab[q] == cur) pm[q] = m;
            cur = block_min(nxt, sh);
        }
        __syncthreads();
    };
    double part = 0.0;
    double* bmean = s;  // free until the iteration
    part_means(nullptr, true, bmean);
    for (int q = tid; q < n; q += nt) x[q] = use_x0 ? (double)xout[q] : 0.0;

    // A y for y in work (FP64), coefficients in T.
    auto apply = [&](const double* y, double* out) {
        __syncthreads();
        for (int q = tid; q < n; q += nt) {
            int i, j, k;
            cell_ijk(d, q, i, j, k);
            const Nbr nb = neighbours(d, q, i, j, k);
            double csum, cv;
            stencil_sums<double>(cx, cy, cz, y, q, nb, csum, cv);
            out[q] = (csum * y[q] - cv) * inv_h2;
        }
        __syncthreads();
    };

    if (use_x0) apply(x, tv);
    part = 0.0;
    for (int q = tid; q < n; q += nt) {
        const double rq = ((double)bin[q] - bmean[q]) - (use_x0 ? tv[q] : 0.0);
        r[q] = rq;
        rh[q] = rq;
        p[q] = 0.0;
        v[q] = 0.0;
        part = fma(rq, rq, part);
    }
    const double bnorm2 = block_sum(part, sh);
    const double tol2 = rtol * rtol * bnorm2;
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    // squared residual of the current iterate and of the kept one (xb)
    double rr_cur = bnorm2, rr_best = bnorm2;
    for (int q = tid; q < n; q += nt) xb[q] = x[q];

    int it = 0;  // iterations begun (each ends in a break or a full step)
    if (bnorm2 > 0.0) {
        for (; it < maxit; it++) {
            part = 0.0;
            for (int q = tid; q < n; q += nt) part = fma(rh[q], r[q], part);
            const double rho1 = block_sum(part, sh);
            if (rho1 == 0.0) break;
            const double beta = (rho1 / rho) * (alpha / omega);
            __syncthreads();
            for (int q = tid; q < n; q += nt) p[q] = r[q] + beta * (p[q] - omega * v[q]);
            apply(p, v);
            part = 0.0;
            for (int q = tid; q < n; q += nt) part = fma(rh[q], v[q], part);
            const double rhv = block_sum(part, sh);
            if (rhv == 0.0) break;
            alpha = rho1 / rhv;
            part = 0.0;
            for (int q = tid; q < n; q += nt) {
                s[q] = r[q] - alpha * v[q];
                part = fma(s[q], s[q], part);
            }
            const double ss = block_sum(part, sh);
            if (ss <= tol2) {
                for (int q = tid; q < n; q += nt) x[q] += alpha * p[q];
                rr_cur = ss;
                break;
            }
            apply(s, tv);
            double p1 = 0.0, p2 = 0.0;
            for (int q = tid; q < n; q += nt) {
                p1 = fma(tv[q], s[q], p1);
                p2 = fma(tv[q], tv[q], p2);
            }
            const double ts = block_sum(p1, sh);
            const double tt = block_sum(p2, sh);
            if (tt == 0.0) {
                for (int q = tid; q < n; q += nt) x[q] += alpha * p[q];
                rr_cur = ss;
                break;
            }
            omega = ts / tt;
            part = 0.0;
            for (int q = tid; q < n; q += nt) {
                x[q] += alpha * p[q] + omega * s[q];
                r[q] = s[q] - omega * tv[q];
                part = fma(r[q], r[q], part);
            }
            const double rr = block_sum(part, sh);
            rho = rho1;
            rr_cur = rr;
            if (rr <= tol2 || omega == 0.0) break;
            if (rr < rr_best) {
                rr_best = rr;
                for (int q = tid; q < n; q += nt) xb[q] = x[q];
            }
        }
    }
    // x when converged, else the kept iterate (the threads that wrote xb read
    // it back, so no barrier is needed before the copy)
    if (!(rr_cur <= tol2))
        for (int q = tid; q < n; q += nt) x[q] = xb[q];
    if (iters && tid == 0) iters[0] += (double)(it < maxit ? it + (bnorm2 > 0.0 ? 1 : 0) : it);
    __syncthreads();
    part_means(x, false, tv);
    for (int q = tid; q < n; q += nt) xout[q] = (T)(x[q] - tv[q]);
}

template <typename T>
void launch_bottom(const Dims& d, const T* rhs, T* phi, const T* cx, const T* cy, const T* cz, double h2, double rtol,
                   int maxit, int use_x0, double* work, double* iters, const double* skip_if_direct, hipStream_t s)
{
    long long n = d.n();
    int nt = (int)((n + 63) / 64) * 64;
    if (nt > 1024) nt = 1024;
    hipLaunchKernelGGL((k_bottom<T>), dim3(1), dim3(nt), 0, s, d, rhs, phi, cx, cy, cz, h2, rtol, maxit, use_x0,
                       work, iters, skip_if_direct);
}

// --------------------------------------------------------- FP64 level 0

template <bool CELL>
__global__ __launch_bounds__(256) void k_apply64(Dims d, const double* __restrict__ x, Coef<double> C, double inv_h2,
                                                 double* __restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= d.nx || j >= d.ny || k >= d.nz) return;
    const long long q = ((long long)k * d.ny + j) * d.nx + i;
    const Nbr nb = neighbours(d, q, i, j, k);
    double c0, c1, c2, c3, c4, c5;
    coef6<double, CELL>(C, d, q, nb, i, j, k, c0, c1, c2, c3, c4, c5);
    // M x = -(A x) = the residual of a zero right-hand side
    y[q] = resid_value<double>(c0, c1, c2, c3, c4, c5, x[nb.xm], x[nb.xp], x[nb.ym], x[nb.yp], x[nb.zm], x[nb.zp],
                                x[q], 0.0, inv_h2);
}

void launch_apply64(const Dims& d, const double* x, const Coef<double>& c, double inv_h2, double* y, hipStream_t s)
{
    const Shape3 sh = cells3(d.nx, d.ny, d.nz);
    if (c.cell)
        hipLaunchKernelGGL(k_apply64<true>, sh.grid, sh.block, 0, s, d, x, c, inv_h2, y);
    else
        hipLaunchKernelGGL(k_apply64<false>, sh.grid, sh.block, 0, s, d, x, c, inv_h2, y);
}

// r = b - A x for a column of lz cells per thread; the column's z-neighbours
// and z-face coefficients stay in registers (in cell mode the z-face value
// formed for the high face of one plane is the low face of the next).  Same
// arithmetic, in the same order, as resid_cell.
template <bool CELL>
__global__ __launch_bounds__(256) void k_resid64(Dims d, int lz, const double* __restrict__ x,
                                                 const double* __restrict__ b, Coef<double> C, double inv_h2,
                                                 float* __restrict__ r32, const double* __restrict__ inv_s,
                                                 double* part)
{
    __shared__ double sh[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int z0 = blockIdx.z * lz;
    const int z1 = min(z0 + lz, d.nz);
    double acc = 0.0;
    if (i < d.nx && j < d.ny) {
        const double is = r32 ? inv_s[0] : 0.0;
        const long long sy = d.nx, sz = (long long)d.nx * d.ny;
        const long long oxm = i > 0 ? -1 : (d.px ? d.nx - 1 : 0);
        const long long oxp = i < d.nx - 1 ? 1 : (d.px ? -(long long)(d.nx - 1) : 0);
        const bool hxm = i > 0 || d.px, hxp = i < d.nx - 1 || d.px;
        const long long oym = j > 0 ? -sy : (d.py ? (long long)(d.ny - 1) * sy : 0);
        const long long oyp = j < d.ny - 1 ? sy : (d.py ? -(long long)(d.ny - 1) * sy : 0);
        const bool hym = j > 0 || d.py, hyp = j < d.ny - 1 || d.py;
        long long q = (long long)z0 * sz + (long long)j * d.nx + i;
        const long long qm = z0 > 0 ? q - sz : (d.pz ? q + (long long)(d.nz - 1) * sz : q);
        double xzm = x[qm];
        double x0 = x[q];
        double cc0 = 0.0, czl;
        if constexpr (CELL) {
            cc0 = C.cell[q];
            czl = (z0 > 0 || d.pz) ? harm(C.cell[qm], cc0) : 0.0;
        } else {
            czl = C.z[q];
        }
        for (int k = z0; k < z1; k++) {
            const bool last = k == d.nz - 1;
            const bool hzp = !last || d.pz;
            const long long qp = !last ? q + sz : (d.pz ? q - (long long)(d.nz - 1) * sz : q);
            const double xzp = x[qp];
            double c0, c1, c2, c3, czh, ccp = 0.0;
            if constexpr (CELL) {
                const double* cc = C.cell;
                ccp = cc[qp];
                czh = hzp ? harm(cc0, ccp) : 0.0;
                c0 = hxm ? harm(cc[q + oxm], cc0) : 0.0;
                c1 = hxp ? harm(cc0, cc[q + oxp]) : 0.0;
                c2 = hym ? harm(cc[q + oym], cc0) : 0.0;
                c3 = hyp ? harm(cc0, cc[q + oyp]) : 0.0;
            } else {
                czh = hzp ? C.z[qp] : 0.0;
                c0 = C.x[q];
                c1 = hxp ? C.x[q + oxp] : 0.0;
                c2 = C.y[q];
                c3 = hyp ? C.y[q + oyp] : 0.0;
            }
            const double r = resid_value<double>(c0, c1, c2, c3, czl, czh, x[q + oxm], x[q + oxp], x[q + oym],
                                                 x[q + oyp], xzm, xzp, x0, b[q], inv_h2);
            acc = fma(r, r, acc);
            if (r32) r32[q] = (float)(r * is);
            xzm = x0;
            x0 = xzp;
            czl = czh;
            cc0 = ccp;
            q += sz;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        part[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

void launch_resid64(const Dims& d, const double* phi, const double* b, const Coef<double>& c, double inv_h2,
                    float* r32, const double* inv_s, double* partials, int* nb_out, hipStream_t s)
{
    const ShapeZ sh = zmarch(d.nx, d.ny, d.nz, kZBlocks);
    *nb_out = (int)sh.blocks();
    if (c.cell)
        hipLaunchKernelGGL(k_resid64<true>, sh.grid, sh.block, 0, s, d, sh.lz, phi, b, c, inv_h2, r32, inv_s,
                           partials);
    else
        hipLaunchKernelGGL(k_resid64<false>, sh.grid, sh.block, 0, s, d, sh.lz, phi, b, c, inv_h2, r32, inv_s,
                           partials);
}

// First refinement step from a zero iterate: the residual is b itself, so
// r32 = float(b * pair_in[1]) (the value the residual kernel would write) and
// the scale pair of the next step is the one of b.
__global__ __launch_bounds__(256) void k_scale32(long long n, const double* __restrict__ b, float* __restrict__ r32,
                                                 const double* __restrict__ pair_in, double* __restrict__ pair_out)
{
    const double is = pair_in[1];
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q == 0) {
        pair_out[0] = pair_in[0];
        pair_out[1] = pair_in[1];
    }
    if (r32 && q < n) r32[q] = (float)(b[q] * is);
}

void launch_scale32(long long n, const double* b, float* r32, const double* pair_in, double* pair_out, hipStream_t st)
{
    const long long work = r32 ? n : 1;
    hipLaunchKernelGGL(k_scale32, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, n, b, r32, pair_in,
                       pair_out);
}

__global__ __launch_bounds__(256) void k_ir_update(long long n, double* __restrict__ x, const float* __restrict__ e,
                                                   const double* __restrict__ s)
{
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q < n) x[q] = fma(s[0], (double)e[q], x[q]);
}

void launch_ir_update(long long n, double* phi, const float* e, const double* s, hipStream_t st)
{
    hipLaunchKernelGGL(k_ir_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, phi, e, s);
}

// ------------------------------------------------------------ instantiations

#define MP_INST(T)                                                                                                    \
    template void launch_rbgs<T>(const Dims&, T*, const T*, const Coef<T>&, T, int, int, hipStream_t);                \
    template void launch_rbgs_e<T>(const Dims&, T*, const T*, const Coef<T>&, T, int, int, const T*, hipStream_t);    \
    template void launch_rb_pair<T>(const Dims&, const T*, T*, const T*, const Coef<T>&, T, int, const T*,           \
                                    hipStream_t);                                                                     \
    template void launch_resid_restrict<T>(const Dims&, const T*, const T*, const Coef<T>&, T, T*, hipStream_t);      \
    template void launch_prolong<T>(const Dims&, T*, const T*, hipStream_t);                                          \
    template void launch_bottom<T>(const Dims&, const T*, T*, const T*, const T*, const T*, double, double, int, int, \
                                   double*, double*, const double*, hipStream_t);
MP_INST(float)
MP_INST(double)

}  // namespace mp
