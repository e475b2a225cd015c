// k_mg.hip -- gfx950 multigrid kernels: red-black Gauss-Seidel smoother,
// fused residual + 8-cell restriction, piecewise-constant prolongation,
// FP64 BiCGStab on the coarsest grid, and the FP64 level-0 residual and
// update of the iterative refinement.
//
// The stencils are bandwidth-bound (about 20 flops per 24-48 bytes), so no
// matrix cores are involved; the design goals are contiguous x-fastest rows
// per wavefront and as few passes over HBM as possible.
#include "mp_device.h"
#include "mp_kernels.h"

#include <math.h>

namespace mp {

static inline unsigned grid1(long long n)
{
    long long b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 1 ? 1 : b);
}

// ------------------------------------------------------------------ smoother

// One colour of a red-black Gauss-Seidel sweep on A x = b (in place).
// Colour of cell (i,j,k) is (i+j+k) mod 2; thread t owns the pair of x
// cells (2p, 2p+1) of one row and updates the one of the requested colour:
//     x_i = (h^2 b_i + sum_f c_f x_nb(f)) / sum_f c_f.
// zero_init: the iterate is zero on entry -- the neighbours are not read and
// the other cell of the pair is set to zero (so no separate clear is needed).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rbgs(Dims d, T* __restrict__ x, const T* __restrict__ b,
                                                 const T* __restrict__ cx, const T* __restrict__ cy,
                                                 const T* __restrict__ cz, T h2, int colour, int zero_init)
{
    const int nxh = (d.nx + 1) >> 1;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long total = (long long)nxh * d.ny * d.nz;
    if (t >= total) return;
    const long long row = t / nxh;
    const int p = (int)(t - row * nxh);
    const int k = (int)(row / d.ny);
    const int j = (int)(row - (long long)k * d.ny);
    const int par = (j + k + colour) & 1;
    const int i = 2 * p + par;
    const long long rbase = row * d.nx;
    if (zero_init) {
        const int io = 2 * p + (1 - par);
        if (io < d.nx) x[rbase + io] = T(0);
    }
    if (i >= d.nx) return;
    const long long q = rbase + i;
    const Nbr nb = neighbours(d, q, i, j, k);
    T csum, cv;
    if (zero_init) {
        const T c0 = cx[q], c1 = ld_or0(cx, nb.cxp), c2 = cy[q], c3 = ld_or0(cy, nb.cyp), c4 = cz[q],
                c5 = ld_or0(cz, nb.czp);
        csum = ((((c0 + c1) + c2) + c3) + c4) + c5;
        cv = T(0);
    } else {
        stencil_sums<T>(cx, cy, cz, x, q, nb, csum, cv);
    }
    x[q] = csum > T(0) ? fma(h2, b[q], cv) / csum : (zero_init ? T(0) : x[q]);
}

template <typename T>
void launch_rbgs(const Dims& d, T* phi, const T* rhs, const T* cx, const T* cy, const T* cz, T h2, int colour,
                 int zero_init, hipStream_t s)
{
    const long long total = (long long)((d.nx + 1) / 2) * d.ny * d.nz;
    hipLaunchKernelGGL((k_rbgs<T>), dim3(grid1(total)), dim3(kBlock), 0, s, d, phi, rhs, cx, cy, cz, h2, colour,
                       zero_init);
}

// --------------------------------------------------------- transfer operators

// Coarse rhs = mean of the 8 fine residuals r = b - A x (one thread per
// coarse cell; lanes read adjacent fine pairs, so rows stay contiguous).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_resid_restrict(Dims d, const T* __restrict__ x, const T* __restrict__ b,
                                                           const T* __restrict__ cx, const T* __restrict__ cy,
                                                           const T* __restrict__ cz, T inv_h2, T* __restrict__ bc)
{
    const int nxc = d.nx / 2, nyc = d.ny / 2, nzc = d.nz / 2;
    const long long qc = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (qc >= (long long)nxc * nyc * nzc) return;
    const long long t = qc / nxc;
    const int I = (int)(qc - t * nxc), K = (int)(t / nyc), J = (int)(t - (long long)K * nyc);
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int bb = 0; bb < 2; bb++)
#pragma unroll
            for (int a = 0; a < 2; a++) {
                const int i = 2 * I + a, j = 2 * J + bb, k = 2 * K + c;
                const long long q = ((long long)k * d.ny + j) * d.nx + i;
                const Nbr nb = neighbours(d, q, i, j, k);
                T csum, cvs;
                stencil_sums<T>(cx, cy, cz, x, q, nb, csum, cvs);
                const T r = b[q] - (csum * x[q] - cvs) * inv_h2;
                acc += r;
            }
    bc[qc] = T(0.125) * acc;
}

template <typename T>
void launch_resid_restrict(const Dims& fine, const T* phi, const T* rhs, const T* cx, const T* cy, const T* cz,
                           T inv_h2, T* coarse_rhs, hipStream_t s)
{
    const long long nc = (long long)(fine.nx / 2) * (fine.ny / 2) * (fine.nz / 2);
    hipLaunchKernelGGL((k_resid_restrict<T>), dim3(grid1(nc)), dim3(kBlock), 0, s, fine, phi, rhs, cx, cy, cz, inv_h2,
                       coarse_rhs);
}

// Fine x += coarse e of the parent cell.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(Dims d, T* __restrict__ x, const T* __restrict__ e)
{
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= d.n()) return;
    int i, j, k;
    cell_ijk(d, q, i, j, k);
    const int nxc = d.nx / 2, nyc = d.ny / 2;
    x[q] += e[((long long)(k >> 1) * nyc + (j >> 1)) * nxc + (i >> 1)];
}

template <typename T>
void launch_prolong(const Dims& fine, T* phi, const T* coarse_phi, hipStream_t s)
{
    hipLaunchKernelGGL((k_prolong<T>), dim3(grid1(fine.n())), dim3(kBlock), 0, s, fine, phi, coarse_phi);
}

// ------------------------------------------------------------ bottom solve

// BiCGStab in FP64 for A x = b on the coarsest grid, run by one workgroup.
// b is made mean-zero first (the system is singular with the constants as
// null space); the result is returned mean-zero.  With use_x0 the iteration
// starts from the x passed in and stops at rtol times the initial residual;
// otherwise it starts from zero.  work holds 7 n doubles.
template <typename T>
__global__ __launch_bounds__(1024) void k_bottom(Dims d, const T* __restrict__ bin, T* __restrict__ xout,
                                                 const T* __restrict__ cx, const T* __restrict__ cy,
                                                 const T* __restrict__ cz, double h2, double rtol, int maxit,
                                                 int use_x0, double* __restrict__ work)
{
    __shared__ double sh[16];
    const int n = (int)d.n();
    const int tid = threadIdx.x, nt = blockDim.x;
    double* x = work;
    double* r = work + n;
    double* rh = work + 2 * n;
    double* p = work + 3 * n;
    double* v = work + 4 * n;
    double* s = work + 5 * n;
    double* tv = work + 6 * n;
    const double inv_h2 = 1.0 / h2;

    double part = 0.0;
    for (int q = tid; q < n; q += nt) part += (double)bin[q];
    const double mean = block_sum(part, sh) / n;
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
        const double rq = ((double)bin[q] - mean) - (use_x0 ? tv[q] : 0.0);
        r[q] = rq;
        rh[q] = rq;
        p[q] = 0.0;
        v[q] = 0.0;
        part = fma(rq, rq, part);
    }
    const double bnorm2 = block_sum(part, sh);
    const double tol2 = rtol * rtol * bnorm2;
    double rho = 1.0, alpha = 1.0, omega = 1.0;

    if (bnorm2 > 0.0) {
        for (int it = 0; it < maxit; it++) {
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
            if (rr <= tol2 || omega == 0.0) break;
        }
    }
    __syncthreads();
    part = 0.0;
    for (int q = tid; q < n; q += nt) part += x[q];
    const double xm = block_sum(part, sh) / n;
    for (int q = tid; q < n; q += nt) xout[q] = (T)(x[q] - xm);
}

template <typename T>
void launch_bottom(const Dims& d, const T* rhs, T* phi, const T* cx, const T* cy, const T* cz, double h2, double rtol,
                   int maxit, int use_x0, double* work, hipStream_t s)
{
    long long n = d.n();
    int nt = (int)((n + 63) / 64) * 64;
    if (nt > 1024) nt = 1024;
    hipLaunchKernelGGL((k_bottom<T>), dim3(1), dim3(nt), 0, s, d, rhs, phi, cx, cy, cz, h2, rtol, maxit, use_x0,
                       work);
}

// --------------------------------------------------------- FP64 level 0

__global__ __launch_bounds__(kBlock) void k_apply64(Dims d, const double* __restrict__ x,
                                                    const double* __restrict__ cx, const double* __restrict__ cy,
                                                    const double* __restrict__ cz, double inv_h2,
                                                    double* __restrict__ y)
{
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= d.n()) return;
    int i, j, k;
    cell_ijk(d, q, i, j, k);
    const Nbr nb = neighbours(d, q, i, j, k);
    double csum, cv;
    stencil_sums<double>(cx, cy, cz, x, q, nb, csum, cv);
    y[q] = (cv - csum * x[q]) * inv_h2;
}

void launch_apply64(const Dims& d, const double* x, const double* cx, const double* cy, const double* cz,
                    double inv_h2, double* y, hipStream_t s)
{
    hipLaunchKernelGGL(k_apply64, dim3(grid1(d.n())), dim3(kBlock), 0, s, d, x, cx, cy, cz, inv_h2, y);
}

__global__ __launch_bounds__(kBlock) void k_resid64(Dims d, const double* __restrict__ x,
                                                    const double* __restrict__ b, const double* __restrict__ cx,
                                                    const double* __restrict__ cy, const double* __restrict__ cz,
                                                    double inv_h2, float* __restrict__ r32,
                                                    const double* __restrict__ inv_s, double* part)
{
    __shared__ double sh[kBlock / kWave];
    const long long n = d.n();
    const double is = r32 ? inv_s[0] : 0.0;
    double acc = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_ijk(d, q, i, j, k);
        const Nbr nb = neighbours(d, q, i, j, k);
        double csum, cv;
        stencil_sums<double>(cx, cy, cz, x, q, nb, csum, cv);
        const double r = b[q] - (csum * x[q] - cv) * inv_h2;
        acc = fma(r, r, acc);
        if (r32) r32[q] = (float)(r * is);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_resid64(const Dims& d, const double* phi, const double* b, const double* cx, const double* cy,
                    const double* cz, double inv_h2, float* r32, const double* inv_s, double* partials, int nb,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_resid64, dim3(nb), dim3(kBlock), 0, s, d, phi, b, cx, cy, cz, inv_h2, r32, inv_s, partials);
}

__global__ __launch_bounds__(kBlock) void k_ir_update(long long n, double* __restrict__ x,
                                                      const float* __restrict__ e, const double* __restrict__ s)
{
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q < n) x[q] = fma(s[0], (double)e[q], x[q]);
}

void launch_ir_update(long long n, double* phi, const float* e, const double* s, hipStream_t st)
{
    hipLaunchKernelGGL(k_ir_update, dim3(grid1(n)), dim3(kBlock), 0, st, n, phi, e, s);
}

// ------------------------------------------------------------ instantiations

#define MP_INST(T)                                                                                                    \
    template void launch_rbgs<T>(const Dims&, T*, const T*, const T*, const T*, const T*, T, int, int, hipStream_t);  \
    template void launch_resid_restrict<T>(const Dims&, const T*, const T*, const T*, const T*, const T*, T, T*,      \
                                           hipStream_t);                                                              \
    template void launch_prolong<T>(const Dims&, T*, const T*, hipStream_t);                                          \
    template void launch_bottom<T>(const Dims&, const T*, T*, const T*, const T*, const T*, double, double, int, int, \
                                   double*, hipStream_t);
MP_INST(float)
MP_INST(double)

}  // namespace mp
