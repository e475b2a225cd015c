// k_setup.hip -- gfx950 kernels for the base-state mapping, the face
// coefficients, the MAC right-hand side, the velocity correction, the
// coefficient gradient and the FP64 reductions.
//
// All of these are HBM-bound elementwise or 7-point passes: one thread per
// cell, x fastest across the 64 lanes of a wavefront so every array access is
// a contiguous 512-byte (FP64) row segment; neighbour reads hit L2.
#include "mp_device.h"
#include "mp_kernels.h"
#include "mp_launch.h"

#include <math.h>

namespace mp {

int red_blocks(long long n)
{
    long long b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > kMaxRedBlocks) b = kMaxRedBlocks;
    return (int)b;
}

static inline unsigned grid1(long long n)
{
    long long b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 1 ? 1 : b);
}

int zred_blocks(const Dims& d) { return (int)zmarch(d.nx, d.ny, d.nz, kZBlocks).blocks(); }

// Index helpers of the 3D launches.
// Workgroup p runs on XCD p % 8, each with its own L2: renumber so that each
// XCD takes one contiguous run of (column tile, plane chunk), keeping the
// rows and planes shared by neighbouring tiles inside one L2.
__device__ __forceinline__ void zcol_tile(int& bx, int& by, int& bz)
{
    const unsigned gx = gridDim.x, gy = gridDim.y, n = gridDim.x * gridDim.y * gridDim.z;
    unsigned p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    if (n % 8 == 0) p = (p % 8) * (n / 8) + p / 8;
    bx = (int)(p % gx);
    by = (int)((p / gx) % gy);
    bz = (int)(p / (gx * gy));
}

#define MP_IJK3                                                                                                       \
    int bx3_, by3_, bz3_;                                                                                             \
    zcol_tile(bx3_, by3_, bz3_);                                                                                      \
    const int i = bx3_ * blockDim.x + threadIdx.x;                                                                    \
    const int j = by3_ * blockDim.y + threadIdx.y;                                                                    \
    const int k = bz3_ * blockDim.z + threadIdx.z;

// Column (i, j) and z range [z0, z1) of a z-marching launch.
#define MP_ZCOL                                                                                                       \
    int bx_, by_, bz_;                                                                                                \
    zcol_tile(bx_, by_, bz_);                                                                                         \
    const int i = bx_ * blockDim.x + threadIdx.x;                                                                     \
    const int j = by_ * blockDim.y + threadIdx.y;                                                                     \
    const int z0 = bz_ * lz;                                                                                          \
    const int z1 = min(z0 + lz, d.nz);                                                                                \
    const bool col = i < d.nx && j < d.ny;

__device__ __forceinline__ void zpart_store(double* part, double s)
{
    if (threadIdx.x == 0 && threadIdx.y == 0)
        part[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// ---------------------------------------------------------------- reductions

__global__ __launch_bounds__(1024) void k_final_sum(const double* __restrict__ part, int nb, double* out, double scale,
                                                    double* rms_out, double count, double* zero_out)
{
    __shared__ double sh[16];
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v += part[b];
    double s = block_sum(v, sh);
    if (threadIdx.x == 0) {
        out[0] = scale * s;
        if (zero_out) zero_out[0] = 0.0;
        if (rms_out) {
            double r = sqrt(s / count);
            rms_out[0] = r > 0.0 ? r : 1.0;
            rms_out[1] = r > 0.0 ? 1.0 / r : 1.0;
        }
    }
}

void launch_final_sum(const double* partials, int nb, double* out, double scale, double* rms_out, double count,
                      hipStream_t s, double* zero_out)
{
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(1024), 0, s, partials, nb, out, scale, rms_out, count, zero_out);
}

__global__ __launch_bounds__(kBlock) void k_sum(const double* __restrict__ x, long long n, double* part)
{
    __shared__ double sh[kBlock / kWave];
    double v = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        v += x[q];
    double s = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_sum(const double* x, long long n, double* partials, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum, dim3(nb), dim3(kBlock), 0, s, x, n, partials);
}

__global__ __launch_bounds__(kBlock) void k_sub_mean_sumsq(double* __restrict__ x, long long n,
                                                           const double* __restrict__ mean, double* part,
                                                           float* __restrict__ x32, const double* __restrict__ pair,
                                                           int keep)
{
    __shared__ double sh[kBlock / kWave];
    const double m = mean[0];
    const double is = x32 ? pair[1] : 0.0;
    double v = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        double a = x[q] - m;
        if (!keep) x[q] = a;
        if (x32) x32[q] = (float)(a * is);
        v = fma(a, a, v);
    }
    double s = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_sub_mean_sumsq(double* x, long long n, const double* mean, double* partials, int nb, hipStream_t s,
                           float* x32, const double* pair, bool keep)
{
    hipLaunchKernelGGL(k_sub_mean_sumsq, dim3(nb), dim3(kBlock), 0, s, x, n, mean, partials, x32, pair, keep ? 1 : 0);
}

__global__ __launch_bounds__(1024) void k_final_moments(const double* __restrict__ part,
                                                        const double* __restrict__ part2, int nb, long long n,
                                                        double* mean_out, double* pair0, double* pair1)
{
    __shared__ double sh[16];
    double v = 0.0, w = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        v += part[b];
        w += part2[b];
    }
    const double s1 = block_sum(v, sh);
    const double s2 = block_sum(w, sh);
    if (threadIdx.x == 0) {
        const double mean = (1.0 / (double)n) * s1;
        const double raw = s2 / (double)n;
        const double var = raw - mean * mean;
        double r = var > 1e-12 * raw ? sqrt(var) : sqrt(raw);
        if (!(r > 0.0) || !isfinite(r)) r = 1.0;
        mean_out[0] = mean;
        pair0[0] = pair1[0] = r;
        pair0[1] = pair1[1] = 1.0 / r;
    }
}

void launch_final_moments(const double* partials, const double* partials2, int nb, long long n, double* mean_out,
                          double* pair0, double* pair1, hipStream_t s)
{
    hipLaunchKernelGGL(k_final_moments, dim3(1), dim3(1024), 0, s, partials, partials2, nb, n, mean_out, pair0,
                       pair1);
}

__global__ __launch_bounds__(kBlock) void k_sub_mean(double* __restrict__ x, long long n,
                                                     const double* __restrict__ mean)
{
    long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q < n) x[q] -= mean[0];
}

void launch_sub_mean(double* x, long long n, const double* mean, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub_mean, dim3(grid1(n)), dim3(kBlock), 0, s, x, n, mean);
}

__global__ __launch_bounds__(kBlock) void k_axpby(long long n, double a, double b, const double* __restrict__ x,
                                                  double* __restrict__ y)
{
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q < n) y[q] = a == 0.0 ? b * x[q] : fma(a, y[q], b * x[q]);
}

void launch_axpby(long long n, double a, double b, const double* x, double* y, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby, dim3(grid1(n)), dim3(kBlock), 0, s, n, a, b, x, y);
}

__global__ __launch_bounds__(kBlock) void k_neg_copy_sum(const double* __restrict__ rhs, double* __restrict__ b,
                                                         long long n, double* part)
{
    __shared__ double sh[kBlock / kWave];
    double v = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        double a = -rhs[q];
        b[q] = a;
        v += a;
    }
    double s = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_neg_copy_sum(const double* rhs, double* b, long long n, double* partials, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_neg_copy_sum, dim3(nb), dim3(kBlock), 0, s, rhs, b, n, partials);
}

__global__ __launch_bounds__(kBlock) void k_copy(const double* __restrict__ src, double* __restrict__ dst, long long n)
{
    long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q < n) dst[q] = src[q];
}

void launch_copy(const double* src, double* dst, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy, dim3(grid1(n)), dim3(kBlock), 0, s, src, dst, n);
}

// ------------------------------------------------------------------- fill

// Fill (Sec. 3.1) of one cell from the 1D table:
//   0 planar: direct injection of the z table;
//   1 spherical: linear interpolation in r on r_j = (j + 1/2) dr;
//   3 spherical: quadratic (Lagrange through the three table points around
//     the nearest one, the stencil kept inside the table) on the same grid;
//   2 spherical irregular base state: the table is indexed by the integer m
//     with |x - centre| = h sqrt(0.75 + 2m) (centre on the middle node);
// interpolated fills hold the end values beyond the table.
__device__ __forceinline__ double fill_value(int geometry, const double* __restrict__ tab, int n1d, double dr,
                                             double x, double y, double z, long long m)
{
    if (geometry == 2) return tab[m];
    const double r = sqrt(x * x + y * y + z * z);
    const double t = r / dr - 0.5;
    if (t <= 0.0) return tab[0];
    if (t >= (double)(n1d - 1)) return tab[n1d - 1];
    if (geometry == 3) {
        int jj = (int)floor(t + 0.5);
        jj = jj < 1 ? 1 : (jj > n1d - 2 ? n1d - 2 : jj);
        const double s = t - jj;
        return tab[jj - 1] * (0.5 * s * (s - 1.0)) + tab[jj] * (1.0 - s * s) + tab[jj + 1] * (0.5 * s * (s + 1.0));
    }
    const int jj = (int)floor(t);
    const double w = t - jj;
    return (1.0 - w) * tab[jj] + w * tab[jj + 1];
}

__global__ __launch_bounds__(kBlock) void k_fill(Dims d, int lz, double h, int geometry,
                                                 const double* __restrict__ tab, int n1d, double dr, double cx0,
                                                 double cy0, double cz0, const double* __restrict__ rho,
                                                 double* __restrict__ beta0, double* __restrict__ ccell,
                                                 float* __restrict__ ccell32, double* part)
{
    __shared__ double sh[kBlock / kWave];
    MP_ZCOL
    double bad = 0.0;
    for (int k = z0; col && k < z1; k++) {
        const long long q = ((long long)k * d.ny + j) * d.nx + i;
        double b;
        if (geometry == 0) {
            b = tab[k];
        } else {
            const long long a2 = 2LL * i + 1 - d.nx, b2 = 2LL * j + 1 - d.ny, c2 = 2LL * k + 1 - d.nz;
            const long long m = (a2 * a2 + b2 * b2 + c2 * c2 - 3) / 8;
            b = fill_value(geometry, tab, n1d, dr, (i + 0.5) * h - cx0, (j + 0.5) * h - cy0, (k + 0.5) * h - cz0, m);
        }
        const double rq = rho[q];
        const double c = b / rq;
        beta0[q] = b;
        ccell[q] = c;
        // FP32 cells as half reciprocals 0.5 / c (the FP32 harmonic mean's input)
        if (ccell32) ccell32[q] = (float)(0.5 * rq / b);
        if (!(rq > 0.0) || !isfinite(rq) || !isfinite(c) || !(b > 0.0)) bad += 1.0;
    }
    zpart_store(part, block_sum(bad, sh));
}

// S - Sbar(cell), Sbar filled from its table like beta0 (the velocity-split
// source after a uniform spherical mapping, geometry 1 or 3).
__global__ __launch_bounds__(kBlock) void k_split_fill(Dims d, double h, int geometry, const double* __restrict__ tab,
                                                       int n1d, double dr, double cx0, double cy0, double cz0,
                                                       const double* __restrict__ S, double* __restrict__ out)
{
    const long long n = d.n();
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % d.nx);
        const long long t = q / d.nx;
        const int j = (int)(t % d.ny), k = (int)(t / d.ny);
        out[q] = S[q] - fill_value(geometry, tab, n1d, dr, (i + 0.5) * h - cx0, (j + 0.5) * h - cy0,
                                   (k + 0.5) * h - cz0, 0);
    }
}

void launch_split_fill(const Dims& d, double h, int geometry, const double* tab, int n1d, double dr,
                       const double* center, const double* S, double* out, hipStream_t s)
{
    long long nb = (d.n() + kBlock - 1) / kBlock;
    nb = nb > 16384 ? 16384 : nb;
    hipLaunchKernelGGL(k_split_fill, dim3((unsigned)nb), dim3(kBlock), 0, s, d, h, geometry, tab, n1d, dr, center[0],
                       center[1], center[2], S, out);
}

void launch_fill(const Dims& d, double h, int geometry, const double* tab, int n1d, double dr, double cx0, double cy0,
                 double cz0, const double* rho, double* beta0, double* ccell, float* ccell32, double* partials,
                 hipStream_t s)
{
    const ShapeZ sh = zmarch(d.nx, d.ny, d.nz, kZBlocks);
    hipLaunchKernelGGL(k_fill, sh.grid, sh.block, 0, s, d, sh.lz, h, geometry, tab, n1d, dr, cx0, cy0, cz0, rho,
                       beta0, ccell, ccell32, partials);
}


// External face indices of the low faces of cell (i,j,k) and of the Neumann
// high walls.
struct ExtIdx {
    long long xl, yl, zl;
};

__device__ __forceinline__ ExtIdx ext_low(const Dims& d, int i, int j, int k)
{
    const int bx = !d.px, by = !d.py;
    ExtIdx e;
    e.xl = ((long long)k * d.ny + j) * (d.nx + bx) + i;
    e.yl = ((long long)k * (d.ny + by) + j) * d.nx + i;
    e.zl = ((long long)k * d.ny + j) * d.nx + i;
    return e;
}

__global__ __launch_bounds__(kBlock) void k_faces_from_cells(Dims d, const double* __restrict__ cc,
                                                             double* __restrict__ c64x, double* __restrict__ c64y,
                                                             double* __restrict__ c64z, float* __restrict__ c32x,
                                                             float* __restrict__ c32y, float* __restrict__ c32z,
                                                             double* __restrict__ ex, double* __restrict__ ey,
                                                             double* __restrict__ ez)
{
    MP_IJK3
    if (i >= d.nx || j >= d.ny || k >= d.nz) return;
    const long long q = ((long long)k * d.ny + j) * d.nx + i;
    const Nbr b = neighbours(d, q, i, j, k);
    const double c0 = cc[q];
    const double fx = (i > 0 || d.px) ? harm(cc[b.xm], c0) : 0.0;
    const double fy = (j > 0 || d.py) ? harm(cc[b.ym], c0) : 0.0;
    const double fz = (k > 0 || d.pz) ? harm(cc[b.zm], c0) : 0.0;
    if (c64x) {
        c64x[q] = fx;
        c64y[q] = fy;
        c64z[q] = fz;
    }
    if (c32x) {
        c32x[q] = (float)fx;
        c32y[q] = (float)fy;
        c32z[q] = (float)fz;
    }
    if (ex) {
        const ExtIdx e = ext_low(d, i, j, k);
        ex[e.xl] = fx;
        ey[e.yl] = fy;
        ez[e.zl] = fz;
        if (!d.px && i == d.nx - 1) ex[e.xl + 1] = 0.0;
        if (!d.py && j == d.ny - 1) ey[e.yl + d.nx] = 0.0;
        if (!d.pz && k == d.nz - 1) ez[e.zl + (long long)d.nx * d.ny] = 0.0;
    }
}

void launch_faces_from_cells(const Dims& d, const double* ccell, double* c64x, double* c64y, double* c64z,
                             float* c32x, float* c32y, float* c32z, double* ex, double* ey, double* ez,
                             hipStream_t s)
{
    const Shape3 sh = cells3(d.nx, d.ny, d.nz);
    hipLaunchKernelGGL(k_faces_from_cells, sh.grid, sh.block, 0, s, d, ccell, c64x, c64y, c64z, c32x, c32y, c32z, ex,
                       ey, ez);
}

__global__ __launch_bounds__(kBlock) void k_import_faces(Dims d, int lz, const double* __restrict__ ex,
                                                         const double* __restrict__ ey, const double* __restrict__ ez,
                                                         double* __restrict__ c64x, double* __restrict__ c64y,
                                                         double* __restrict__ c64z, float* __restrict__ c32x,
                                                         float* __restrict__ c32y, float* __restrict__ c32z,
                                                         double* part)
{
    __shared__ double sh[kBlock / kWave];
    MP_ZCOL
    double bad = 0.0;
    for (int k = z0; col && k < z1; k++) {
        const long long q = ((long long)k * d.ny + j) * d.nx + i;
        const ExtIdx e = ext_low(d, i, j, k);
        const double fx = (i > 0 || d.px) ? ex[e.xl] : 0.0;
        const double fy = (j > 0 || d.py) ? ey[e.yl] : 0.0;
        const double fz = (k > 0 || d.pz) ? ez[e.zl] : 0.0;
        if (!(fx >= 0.0) || !(fy >= 0.0) || !(fz >= 0.0) || !isfinite(fx) || !isfinite(fy) || !isfinite(fz))
            bad += 1.0;
        c64x[q] = fx;
        c64y[q] = fy;
        c64z[q] = fz;
        if (c32x) {
            c32x[q] = (float)fx;
            c32y[q] = (float)fy;
            c32z[q] = (float)fz;
        }
    }
    zpart_store(part, block_sum(bad, sh));
}

void launch_import_faces(const Dims& d, const double* ex, const double* ey, const double* ez, double* c64x,
                         double* c64y, double* c64z, float* c32x, float* c32y, float* c32z, double* partials,
                         hipStream_t s)
{
    const ShapeZ sh = zmarch(d.nx, d.ny, d.nz, kZBlocks);
    hipLaunchKernelGGL(k_import_faces, sh.grid, sh.block, 0, s, d, sh.lz, ex, ey, ez, c64x, c64y, c64z, c32x, c32y,
                       c32z, partials);
}

// Coarse low face of coarse cell (I,J,K) = mean of the 4 fine low faces of the
// fine cells that touch it.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_coef_restrict(Dims f, const Tin* __restrict__ fx,
                                                          const Tin* __restrict__ fy, const Tin* __restrict__ fz,
                                                          Tout* __restrict__ cx, Tout* __restrict__ cy,
                                                          Tout* __restrict__ cz)
{
    const int nxc = f.nx / 2, nyc = f.ny / 2, nzc = f.nz / 2;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= nxc || J >= nyc || K >= nzc) return;
    const long long q = ((long long)K * nyc + J) * nxc + I;
    const long long sy = f.nx, sz = (long long)f.nx * f.ny;
    const long long base = (long long)(2 * K) * sz + (long long)(2 * J) * sy + 2 * I;
    const double ax = (double)fx[base] + (double)fx[base + sy] + (double)fx[base + sz] + (double)fx[base + sy + sz];
    const double ay = (double)fy[base] + (double)fy[base + 1] + (double)fy[base + sz] + (double)fy[base + 1 + sz];
    const double az = (double)fz[base] + (double)fz[base + 1] + (double)fz[base + sy] + (double)fz[base + 1 + sy];
    cx[q] = (Tout)(0.25 * ax);
    cy[q] = (Tout)(0.25 * ay);
    cz[q] = (Tout)(0.25 * az);
}

template <typename Tin, typename Tout>
void launch_coef_restrict(const Dims& fine, const Tin* fx, const Tin* fy, const Tin* fz, Tout* cx, Tout* cy,
                          Tout* cz, hipStream_t s)
{
    const Shape3 sh = cells3(fine.nx / 2, fine.ny / 2, fine.nz / 2);
    hipLaunchKernelGGL((k_coef_restrict<Tin, Tout>), sh.grid, sh.block, 0, s, fine, fx, fy, fz, cx, cy, cz);
}

// Coarse low faces from fine cell values: the fine faces are harmonic means
// (FP64, as in face mode) summed in the same order as k_coef_restrict.
template <typename Tout>
__global__ __launch_bounds__(kBlock) void k_coef_restrict_cells(Dims f, const double* __restrict__ cc,
                                                                Tout* __restrict__ cx, Tout* __restrict__ cy,
                                                                Tout* __restrict__ cz)
{
    const int nxc = f.nx / 2, nyc = f.ny / 2, nzc = f.nz / 2;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= nxc || J >= nyc || K >= nzc) return;
    const long long q = ((long long)K * nyc + J) * nxc + I;
    const long long sy = f.nx, sz = (long long)f.nx * f.ny;
    const long long base = (long long)(2 * K) * sz + (long long)(2 * J) * sy + 2 * I;
    // low faces of the fine cells at i = 2I (x), j = 2J (y), k = 2K (z)
    auto fx = [&](long long qq) {
        const long long qm = I > 0 ? qq - 1 : (f.px ? qq + f.nx - 1 : -1);
        return qm >= 0 ? harm(cc[qm], cc[qq]) : 0.0;
    };
    auto fy = [&](long long qq) {
        const long long qm = J > 0 ? qq - sy : (f.py ? qq + (long long)(f.ny - 1) * sy : -1);
        return qm >= 0 ? harm(cc[qm], cc[qq]) : 0.0;
    };
    auto fz = [&](long long qq) {
        const long long qm = K > 0 ? qq - sz : (f.pz ? qq + (long long)(f.nz - 1) * sz : -1);
        return qm >= 0 ? harm(cc[qm], cc[qq]) : 0.0;
    };
    const double ax = fx(base) + fx(base + sy) + fx(base + sz) + fx(base + sy + sz);
    const double ay = fy(base) + fy(base + 1) + fy(base + sz) + fy(base + 1 + sz);
    const double az = fz(base) + fz(base + 1) + fz(base + sy) + fz(base + 1 + sy);
    cx[q] = (Tout)(0.25 * ax);
    cy[q] = (Tout)(0.25 * ay);
    cz[q] = (Tout)(0.25 * az);
}

template <typename Tout>
void launch_coef_restrict_cells(const Dims& fine, const double* cc, Tout* cx, Tout* cy, Tout* cz, hipStream_t s)
{
    const Shape3 sh = cells3(fine.nx / 2, fine.ny / 2, fine.nz / 2);
    hipLaunchKernelGGL((k_coef_restrict_cells<Tout>), sh.grid, sh.block, 0, s, fine, cc, cx, cy, cz);
}

// FP32 restriction from half reciprocals: each coarse cell's three low faces
// are the means of the 4 fine faces covering them, a fine face being the
// FP32 harmonic mean harm(h_a, h_b) of its two cells.
__global__ __launch_bounds__(kBlock) void k_coef_restrict_cells32(Dims f, const float* __restrict__ hc,
                                                                  float* __restrict__ cx, float* __restrict__ cy,
                                                                  float* __restrict__ cz)
{
    const int nxc = f.nx / 2, nyc = f.ny / 2, nzc = f.nz / 2;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= nxc || J >= nyc || K >= nzc) return;
    const long long q = ((long long)K * nyc + J) * nxc + I;
    const long long sy = f.nx, sz = (long long)f.nx * f.ny;
    const long long base = (long long)(2 * K) * sz + (long long)(2 * J) * sy + 2 * I;
    // the low neighbours of the children on the coarse cell's low faces
    const long long ox = I > 0 ? -1 : (f.px ? f.nx - 1 : 0);
    const long long oy = J > 0 ? -sy : (f.py ? (long long)(f.ny - 1) * sy : 0);
    const long long oz = K > 0 ? -sz : (f.pz ? (long long)(f.nz - 1) * sz : 0);
    const bool hx = I > 0 || f.px, hy = J > 0 || f.py, hz = K > 0 || f.pz;
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const long long qx = base + a * sz + b * sy, qy = base + a * sz + b, qz = base + a * sy + b;
            ax += hx ? harm(hc[qx + ox], hc[qx]) : 0.0f;
            ay += hy ? harm(hc[qy + oy], hc[qy]) : 0.0f;
            az += hz ? harm(hc[qz + oz], hc[qz]) : 0.0f;
        }
    cx[q] = 0.25f * ax;
    cy[q] = 0.25f * ay;
    cz[q] = 0.25f * az;
}

// The same for two x-adjacent coarse cells per thread (nx a multiple of 4):
// the four fine cells of a row segment as one 16-byte load, the x neighbour
// below the segment as one word; the same faces summed in the same order.
__global__ __launch_bounds__(kBlock) void k_coef_restrict_cells32x2(Dims f, const float* __restrict__ hc,
                                                                    float* __restrict__ cx, float* __restrict__ cy,
                                                                    float* __restrict__ cz)
{
    const int nxc = f.nx / 2, nyc = f.ny / 2, nzc = f.nz / 2;
    const int I2 = blockIdx.x * blockDim.x + threadIdx.x;  // coarse cells 2 I2, 2 I2 + 1
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (2 * I2 >= nxc || J >= nyc || K >= nzc) return;
    const long long sy = f.nx, sz = (long long)f.nx * f.ny;
    const long long base = (long long)(2 * K) * sz + (long long)(2 * J) * sy + 4 * I2;
    const long long ox = I2 > 0 ? -1 : (f.px ? f.nx - 1 : 0);
    const long long oy = J > 0 ? -sy : (f.py ? (long long)(f.ny - 1) * sy : 0);
    const long long oz = K > 0 ? -sz : (f.pz ? (long long)(f.nz - 1) * sz : 0);
    const bool hx = I2 > 0 || f.px, hy = J > 0 || f.py, hz = K > 0 || f.pz;
    auto ld4 = [&](long long q) { return *reinterpret_cast<const float4*>(hc + q); };
    // children rows (a = k child, b = j child) and their low neighbours
    float4 ch[2][2], ny_[2], nz_[2];
    float nx_[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
            ch[a][b] = ld4(base + a * sz + b * sy);
            nx_[a][b] = hx ? hc[base + a * sz + b * sy + ox] : 0.0f;
        }
#pragma unroll
    for (int a = 0; a < 2; a++) ny_[a] = hy ? ld4(base + a * sz + oy) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int b = 0; b < 2; b++) nz_[b] = hz ? ld4(base + b * sy + oz) : make_float4(0.f, 0.f, 0.f, 0.f);
    // coarse cell u (0: fine x 0, 1; 1: fine x 2, 3); accumulation order of
    // k_coef_restrict_cells32: (a, b) = (0,0), (0,1), (1,0), (1,1)
#pragma unroll
    for (int u = 0; u < 2; u++) {
        float ax = 0.0f, ay = 0.0f, az = 0.0f;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++) {
                // x face at fine x 2u: neighbour 2u - 1 (the word below the segment for u = 0)
                const float xo = u == 0 ? nx_[a][b] : ch[a][b].y;
                const float xi = u == 0 ? ch[a][b].x : ch[a][b].z;
                ax += (u == 1 || hx) ? harm(xo, xi) : 0.0f;
                // y face (children k = a, x = 2u + b) and z face (children j = a, x = 2u + b)
                const float4& cy0 = ch[a][0];
                const float4& cz0 = ch[0][a];
                const float yi = b == 0 ? (u == 0 ? cy0.x : cy0.z) : (u == 0 ? cy0.y : cy0.w);
                const float yo = b == 0 ? (u == 0 ? ny_[a].x : ny_[a].z) : (u == 0 ? ny_[a].y : ny_[a].w);
                const float zi = b == 0 ? (u == 0 ? cz0.x : cz0.z) : (u == 0 ? cz0.y : cz0.w);
                const float zo = b == 0 ? (u == 0 ? nz_[a].x : nz_[a].z) : (u == 0 ? nz_[a].y : nz_[a].w);
                ay += hy ? harm(yo, yi) : 0.0f;
                az += hz ? harm(zo, zi) : 0.0f;
            }
        const long long q = ((long long)K * nyc + J) * nxc + 2 * I2 + u;
        cx[q] = 0.25f * ax;
        cy[q] = 0.25f * ay;
        cz[q] = 0.25f * az;
    }
}

void launch_coef_restrict_cells32(const Dims& fine, const float* hc, float* cx, float* cy, float* cz, hipStream_t s)
{
    if (fine.nx % 4 == 0) {
        const Shape3 sh = cells3(fine.nx / 4, fine.ny / 2, fine.nz / 2);
        hipLaunchKernelGGL(k_coef_restrict_cells32x2, sh.grid, sh.block, 0, s, fine, hc, cx, cy, cz);
    } else {
        const Shape3 sh = cells3(fine.nx / 2, fine.ny / 2, fine.nz / 2);
        hipLaunchKernelGGL(k_coef_restrict_cells32, sh.grid, sh.block, 0, s, fine, hc, cx, cy, cz);
    }
}

template void launch_coef_restrict_cells<double>(const Dims&, const double*, double*, double*, double*, hipStream_t);
template void launch_coef_restrict_cells<float>(const Dims&, const double*, float*, float*, float*, hipStream_t);

template void launch_coef_restrict<double, double>(const Dims&, const double*, const double*, const double*, double*,
                                                   double*, double*, hipStream_t);
template void launch_coef_restrict<double, float>(const Dims&, const double*, const double*, const double*, float*,
                                                  float*, float*, hipStream_t);
template void launch_coef_restrict<float, float>(const Dims&, const float*, const float*, const float*, float*,
                                                 float*, float*, hipStream_t);

// ---------------------------------------------------------------- projection

// beta0 on a face: arithmetic mean of the two cells.
// b = beta0 S - D(beta0 U): minus the MAC right-hand side of Sec. 3.2 Steps 3/7.
// Source of a cell: S, or S - Sbar for the velocity-split constraint
// (Appendix A) with Sbar the lateral average per plane (smode 1) or per
// irregular radius (smode 2).
__device__ __forceinline__ double cell_source(const Dims& d, const double* __restrict__ S,
                                              const double* __restrict__ sbar, int smode, long long q, int i, int j,
                                              int k)
{
    if (smode == 1) return S[q] - sbar[k];
    if (smode == 2) {
        const long long a = 2LL * i + 1 - d.nx, b = 2LL * j + 1 - d.ny, c = 2LL * k + 1 - d.nz;
        return S[q] - sbar[(a * a + b * b + c * c - 3) / 8];
    }
    return S[q];
}

__global__ __launch_bounds__(kBlock) void k_mac_rhs(Dims d, int lz, double inv_h, const double* __restrict__ beta0,
                                                    const double* __restrict__ ux, const double* __restrict__ uy,
                                                    const double* __restrict__ uz, const double* __restrict__ S,
                                                    const double* __restrict__ sbar, int smode,
                                                    double* __restrict__ b, double* part,
                                                    const double* __restrict__ shift, double* part2)
{
    // shift == nullptr: write b, partials = sum b (and part2 = sum b^2 when
    // part2 != nullptr).
    // shift != nullptr: no write, partials = sum (b - shift[0])^2.
    const double sh0 = shift ? shift[0] : 0.0;
    __shared__ double sh[kBlock / kWave];
    MP_ZCOL
    double acc = 0.0, acc2 = 0.0;
    // the z flux through the low face of plane k; the high face's flux of
    // plane k is carried to plane k+1 (same operands, same value)
    double fzl = 0.0, b0 = 0.0;
    if (col) {
        const long long q = ((long long)z0 * d.ny + j) * d.nx + i;
        b0 = beta0[q];
        if (z0 > 0 || d.pz) {
            const long long qm = z0 > 0 ? q - (long long)d.nx * d.ny : q + (long long)(d.nz - 1) * d.nx * d.ny;
            fzl = 0.5 * (beta0[qm] + b0) * uz[ext_low(d, i, j, z0).zl];
        }
    }
    for (int k = z0; col && k < z1; k++) {
        const long long q = ((long long)k * d.ny + j) * d.nx + i;
        const Nbr nb = neighbours(d, q, i, j, k);
        const ExtIdx e = ext_low(d, i, j, k);
        // low faces
        const double fxl = (i > 0 || d.px) ? 0.5 * (beta0[nb.xm] + b0) * ux[e.xl] : 0.0;
        const double fyl = (j > 0 || d.py) ? 0.5 * (beta0[nb.ym] + b0) * uy[e.yl] : 0.0;
        // high faces
        double fxh = 0.0, fyh = 0.0, fzh = 0.0;
        if (i < d.nx - 1) fxh = 0.5 * (b0 + beta0[nb.xp]) * ux[e.xl + 1];
        else if (d.px) fxh = 0.5 * (b0 + beta0[nb.xp]) * ux[e.xl - (d.nx - 1)];
        if (j < d.ny - 1) fyh = 0.5 * (b0 + beta0[nb.yp]) * uy[e.yl + d.nx];
        else if (d.py) fyh = 0.5 * (b0 + beta0[nb.yp]) * uy[e.yl - (long long)(d.ny - 1) * d.nx];
        const double bzp = beta0[nb.zp];
        if (k < d.nz - 1) fzh = 0.5 * (b0 + bzp) * uz[e.zl + (long long)d.nx * d.ny];
        else if (d.pz) fzh = 0.5 * (b0 + bzp) * uz[e.zl - (long long)(d.nz - 1) * d.nx * d.ny];
        const double div = ((fxh - fxl) + (fyh - fyl) + (fzh - fzl)) * inv_h;
        const double v = b0 * cell_source(d, S, sbar, smode, q, i, j, k) - div;
        if (shift) {
            const double e2 = v - sh0;
            acc = fma(e2, e2, acc);
        } else {
            b[q] = v;
            acc += v;
            acc2 = fma(v, v, acc2);
        }
        fzl = fzh;
        b0 = bzp;
    }
    zpart_store(part, block_sum(acc, sh));
    if (part2) zpart_store(part2, block_sum(acc2, sh));
}

void launch_mac_rhs(const Dims& d, double inv_h, const double* beta0, const double* ux, const double* uy,
                    const double* uz, const double* S, const double* sbar, int smode, double* b, double* partials,
                    hipStream_t s, double* partials2)
{
    const ShapeZ sh = zmarch(d.nx, d.ny, d.nz, kZBlocks);
    hipLaunchKernelGGL(k_mac_rhs, sh.grid, sh.block, 0, s, d, sh.lz, inv_h, beta0, ux, uy, uz, S, sbar, smode, b,
                       partials, (const double*)nullptr, partials2);
}

void launch_rhs_defect(const Dims& d, double inv_h, const double* beta0, const double* ux, const double* uy,
                       const double* uz, const double* S, const double* sbar, int smode, const double* shift,
                       double* partials, hipStream_t s)
{
    const ShapeZ sh = zmarch(d.nx, d.ny, d.nz, kZBlocks);
    hipLaunchKernelGGL(k_mac_rhs, sh.grid, sh.block, 0, s, d, sh.lz, inv_h, beta0, ux, uy, uz, S, sbar, smode,
                       (double*)nullptr, partials, shift, (double*)nullptr);
}

// Lateral average of a planar atmosphere (Sec. 3.1): one block per plane,
// fixed-order sum of its cells, divided by their number.
__global__ __launch_bounds__(kBlock) void k_plane_average(Dims d, const double* __restrict__ phi,
                                                          double* __restrict__ avg)
{
    __shared__ double sh[kBlock / kWave];
    const long long np = (long long)d.nx * d.ny;
    const double* p = phi + (long long)blockIdx.x * np;
    double s = 0.0;
    for (long long q = threadIdx.x; q < np; q += kBlock) s += p[q];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) avg[blockIdx.x] = s / (double)np;
}

void launch_plane_average(const Dims& d, const double* phi, double* avg, hipStream_t s)
{
    hipLaunchKernelGGL(k_plane_average, dim3((unsigned)d.nz), dim3(kBlock), 0, s, d, phi, avg);
}

// Velocity correction of one face: U - (c / beta0_f) (phi_R - phi_L) / h.
__device__ __forceinline__ double corrected(double u, double c, double bl, double br, double pl, double pr,
                                            double inv_h)
{
    return u - c / (0.5 * (bl + br)) * ((pr - pl) * inv_h);
}

// Each thread owns the low faces of its cell: it alone reads and writes them,
// so the update is race-free in place.  Neumann walls are left unchanged.
template <bool CELL>
__global__ __launch_bounds__(kBlock) void k_vel_correct(Dims d, double inv_h, Coef<double> C,
                                                        const double* __restrict__ beta0,
                                                        const double* __restrict__ phi, double* __restrict__ ux,
                                                        double* __restrict__ uy, double* __restrict__ uz)
{
    MP_IJK3
    if (i >= d.nx || j >= d.ny || k >= d.nz) return;
    const long long q = ((long long)k * d.ny + j) * d.nx + i;
    const Nbr nb = neighbours(d, q, i, j, k);
    const ExtIdx e = ext_low(d, i, j, k);
    const double b0 = beta0[q], p0 = phi[q];
    double c0, c1, c2, c3, c4, c5;
    coef6<double, CELL>(C, d, q, nb, i, j, k, c0, c1, c2, c3, c4, c5);
    if (i > 0 || d.px) ux[e.xl] = corrected(ux[e.xl], c0, beta0[nb.xm], b0, phi[nb.xm], p0, inv_h);
    if (j > 0 || d.py) uy[e.yl] = corrected(uy[e.yl], c2, beta0[nb.ym], b0, phi[nb.ym], p0, inv_h);
    if (k > 0 || d.pz) uz[e.zl] = corrected(uz[e.zl], c4, beta0[nb.zm], b0, phi[nb.zm], p0, inv_h);
}

void launch_vel_correct(const Dims& d, double inv_h, const Coef<double>& c64, const double* beta0, const double* phi,
                        double* ux, double* uy, double* uz, hipStream_t s)
{
    const Shape3 sh = cells3(d.nx, d.ny, d.nz);
    if (c64.cell)
        hipLaunchKernelGGL(k_vel_correct<true>, sh.grid, sh.block, 0, s, d, inv_h, c64, beta0, phi, ux, uy, uz);
    else
        hipLaunchKernelGGL(k_vel_correct<false>, sh.grid, sh.block, 0, s, d, inv_h, c64, beta0, phi, ux, uy, uz);
}

// Coefficient gradient on the low faces of each cell; Neumann high walls 0.
__global__ __launch_bounds__(kBlock) void k_coef_grad(Dims d, double inv_h2, const double* __restrict__ lam,
                                                      const double* __restrict__ phi, double* __restrict__ gx,
                                                      double* __restrict__ gy, double* __restrict__ gz)
{
    MP_IJK3
    if (i >= d.nx || j >= d.ny || k >= d.nz) return;
    const long long q = ((long long)k * d.ny + j) * d.nx + i;
    const Nbr nb = neighbours(d, q, i, j, k);
    const ExtIdx e = ext_low(d, i, j, k);
    const double l0 = lam[q], p0 = phi[q];
    gx[e.xl] = (i > 0 || d.px) ? (l0 - lam[nb.xm]) * (p0 - phi[nb.xm]) * inv_h2 : 0.0;
    gy[e.yl] = (j > 0 || d.py) ? (l0 - lam[nb.ym]) * (p0 - phi[nb.ym]) * inv_h2 : 0.0;
    gz[e.zl] = (k > 0 || d.pz) ? (l0 - lam[nb.zm]) * (p0 - phi[nb.zm]) * inv_h2 : 0.0;
    if (!d.px && i == d.nx - 1) gx[e.xl + 1] = 0.0;
    if (!d.py && j == d.ny - 1) gy[e.yl + d.nx] = 0.0;
    if (!d.pz && k == d.nz - 1) gz[e.zl + (long long)d.nx * d.ny] = 0.0;
}

void launch_coef_grad(const Dims& d, double inv_h2, const double* lam, const double* phi, double* gx, double* gy,
                      double* gz, hipStream_t s)
{
    const Shape3 sh = cells3(d.nx, d.ny, d.nz);
    hipLaunchKernelGGL(k_coef_grad, sh.grid, sh.block, 0, s, d, inv_h2, lam, phi, gx, gy, gz);
}

}  // namespace mp
