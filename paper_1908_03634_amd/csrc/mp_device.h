// mp_device.h -- device helpers shared by the gfx950 kernels of libmproj.
//
// Internal face layout ("low-face" layout): every coefficient array has the
// cell shape [nz][ny][nx]; entry (k,j,i) of the x array is the coefficient on
// the low x face of cell (i,j,k) (0 on a Neumann wall).  The high x face of
// cell i is the low face of cell i+1, of cell 0 across a periodic wrap, or a
// wall (0) at a Neumann end.  The same holds for y and z.  One shape for all
// arrays keeps every stencil read x-contiguous and free of per-axis strides.
//
// Sign convention inside the library: A = -M = G^T C G, so A is symmetric
// positive semi-definite and the solver works on A x = b with b = -rhs:
//   (A x)_i = (1/h^2) sum_f c_f (x_i - x_nb(f)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mp_kernels.h"

#pragma clang fp contract(off)

namespace mp {

constexpr int kWave = 64;

struct Dims {
    int nx, ny, nz;
    int px, py, pz;  // 1 = periodic axis, 0 = Neumann walls
    __host__ __device__ long long n() const { return (long long)nx * ny * nz; }
};

// Neighbour offsets and high-face coefficients of cell (i,j,k) at linear index q.
// Quotient by a divisor fixed for a loop: q = (e * m) >> 32 with
// m = ceil(2^32 / d), exact whenever e * d < 2^32 (the single-workgroup
// coarse cycles index at most a few thousand cells), in place of the generic
// integer division.  ceil(2^32 / d) = floor((2^32 - 1) / d) + 1 for d >= 2,
// one 32-bit division per loop; d = 1 divides by itself.
struct FastDiv {
    unsigned m, d;
    __device__ __forceinline__ explicit FastDiv(unsigned dv) : m(dv > 1 ? 0xFFFFFFFFu / dv + 1u : 0u), d(dv) {}
    __device__ __forceinline__ unsigned div(unsigned e) const { return d > 1 ? __umulhi(e, m) : e; }
};

// (a, b, c) of e = a + na (b + nb c).
__device__ __forceinline__ void split3(unsigned e, const FastDiv& na, const FastDiv& nb, int& a, int& b, int& c)
{
    const unsigned t = na.div(e), u = nb.div(t);
    a = (int)(e - t * na.d);
    b = (int)(t - u * nb.d);
    c = (int)u;
}

struct Nbr {
    long long xm, xp, ym, yp, zm, zp;  // neighbour linear indices (self at a wall)
    long long cxp, cyp, czp;            // index of the high-face coefficient, -1 at a wall
};

__device__ __forceinline__ Nbr neighbours(const Dims& d, long long q, int i, int j, int k)
{
    Nbr b;
    const long long sx = 1, sy = d.nx, sz = (long long)d.nx * d.ny;
    // x
    if (i > 0) b.xm = q - sx;
    else b.xm = d.px ? q + (long long)(d.nx - 1) * sx : q;
    if (i < d.nx - 1) { b.xp = q + sx; b.cxp = q + sx; }
    else if (d.px) { b.xp = q - (long long)(d.nx - 1) * sx; b.cxp = b.xp; }
    else { b.xp = q; b.cxp = -1; }
    // y
    if (j > 0) b.ym = q - sy;
    else b.ym = d.py ? q + (long long)(d.ny - 1) * sy : q;
    if (j < d.ny - 1) { b.yp = q + sy; b.cyp = q + sy; }
    else if (d.py) { b.yp = q - (long long)(d.ny - 1) * sy; b.cyp = b.yp; }
    else { b.yp = q; b.cyp = -1; }
    // z
    if (k > 0) b.zm = q - sz;
    else b.zm = d.pz ? q + (long long)(d.nz - 1) * sz : q;
    if (k < d.nz - 1) { b.zp = q + sz; b.czp = q + sz; }
    else if (d.pz) { b.zp = q - (long long)(d.nz - 1) * sz; b.czp = b.zp; }
    else { b.zp = q; b.czp = -1; }
    return b;
}

// The neighbours of neighbours() in 32-bit arithmetic, for levels of fewer
// than 2^31 cells (a neighbour behind a wall is the cell itself; hx, hy, hz:
// the high face lies inside the domain, else its coefficient is 0).
struct Nb32 {
    int xm, xp, ym, yp, zm, zp;
    bool hx, hy, hz;
};

__device__ __forceinline__ Nb32 nb32(const Dims& d, int q, int i, int j, int k)
{
    const int sy = d.nx, sz = d.nx * d.ny;
    Nb32 b;
    b.xm = i > 0 ? q - 1 : (d.px ? q + (d.nx - 1) : q);
    b.xp = i < d.nx - 1 ? q + 1 : (d.px ? q - (d.nx - 1) : q);
    b.ym = j > 0 ? q - sy : (d.py ? q + (d.ny - 1) * sy : q);
    b.yp = j < d.ny - 1 ? q + sy : (d.py ? q - (d.ny - 1) * sy : q);
    b.zm = k > 0 ? q - sz : (d.pz ? q + (d.nz - 1) * sz : q);
    b.zp = k < d.nz - 1 ? q + sz : (d.pz ? q - (d.nz - 1) * sz : q);
    b.hx = i < d.nx - 1 || d.px;
    b.hy = j < d.ny - 1 || d.py;
    b.hz = k < d.nz - 1 || d.pz;
    return b;
}

template <typename Tc>
__device__ __forceinline__ Tc ld_or0(const Tc* a, long long q)
{
    return q >= 0 ? a[q] : Tc(0);
}

// Sum of the six face coefficients (csum) and sum of c_f * x_nb(f) (cx) in a
// fixed order, computed in Acc precision.
template <typename Acc, typename Tc, typename Tv>
__device__ __forceinline__ void stencil_sums(const Tc* __restrict__ cxa, const Tc* __restrict__ cya,
                                             const Tc* __restrict__ cza, const Tv* __restrict__ x, long long q,
                                             const Nbr& b, Acc& csum, Acc& cx)
{
    const Acc c0 = (Acc)cxa[q], c1 = (Acc)ld_or0(cxa, b.cxp);
    const Acc c2 = (Acc)cya[q], c3 = (Acc)ld_or0(cya, b.cyp);
    const Acc c4 = (Acc)cza[q], c5 = (Acc)ld_or0(cza, b.czp);
    csum = ((((c0 + c1) + c2) + c3) + c4) + c5;
    Acc s = c0 * (Acc)x[b.xm];
    s = fma(c1, (Acc)x[b.xp], s);
    s = fma(c2, (Acc)x[b.ym], s);
    s = fma(c3, (Acc)x[b.yp], s);
    s = fma(c4, (Acc)x[b.zm], s);
    s = fma(c5, (Acc)x[b.zp], s);
    cx = s;
}

// Decompose a linear cell index.
__device__ __forceinline__ void cell_ijk(const Dims& d, long long q, int& i, int& j, int& k)
{
    long long t = q / d.nx;
    i = (int)(q - t * d.nx);
    k = (int)(t / d.ny);
    j = (int)(t - (long long)k * d.ny);
}

// Wavefront sum (every lane holds the total; lane 0's value is the one used).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Wavefront sum whose value is lane 0's result broadcast to every lane, so all
// lanes take identical branches on it.
__device__ __forceinline__ double wave_sum_bcast(double v)
{
    v = wave_sum(v);
    return __shfl(v, 0, kWave);
}

// Block sum in a fixed order; every thread receives the same value.  Works
// for 1D, 2D and 3D blocks whose thread count is a multiple of 64 (full
// wavefronts).  `sh` must hold (threads per block) / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    const int lane = t & (kWave - 1), w = t / kWave;
    const int nw = (nthr + kWave - 1) / kWave;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; q++) s += sh[q];
    return s;
}

// ---------------------------------------------------------------------------
// Per-cell multigrid operations.  Every kernel variant (one launch per colour,
// the single-workgroup coarse cycle, the fused sweep) evaluates a cell with
// exactly this arithmetic, so the variants agree bit for bit.

// Harmonic mean 2ab/(a+b) of two cell values.  FP64 takes the values a, b
// and the same expression as the stored face coefficients (so both modes
// agree bit for bit).  FP32, used only inside the refinement's V-cycles, holds
// every cell as its half reciprocal 0.5/c (written by the mapping), so the
// mean of two cells is the hardware reciprocal of their sum: one add and one
// reciprocal per face instead of three multiplies more.
__device__ __forceinline__ double harm(double a, double b) { return 2.0 * a * b / (a + b); }
__device__ __forceinline__ float harm(float ha, float hb) { return __builtin_amdgcn_rcpf(ha + hb); }

// The six face coefficients of cell q in stencil order (x low, x high,
// y low, y high, z low, z high); walls give 0.
template <typename T, bool CELL>
__device__ __forceinline__ void coef6(const Coef<T>& C, const Dims& d, long long q, const Nbr& nb, int i, int j, int k,
                                      T& c0, T& c1, T& c2, T& c3, T& c4, T& c5)
{
    if constexpr (CELL) {
        const T* cc = C.cell;
        const T cq = cc[q];
        c0 = (i > 0 || d.px) ? harm(cc[nb.xm], cq) : T(0);
        c1 = nb.cxp >= 0 ? harm(cq, cc[nb.xp]) : T(0);
        c2 = (j > 0 || d.py) ? harm(cc[nb.ym], cq) : T(0);
        c3 = nb.cyp >= 0 ? harm(cq, cc[nb.yp]) : T(0);
        c4 = (k > 0 || d.pz) ? harm(cc[nb.zm], cq) : T(0);
        c5 = nb.czp >= 0 ? harm(cq, cc[nb.zp]) : T(0);
    } else {
        c0 = C.x[q];
        c1 = ld_or0(C.x, nb.cxp);
        c2 = C.y[q];
        c3 = ld_or0(C.y, nb.cyp);
        c4 = C.z[q];
        c5 = ld_or0(C.z, nb.czp);
    }
}

// Quotient of the Gauss-Seidel update: correctly rounded in FP64; in FP32
// (the refinement's V-cycles only) a multiply by the hardware reciprocal.
__device__ __forceinline__ double gs_div(double n, double d) { return n / d; }
__device__ __forceinline__ float gs_div(float n, float d) { return n * __builtin_amdgcn_rcpf(d); }

// Gauss-Seidel value of cell q from its neighbours in x:
//   (h^2 b_q + sum_f c_f x_nb(f)) / sum_f c_f,
// or the old value when the cell has no coupling.
template <typename T>
__device__ __forceinline__ T coef_sum(T c0, T c1, T c2, T c3, T c4, T c5)
{
    return ((((c0 + c1) + c2) + c3) + c4) + c5;
}

// Over-relaxation factor w of the red-black sweep: a cell moves from its old
// value x to x + w (g - x), g its Gauss-Seidel value.  Red-black smoothing in
// multigrid contracts fastest with w a little above 1 (I. Yavneh, On red-black
// SOR smoothing in multigrid, SIAM J. Sci. Comput. 17, 1996).
constexpr double kSorOmega = 1.08;

// The same with the coefficient sum csum = coef_sum(c0..c5) given; old is the
// cell's value before the update (0 from a zero iterate).
template <typename T>
__device__ __forceinline__ T gs_value_cs(T csum, T c0, T c1, T c2, T c3, T c4, T c5, T xm, T xp, T ym, T yp, T zm,
                                         T zp, T bq, T h2, T old)
{
    T s = c0 * xm;
    s = fma(c1, xp, s);
    s = fma(c2, ym, s);
    s = fma(c3, yp, s);
    s = fma(c4, zm, s);
    s = fma(c5, zp, s);
    return csum > T(0) ? fma(T(kSorOmega), gs_div(fma(h2, bq, s), csum) - old, old) : old;
}

template <typename T>
__device__ __forceinline__ T gs_value(T c0, T c1, T c2, T c3, T c4, T c5, T xm, T xp, T ym, T yp, T zm, T zp, T bq,
                                      T h2, T old)
{
    return gs_value_cs<T>(coef_sum<T>(c0, c1, c2, c3, c4, c5), c0, c1, c2, c3, c4, c5, xm, xp, ym, yp, zm, zp, bq, h2,
                          old);
}

// Residual b - A x of one cell from its coefficients (sum csum) and
// neighbour values.
template <typename T>
__device__ __forceinline__ T resid_value_cs(T csum, T c0, T c1, T c2, T c3, T c4, T c5, T xm, T xp, T ym, T yp, T zm,
                                            T zp, T x0, T bq, T inv_h2)
{
    T s = c0 * xm;
    s = fma(c1, xp, s);
    s = fma(c2, ym, s);
    s = fma(c3, yp, s);
    s = fma(c4, zm, s);
    s = fma(c5, zp, s);
    return bq - (csum * x0 - s) * inv_h2;
}

template <typename T>
__device__ __forceinline__ T resid_value(T c0, T c1, T c2, T c3, T c4, T c5, T xm, T xp, T ym, T yp, T zm, T zp, T x0,
                                         T bq, T inv_h2)
{
    return resid_value_cs<T>(coef_sum<T>(c0, c1, c2, c3, c4, c5), c0, c1, c2, c3, c4, c5, xm, xp, ym, yp, zm, zp, x0,
                             bq, inv_h2);
}

// One cell of one colour of red-black Gauss-Seidel on A x = b, in place.
// (p, j, k): pair index along x, row, plane; the cell updated is the one of
// the pair with (i + j + k) % 2 == colour.  zero_init: x is zero on entry;
// neighbours are not read and the other cell of the pair is cleared.
template <typename T, bool CELL>
__device__ __forceinline__ void rbgs_cell(const Dims& d, T* __restrict__ x, const T* __restrict__ b, const Coef<T>& C,
                                          T h2, int colour, int zero_init, int p, int j, int k)
{
    const int par = (j + k + colour) & 1;
    const int i = 2 * p + par;
    const long long rbase = ((long long)k * d.ny + j) * d.nx;
    if (zero_init) {
        const int io = 2 * p + (1 - par);
        if (io < d.nx) x[rbase + io] = T(0);
    }
    if (i >= d.nx) return;
    const long long q = rbase + i;
    const Nbr nb = neighbours(d, q, i, j, k);
    T c0, c1, c2, c3, c4, c5;
    coef6<T, CELL>(C, d, q, nb, i, j, k, c0, c1, c2, c3, c4, c5);
    if (zero_init)
        x[q] = gs_value<T>(c0, c1, c2, c3, c4, c5, T(0), T(0), T(0), T(0), T(0), T(0), b[q], h2, T(0));
    else
        x[q] = gs_value<T>(c0, c1, c2, c3, c4, c5, x[nb.xm], x[nb.xp], x[nb.ym], x[nb.yp], x[nb.zm], x[nb.zp], b[q],
                           h2, x[q]);
}

// Residual r = b - A x at one cell.
template <typename T, bool CELL>
__device__ __forceinline__ T resid_cell(const Dims& d, const T* __restrict__ x, const T* __restrict__ b,
                                        const Coef<T>& C, T inv_h2, int i, int j, int k)
{
    const long long q = ((long long)k * d.ny + j) * d.nx + i;
    const Nbr nb = neighbours(d, q, i, j, k);
    T c0, c1, c2, c3, c4, c5;
    coef6<T, CELL>(C, d, q, nb, i, j, k, c0, c1, c2, c3, c4, c5);
    return resid_value<T>(c0, c1, c2, c3, c4, c5, x[nb.xm], x[nb.xp], x[nb.ym], x[nb.yp], x[nb.zm], x[nb.zp], x[q],
                          b[q], inv_h2);
}

// Coarse right-hand side of coarse cell (I,J,K): mean of the 8 fine residuals.
template <typename T, bool CELL>
__device__ __forceinline__ T restrict_cell(const Dims& d, const T* __restrict__ x, const T* __restrict__ b,
                                           const Coef<T>& C, T inv_h2, int I, int J, int K)
{
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int bb = 0; bb < 2; bb++)
#pragma unroll
            for (int a = 0; a < 2; a++)
                acc += resid_cell<T, CELL>(d, x, b, C, inv_h2, 2 * I + a, 2 * J + bb, 2 * K + c);
    return T(0.125) * acc;
}

}  // namespace mp
