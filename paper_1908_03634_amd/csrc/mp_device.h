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

#pragma clang fp contract(off)

namespace mp {

constexpr int kWave = 64;

struct Dims {
    int nx, ny, nz;
    int px, py, pz;  // 1 = periodic axis, 0 = Neumann walls
    __host__ __device__ long long n() const { return (long long)nx * ny * nz; }
};

// Neighbour offsets and high-face coefficients of cell (i,j,k) at linear index q.
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

// Block sum in a fixed order; every thread receives the same value.
// `sh` must hold blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; q++) s += sh[q];
    return s;
}

}  // namespace mp
