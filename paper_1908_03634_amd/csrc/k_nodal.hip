// k_nodal.hip -- nodal projection kernels (Sec. 3.2 Step 11, Appendix A).
//
// phi lives on the grid nodes, the velocity U and sigma = beta0/rho at cell
// centres.  The discretisation is trilinear finite elements on the cells (the
// paper defers it to an earlier paper): with the hat function N_n of node n,
//   (A phi)_n = h^-3 sum_e sigma_e int_e grad phi_h . grad N_n   (A = -M, SPD)
// For a cube cell the element matrix couples a node to the three corners
// across a face of the cell (two axes differ) and the far corner (three
// differ) with weight -h/12 each, to itself with h/3, and not at all to the
// three corners along an edge.  So, with S_e the sum of phi over those four
// corners of cell e,
//   (A phi)_n = (1/(12 h^2)) sum_e sigma_e (4 phi_n - S_e),
// a 21-point stencil in which nodes of equal (i mod 2, j mod 2) never couple:
// Gauss-Seidel runs in four colours.
//   divergence of a cell field V:  (D V)_n = -(1/(4h)) sum_e sum_d s_d V_e,d
//   cell-average gradient:         (G phi)_e,d = (1/(4h)) sum_B s_d(B) phi_B
//   load of a cell field f:        (L f)_n = (1/8) sum_e f_e
// where s_d = +1 when the node (corner B) is on the high side of the cell
// along d and -1 otherwise.
//
// Nodes: n per periodic axis (node n is node 0), n + 1 per axis with Neumann
// walls; wall nodes are unknowns whose equations take only the cells inside.
// Layout [mz][my][mx], x fastest; cells [nz][ny][nx].
#include "mp_device.h"
#include "mp_kernels.h"
#include "mp_launch.h"

namespace mp {

namespace {

// Node neighbours along one axis (offsets -1, 0, +1) and the cells below and
// above the node (offsets -1, 0).  Missing ones (beyond a wall) are flagged
// and point at the node itself / cell 0 so every load stays in bounds.
struct Axis {
    int nd[3];
    bool nok[3];
    int ce[2];
    bool cok[2];
};

__device__ __forceinline__ Axis axis_of(int i, int n, int per)
{
    Axis a;
#pragma unroll
    for (int o = 0; o < 3; o++) {
        int t = i + o - 1;
        if (per) {
            t = t < 0 ? t + n : (t >= n ? t - n : t);
            a.nd[o] = t;
            a.nok[o] = true;
        } else {
            a.nok[o] = t >= 0 && t <= n;
            a.nd[o] = a.nok[o] ? t : i;
        }
    }
#pragma unroll
    for (int o = 0; o < 2; o++) {
        int t = i + o - 1;
        if (per) {
            t = t < 0 ? t + n : t;
            a.ce[o] = t;
            a.cok[o] = true;
        } else {
            a.cok[o] = t >= 0 && t < n;
            a.ce[o] = a.cok[o] ? t : 0;
        }
    }
    return a;
}

// Sums of the stencil at node (i,j,k) in precision T (fixed order: cells by
// z, y, x offset; in each cell the three face-diagonal corners, then the far
// corner).
template <typename T>
__device__ __forceinline__ void node_sums(const NDims& d, const T* __restrict__ x, const T* __restrict__ sg, int i,
                                          int j, int k, T& ssig, T& ss)
{
    const Axis ax = axis_of(i, d.nx, d.px), ay = axis_of(j, d.ny, d.py), az = axis_of(k, d.nz, d.pz);
    const long long sy = d.mx, sz = (long long)d.mx * d.my;
    T v[3][3][3];
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const int dist = (a != 1) + (b != 1) + (c != 1);
                if (dist >= 2) {
                    const bool ok = ax.nok[a] && ay.nok[b] && az.nok[c];
                    v[c][b][a] = ok ? x[az.nd[c] * sz + ay.nd[b] * sy + ax.nd[a]] : T(0);
                } else {
                    v[c][b][a] = T(0);
                }
            }
    const long long cy = d.nx, cz = (long long)d.nx * d.ny;
    T s1 = T(0), s2 = T(0);
#pragma unroll
    for (int oz = 0; oz < 2; oz++)
#pragma unroll
        for (int oy = 0; oy < 2; oy++)
#pragma unroll
            for (int ox = 0; ox < 2; ox++) {
                const bool ok = ax.cok[ox] && ay.cok[oy] && az.cok[oz];
                const T se = ok ? sg[az.ce[oz] * cz + ay.ce[oy] * cy + ax.ce[ox]] : T(0);
                // the cell lies on side ox (0 = below, 1 = above) of the node;
                // its other corners are at node offsets 2*ox (i.e. -1 or +1)
                const int a = ox * 2, b = oy * 2, c = oz * 2;
                const T sum = ((v[1][b][a] + v[c][1][a]) + v[c][b][1]) + v[c][b][a];
                s1 += se;
                s2 = fma(se, sum, s2);
            }
    ssig = s1;
    ss = s2;
}

__device__ __forceinline__ long long node_index(const NDims& d, int i, int j, int k)
{
    return ((long long)k * d.my + j) * d.mx + i;
}

}  // namespace

// ------------------------------------------------------------- smoother

// One colour of the four-colour Gauss-Seidel sweep on A x = b:
//   x_n = (sum_e sigma_e S_e + 12 h^2 b_n) / (4 sum_e sigma_e)
// for the nodes with (i mod 2, j mod 2) = (colour & 1, colour >> 1).
template <typename T>
__global__ __launch_bounds__(256) void k_nd_gs(NDims d, T* __restrict__ x, const T* __restrict__ b,
                                               const T* __restrict__ sg, T h12, int colour)
{
    const int i = 2 * (blockIdx.x * blockDim.x + threadIdx.x) + (colour & 1);
    const int j = 2 * (blockIdx.y * blockDim.y + threadIdx.y) + (colour >> 1);
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= d.mx || j >= d.my || k >= d.mz) return;
    T ssig, ss;
    node_sums<T>(d, x, sg, i, j, k, ssig, ss);
    const long long q = node_index(d, i, j, k);
    x[q] = (ss + h12 * b[q]) / (T(4) * ssig);
}

template <typename T>
void launch_nd_gs(const NDims& d, T* x, const T* b, const T* sg, T h12, int colour, hipStream_t s)
{
    const int ni = (d.mx - (colour & 1) + 1) / 2, nj = (d.my - (colour >> 1) + 1) / 2;
    const Shape3 sh = cells3(ni, nj, d.mz);
    hipLaunchKernelGGL((k_nd_gs<T>), sh.grid, sh.block, 0, s, d, x, b, sg, h12, colour);
}

// r = b - A x on every node.
template <typename T>
__global__ __launch_bounds__(256) void k_nd_resid(NDims d, const T* __restrict__ x, const T* __restrict__ b,
                                                  const T* __restrict__ sg, T inv_h12, T* __restrict__ r)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= d.mx || j >= d.my || k >= d.mz) return;
    T ssig, ss;
    node_sums<T>(d, x, sg, i, j, k, ssig, ss);
    const long long q = node_index(d, i, j, k);
    r[q] = b[q] - (T(4) * ssig * x[q] - ss) * inv_h12;
}

template <typename T>
void launch_nd_resid(const NDims& d, const T* x, const T* b, const T* sg, T inv_h12, T* r, hipStream_t s)
{
    const Shape3 sh = cells3(d.mx, d.my, d.mz);
    hipLaunchKernelGGL((k_nd_resid<T>), sh.grid, sh.block, 0, s, d, x, b, sg, inv_h12, r);
}

// ------------------------------------------------------------- z-marching

// The same stencil evaluated by threads that each walk one node column (i, j)
// through lz planes: the 3 x 3 neighbour columns of planes k-1, k, k+1 and the
// 2 x 2 cell columns below and above stay in registers, so each node costs
// one new plane of 8 neighbour values and 4 sigma values instead of 20 + 8
// loads.  Same arithmetic in the same order as node_sums (bitwise equal).
//   ND_GS:      one Gauss-Seidel colour (columns of that i, j parity);
//   ND_RESID:   r = b - A x on every node;
//   ND_RESID64: the same in FP64, r32 = float(r * inv_s) and per-block
//               partial sums of r^2.
enum { ND_GS = 0, ND_RESID = 1, ND_RESID64 = 2 };

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_nd_col(NDims d, int lz, T* __restrict__ x, const T* __restrict__ b,
                                                const T* __restrict__ sg, T h12, T inv_h12, int colour,
                                                T* __restrict__ r, float* __restrict__ r32,
                                                const double* __restrict__ inv_s, double* part)
{
    const int ti = blockIdx.x * blockDim.x + threadIdx.x;
    const int tj = blockIdx.y * blockDim.y + threadIdx.y;
    const int i = MODE == ND_GS ? 2 * ti + (colour & 1) : ti;
    const int j = MODE == ND_GS ? 2 * tj + (colour >> 1) : tj;
    const int k0 = blockIdx.z * lz;
    const int k1 = min(k0 + lz, d.mz);
    double acc = 0.0;
    if (i < d.mx && j < d.my) {
        const Axis ax = axis_of(i, d.nx, d.px), ay = axis_of(j, d.ny, d.py);
        const long long sy = d.mx, sz = (long long)d.mx * d.my;
        const long long cy = d.nx, cz = (long long)d.nx * d.ny;
        long long col[3][3];
        bool cok[3][3];
#pragma unroll
        for (int bb = 0; bb < 3; bb++)
#pragma unroll
            for (int aa = 0; aa < 3; aa++) {
                col[bb][aa] = ay.nd[bb] * sy + ax.nd[aa];
                cok[bb][aa] = ax.nok[aa] && ay.nok[bb];
            }
        long long ccol[2][2];
        bool ccok[2][2];
#pragma unroll
        for (int oy = 0; oy < 2; oy++)
#pragma unroll
            for (int ox = 0; ox < 2; ox++) {
                ccol[oy][ox] = ay.ce[oy] * cy + ax.ce[ox];
                ccok[oy][ox] = ax.cok[ox] && ay.cok[oy];
            }
        // node plane kk (may be -1 or mz: wrapped when periodic, absent at a wall)
        auto ld_plane = [&](int kk, T (&v)[3][3]) {
            bool okz = true;
            if (d.pz) kk = kk < 0 ? kk + d.nz : (kk >= d.nz ? kk - d.nz : kk);
            else okz = kk >= 0 && kk <= d.nz;
#pragma unroll
            for (int bb = 0; bb < 3; bb++)
#pragma unroll
                for (int aa = 0; aa < 3; aa++) {
                    const bool need = MODE == ND_GS ? !(aa == 1 && bb == 1) : true;
                    v[bb][aa] = (need && okz && cok[bb][aa]) ? x[(long long)kk * sz + col[bb][aa]] : T(0);
                }
        };
        // cell plane kc (below node k: k-1; above: k)
        auto ld_cells = [&](int kc, T (&s)[2][2]) {
            bool okz = true;
            if (d.pz) kc = kc < 0 ? kc + d.nz : kc;
            else okz = kc >= 0 && kc < d.nz;
#pragma unroll
            for (int oy = 0; oy < 2; oy++)
#pragma unroll
                for (int ox = 0; ox < 2; ox++)
                    s[oy][ox] = (okz && ccok[oy][ox]) ? sg[(long long)(okz ? kc : 0) * cz + ccol[oy][ox]] : T(0);
        };
        T v0[3][3], v1[3][3], v2[3][3], s0[2][2], s1[2][2];
        ld_plane(k0 - 1, v0);
        ld_plane(k0, v1);
        ld_cells(k0 - 1, s0);
        const double is = MODE == ND_RESID64 ? inv_s[0] : 0.0;
        for (int k = k0; k < k1; k++) {
            ld_plane(k + 1, v2);
            ld_cells(k, s1);
            const long long q = (long long)k * sz + (long long)j * sy + i;
            T a1 = T(0), a2 = T(0);
#pragma unroll
            for (int oz = 0; oz < 2; oz++)
#pragma unroll
                for (int oy = 0; oy < 2; oy++)
#pragma unroll
                    for (int ox = 0; ox < 2; ox++) {
                        const T se = oz ? s1[oy][ox] : s0[oy][ox];
                        const int aa = ox * 2, bb = oy * 2;
                        const T(&vc)[3][3] = oz ? v2 : v0;
                        const T sum = ((v1[bb][aa] + vc[1][aa]) + vc[bb][1]) + vc[bb][aa];
                        a1 += se;
                        a2 = fma(se, sum, a2);
                    }
            if constexpr (MODE == ND_GS) {
                x[q] = (a2 + h12 * b[q]) / (T(4) * a1);
            } else {
                const T rv = b[q] - (T(4) * a1 * v1[1][1] - a2) * inv_h12;
                if constexpr (MODE == ND_RESID) {
                    r[q] = rv;
                } else {
                    if (r32) r32[q] = (float)((double)rv * is);
                    acc = fma((double)rv, (double)rv, acc);
                }
            }
#pragma unroll
            for (int bb = 0; bb < 3; bb++)
#pragma unroll
                for (int aa = 0; aa < 3; aa++) {
                    v0[bb][aa] = v1[bb][aa];
                    v1[bb][aa] = v2[bb][aa];
                }
#pragma unroll
            for (int oy = 0; oy < 2; oy++)
#pragma unroll
                for (int ox = 0; ox < 2; ox++) s0[oy][ox] = s1[oy][ox];
        }
    }
    if constexpr (MODE == ND_RESID64) {
        __shared__ double sh[kBlock / kWave];
        const double sblk = block_sum(acc, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0)
            part[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = sblk;
    }
}

// The nodal right-hand side b = L(beta0 S - m) - D(beta0 U) (or, with
// squares, its sum of squares alone) by threads that walk node columns: the
// 2 x 2 cell columns around the column keep the cell plane below the node in
// registers, so each node loads one new plane of 4 cells.  Same operands in
// the same order as k_nd_rhs (bitwise equal); per-block partial sums.
__global__ __launch_bounds__(256) void k_nd_rhs_col(NDims d, int lz, double inv4h, const double* __restrict__ beta0,
                                                    const double* __restrict__ ux, const double* __restrict__ uy,
                                                    const double* __restrict__ uz, const double* __restrict__ S,
                                                    const double* __restrict__ mean, double* __restrict__ out,
                                                    int squares, double* part)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k0 = blockIdx.z * lz;
    const int k1 = min(k0 + lz, d.mz);
    double acc = 0.0;
    if (i < d.mx && j < d.my) {
        const double m = mean[0];
        const Axis ax = axis_of(i, d.nx, d.px), ay = axis_of(j, d.ny, d.py);
        const long long cy = d.nx, cz = (long long)d.nx * d.ny;
        long long ccol[2][2];
        bool ccok[2][2];
#pragma unroll
        for (int oy = 0; oy < 2; oy++)
#pragma unroll
            for (int ox = 0; ox < 2; ox++) {
                ccol[oy][ox] = ay.ce[oy] * cy + ax.ce[ox];
                ccok[oy][ox] = ax.cok[ox] && ay.cok[oy];
            }
        // the five cell fields of the 2 x 2 columns in cell plane kc
        struct CP {
            double b0[2][2], s[2][2], u[2][2], v[2][2], w[2][2];
            bool ok;
        };
        auto ld = [&](int kc, CP& c) {
            bool okz = true;
            if (d.pz) kc = kc < 0 ? kc + d.nz : kc;
            else okz = kc >= 0 && kc < d.nz;
            c.ok = okz;
#pragma unroll
            for (int oy = 0; oy < 2; oy++)
#pragma unroll
                for (int ox = 0; ox < 2; ox++) {
                    const bool ok = okz && ccok[oy][ox];
                    const long long e = (long long)(okz ? kc : 0) * cz + ccol[oy][ox];
                    c.b0[oy][ox] = ok ? beta0[e] : 0.0;
                    c.s[oy][ox] = ok ? S[e] : 0.0;
                    c.u[oy][ox] = ok ? ux[e] : 0.0;
                    c.v[oy][ox] = ok ? uy[e] : 0.0;
                    c.w[oy][ox] = ok ? uz[e] : 0.0;
                }
        };
        CP lo, hi;
        ld(k0 - 1, lo);
        for (int k = k0; k < k1; k++) {
            ld(k, hi);
            double src = 0.0, div = 0.0;
#pragma unroll
            for (int oz = 0; oz < 2; oz++) {
                const CP& c = oz ? hi : lo;
#pragma unroll
                for (int oy = 0; oy < 2; oy++)
#pragma unroll
                    for (int ox = 0; ox < 2; ox++) {
                        if (!(c.ok && ccok[oy][ox])) continue;
                        const double b0 = c.b0[oy][ox];
                        src += fma(b0, c.s[oy][ox], -m);
                        const double vx = b0 * c.u[oy][ox], vy = b0 * c.v[oy][ox], vz = b0 * c.w[oy][ox];
                        div += (ox ? -vx : vx) + (oy ? -vy : vy) + (oz ? -vz : vz);
                    }
            }
            const double bn = 0.125 * src + inv4h * div;
            if (out) out[((long long)k * d.my + j) * d.mx + i] = bn;
            acc = squares ? fma(bn, bn, acc) : acc + bn;
            lo = hi;
        }
    }
    __shared__ double sh[kBlock / kWave];
    const double sblk = block_sum(acc, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        part[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = sblk;
}

namespace {

// Columns (ni x nj) in 64 x 4 blocks, planes in chunks of lz: the largest lz
// (<= 16) that still gives at least min_blocks blocks, then doubled while
// the count exceeds max_blocks.
struct ColShape {
    dim3 grid, block;
    int lz;
};

ColShape col_shape(int ni, int nj, int mz, long long min_blocks, long long max_blocks)
{
    ColShape c;
    c.block = dim3(64, 4, 1);
    const long long bxy = (long long)((ni + 63) / 64) * ((nj + 3) / 4);
    int lz = 16;
    while (lz > 2 && bxy * ((mz + lz - 1) / lz) < min_blocks) lz /= 2;
    while (bxy * ((mz + lz - 1) / lz) > max_blocks && lz < mz) lz *= 2;
    c.lz = lz;
    c.grid = dim3((ni + 63) / 64, (nj + 3) / 4, (mz + lz - 1) / lz);
    return c;
}

}  // namespace

bool nd_col_supported(const NDims& d) { return d.mz >= 2; }

int nd_col_reduce_blocks(const NDims& d)
{
    const ColShape c = col_shape(d.mx, d.my, d.mz, 1024, kMaxRedBlocks);
    return (int)(c.grid.x * c.grid.y * c.grid.z);
}

template <typename T>
void launch_nd_gs_col(const NDims& d, T* x, const T* b, const T* sg, T h12, int colour, hipStream_t s)
{
    const int ni = (d.mx - (colour & 1) + 1) / 2, nj = (d.my - (colour >> 1) + 1) / 2;
    const ColShape c = col_shape(ni, nj, d.mz, 2048, 1LL << 30);
    hipLaunchKernelGGL((k_nd_col<T, ND_GS>), c.grid, c.block, 0, s, d, c.lz, x, b, sg, h12, T(0), colour,
                       (T*)nullptr, (float*)nullptr, (const double*)nullptr, (double*)nullptr);
}

template <typename T>
void launch_nd_resid_col(const NDims& d, const T* x, const T* b, const T* sg, T inv_h12, T* r, hipStream_t s)
{
    const ColShape c = col_shape(d.mx, d.my, d.mz, 2048, 1LL << 30);
    hipLaunchKernelGGL((k_nd_col<T, ND_RESID>), c.grid, c.block, 0, s, d, c.lz, const_cast<T*>(x), b, sg, T(0),
                       inv_h12, 0, r, (float*)nullptr, (const double*)nullptr, (double*)nullptr);
}

void launch_nd_resid64_col(const NDims& d, const double* x, const double* b, const double* sg, double inv_h12,
                           float* r32, const double* inv_s, double* partials, int* nb_out, hipStream_t s)
{
    const ColShape c = col_shape(d.mx, d.my, d.mz, 1024, kMaxRedBlocks);
    *nb_out = (int)(c.grid.x * c.grid.y * c.grid.z);
    hipLaunchKernelGGL((k_nd_col<double, ND_RESID64>), c.grid, c.block, 0, s, d, c.lz, const_cast<double*>(x), b,
                       sg, 0.0, inv_h12, 0, (double*)nullptr, r32, inv_s, partials);
}

void launch_nd_rhs_col(const NDims& d, double inv4h, const double* beta0, const double* ux, const double* uy,
                       const double* uz, const double* S, const double* mean, double* out, int squares,
                       double* partials, int* nb_out, hipStream_t s)
{
    const ColShape c = col_shape(d.mx, d.my, d.mz, 1024, kMaxRedBlocks);
    *nb_out = (int)(c.grid.x * c.grid.y * c.grid.z);
    hipLaunchKernelGGL(k_nd_rhs_col, c.grid, c.block, 0, s, d, c.lz, inv4h, beta0, ux, uy, uz, S, mean, out, squares,
                       partials);
}

template void launch_nd_gs_col<float>(const NDims&, float*, const float*, const float*, float, int, hipStream_t);
template void launch_nd_gs_col<double>(const NDims&, double*, const double*, const double*, double, int,
                                       hipStream_t);
template void launch_nd_resid_col<float>(const NDims&, const float*, const float*, const float*, float, float*,
                                         hipStream_t);
template void launch_nd_resid_col<double>(const NDims&, const double*, const double*, const double*, double,
                                          double*, hipStream_t);

// ------------------------------------------------------------- transfers

// Coarse right-hand side = (1/8) P^T r at coarse node (I, J, K): the fine
// nodes 2I-1, 2I, 2I+1 per axis with weights 1/2, 1, 1/2 (wrapped when
// periodic, dropped beyond a wall).
template <typename T>
__device__ __forceinline__ T nd_restrict_node(const NDims& f, const T* __restrict__ rf, int I, int J, int K)
{
    const Axis ax = axis_of(2 * I, f.nx, f.px), ay = axis_of(2 * J, f.ny, f.py), az = axis_of(2 * K, f.nz, f.pz);
    const long long sy = f.mx, sz = (long long)f.mx * f.my;
    T acc = T(0);
#pragma unroll
    for (int cc = 0; cc < 3; cc++) {
        T row = T(0);
#pragma unroll
        for (int bb = 0; bb < 3; bb++) {
            T line = T(0);
#pragma unroll
            for (int aa = 0; aa < 3; aa++) {
                const bool ok = ax.nok[aa] && ay.nok[bb] && az.nok[cc];
                const T v = ok ? rf[az.nd[cc] * sz + ay.nd[bb] * sy + ax.nd[aa]] : T(0);
                line += aa == 1 ? v : T(0.5) * v;
            }
            row += bb == 1 ? line : T(0.5) * line;
        }
        acc += cc == 1 ? row : T(0.5) * row;
    }
    return T(0.125) * acc;
}

// P e_c at fine node (i, j, k), trilinear: an even fine index takes coarse
// node i/2, an odd one the mean of coarse nodes (i-1)/2 and (i+1)/2 (wrapped
// when periodic).
template <typename T>
__device__ __forceinline__ T nd_prolong_node(const NDims& c, const T* __restrict__ ec, int i, int j, int k)
{
    int I[2], J[2], K[2];
    I[0] = i >> 1;
    I[1] = (i & 1) ? ((i + 1) >> 1 == c.mx ? 0 : (i + 1) >> 1) : I[0];
    J[0] = j >> 1;
    J[1] = (j & 1) ? ((j + 1) >> 1 == c.my ? 0 : (j + 1) >> 1) : J[0];
    K[0] = k >> 1;
    K[1] = (k & 1) ? ((k + 1) >> 1 == c.mz ? 0 : (k + 1) >> 1) : K[0];
    const long long sy = c.mx, sz = (long long)c.mx * c.my;
    T acc = T(0);
#pragma unroll
    for (int cc = 0; cc < 2; cc++) {
        T row = T(0);
#pragma unroll
        for (int bb = 0; bb < 2; bb++) {
            const T l = ec[K[cc] * sz + J[bb] * sy + I[0]] + ec[K[cc] * sz + J[bb] * sy + I[1]];
            row += l;
        }
        acc += row;
    }
    return T(0.125) * acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_nd_restrict(NDims f, NDims c, const T* __restrict__ rf, T* __restrict__ bc)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= c.mx || J >= c.my || K >= c.mz) return;
    bc[((long long)K * c.my + J) * c.mx + I] = nd_restrict_node<T>(f, rf, I, J, K);
}

template <typename T>
void launch_nd_restrict(const NDims& f, const NDims& c, const T* rf, T* bc, hipStream_t s)
{
    const Shape3 sh = cells3(c.mx, c.my, c.mz);
    hipLaunchKernelGGL((k_nd_restrict<T>), sh.grid, sh.block, 0, s, f, c, rf, bc);
}

// x_f += P e_c.
template <typename T>
__global__ __launch_bounds__(256) void k_nd_prolong(NDims f, NDims c, T* __restrict__ xf, const T* __restrict__ ec)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= f.mx || j >= f.my || k >= f.mz) return;
    xf[((long long)k * f.my + j) * f.mx + i] += nd_prolong_node<T>(c, ec, i, j, k);
}

// x_f += P e_c for a column of fine nodes per thread: the sum over the two
// coarse rows of a coarse plane (the inner two loops of nd_prolong_node) is
// formed once per coarse plane and serves the two or three fine planes that
// read it; each node then adds the sums of its planes in the order of
// nd_prolong_node (bitwise equal).
template <typename T>
__global__ __launch_bounds__(256) void k_nd_prolong_col(NDims f, NDims c, int lz, T* __restrict__ xf,
                                                        const T* __restrict__ ec)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k0 = blockIdx.z * lz;
    const int k1 = min(k0 + lz, f.mz);
    if (i >= f.mx || j >= f.my) return;
    const int I0 = i >> 1, I1 = (i & 1) ? ((i + 1) >> 1 == c.mx ? 0 : (i + 1) >> 1) : I0;
    const int J0 = j >> 1, J1 = (j & 1) ? ((j + 1) >> 1 == c.my ? 0 : (j + 1) >> 1) : J0;
    const long long sy = c.mx, sz = (long long)c.mx * c.my;
    auto plane_sum = [&](int K) {
        T row = T(0);
        row += ec[K * sz + J0 * sy + I0] + ec[K * sz + J0 * sy + I1];
        row += ec[K * sz + J1 * sy + I0] + ec[K * sz + J1 * sy + I1];
        return row;
    };
    int kc = -1;  // coarse plane whose sum is held in rc
    T rc = T(0);
    auto sum_of = [&](int K) {
        if (K != kc) {
            rc = plane_sum(K);
            kc = K;
        }
        return rc;
    };
    const long long fsy = f.mx, fsz = (long long)f.mx * f.my;
    for (int k = k0; k < k1; k++) {
        const int K0 = k >> 1, K1 = (k & 1) ? ((k + 1) >> 1 == c.mz ? 0 : (k + 1) >> 1) : K0;
        T acc = T(0);
        acc += sum_of(K0);
        acc += sum_of(K1);
        const long long q = k * fsz + j * fsy + i;
        xf[q] += T(0.125) * acc;
    }
}

template <typename T>
void launch_nd_prolong(const NDims& f, const NDims& c, T* xf, const T* ec, int col, hipStream_t s)
{
    if (col && f.mz >= 2) {
        const ColShape cs = col_shape(f.mx, f.my, f.mz, 1024, 1LL << 30);
        hipLaunchKernelGGL((k_nd_prolong_col<T>), cs.grid, cs.block, 0, s, f, c, cs.lz, xf, ec);
        return;
    }
    const Shape3 sh = cells3(f.mx, f.my, f.mz);
    hipLaunchKernelGGL((k_nd_prolong<T>), sh.grid, sh.block, 0, s, f, c, xf, ec);
}

// Coarse cell sigma = mean of its 8 children; with fine == coarse shape
// (same dims) it is a plain precision conversion.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_nd_sigma(int nx, int ny, int nz, const Tin* __restrict__ sf,
                                                  Tout* __restrict__ sc, int coarsen)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    const int NX = coarsen ? nx / 2 : nx, NY = coarsen ? ny / 2 : ny, NZ = coarsen ? nz / 2 : nz;
    if (I >= NX || J >= NY || K >= NZ) return;
    const long long qc = ((long long)K * NY + J) * NX + I;
    if (!coarsen) {
        sc[qc] = (Tout)sf[qc];
        return;
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int a = 0; a < 2; a++) s += (double)sf[((long long)(2 * K + c) * ny + 2 * J + b) * nx + 2 * I + a];
    sc[qc] = (Tout)(0.125 * s);
}

template <typename Tin, typename Tout>
void launch_nd_sigma(int nx, int ny, int nz, const Tin* sf, Tout* sc, int coarsen, hipStream_t s)
{
    const Shape3 sh = coarsen ? cells3(nx / 2, ny / 2, nz / 2) : cells3(nx, ny, nz);
    hipLaunchKernelGGL((k_nd_sigma<Tin, Tout>), sh.grid, sh.block, 0, s, nx, ny, nz, sf, sc, coarsen);
}

// ------------------------------------------------------------- FP64 level 0

__device__ __forceinline__ void node_ijk(const NDims& d, long long q, int& i, int& j, int& k)
{
    const long long t = q / d.mx;
    i = (int)(q - t * d.mx);
    k = (int)(t / d.my);
    j = (int)(t - (long long)k * d.my);
}

// partials[block] = sum over the cells of beta0 * S (grid-stride).
__global__ __launch_bounds__(kBlock) void k_nd_src_sum(long long n, const double* __restrict__ beta0,
                                                       const double* __restrict__ S, double* part)
{
    __shared__ double sh[kBlock / kWave];
    double v = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        v = fma(beta0[q], S[q], v);
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_nd_src_sum(long long n, const double* beta0, const double* S, double* partials, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_nd_src_sum, dim3(nb), dim3(kBlock), 0, s, n, beta0, S, partials);
}

// b_n = L(beta0 S - m)_n - D(beta0 U)_n  (= minus the nodal right-hand side),
//     = sum_e [ (beta0_e S_e - m) / 8 + (1/(4h)) sum_d s_d beta0_e U_e,d ].
// out != nullptr: written; partials[block] = sum of b_n^2 (squares) or of b_n
// (grid-stride).
__global__ __launch_bounds__(kBlock) void k_nd_rhs(NDims d, double inv4h, const double* __restrict__ beta0,
                                                   const double* __restrict__ ux, const double* __restrict__ uy,
                                                   const double* __restrict__ uz, const double* __restrict__ S,
                                                   const double* __restrict__ mean, double* __restrict__ out,
                                                   int squares, double* part)
{
    __shared__ double sh[kBlock / kWave];
    const long long nn = (long long)d.mx * d.my * d.mz;
    const double m = mean[0];
    const long long cy = d.nx, cz = (long long)d.nx * d.ny;
    double acc = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nn;
         q += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(d, q, i, j, k);
        const Axis ax = axis_of(i, d.nx, d.px), ay = axis_of(j, d.ny, d.py), az = axis_of(k, d.nz, d.pz);
        double src = 0.0, div = 0.0;
        for (int oz = 0; oz < 2; oz++)
            for (int oy = 0; oy < 2; oy++)
                for (int ox = 0; ox < 2; ox++) {
                    if (!(ax.cok[ox] && ay.cok[oy] && az.cok[oz])) continue;
                    const long long e = az.ce[oz] * cz + ay.ce[oy] * cy + ax.ce[ox];
                    const double b0 = beta0[e];
                    src += fma(b0, S[e], -m);
                    // the node is the high corner of the cell below it (o = 0)
                    const double vx = b0 * ux[e], vy = b0 * uy[e], vz = b0 * uz[e];
                    div += (ox ? -vx : vx) + (oy ? -vy : vy) + (oz ? -vz : vz);
                }
        const double bn = 0.125 * src + inv4h * div;
        if (out) out[q] = bn;
        acc = squares ? fma(bn, bn, acc) : acc + bn;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_nd_rhs(const NDims& d, double inv4h, const double* beta0, const double* ux, const double* uy,
                   const double* uz, const double* S, const double* mean, double* out, int squares,
                   double* partials, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_nd_rhs, dim3(nb), dim3(kBlock), 0, s, d, inv4h, beta0, ux, uy, uz, S, mean, out, squares,
                       partials);
}

// r = b - A x in FP64; r32 = float(r * inv_s[0]) when r32 != nullptr;
// partials[block] = sum r^2 (grid-stride).
__global__ __launch_bounds__(kBlock) void k_nd_resid64(NDims d, const double* __restrict__ x,
                                                       const double* __restrict__ b, const double* __restrict__ sg,
                                                       double inv_h12, float* __restrict__ r32,
                                                       const double* __restrict__ inv_s, double* part)
{
    __shared__ double sh[kBlock / kWave];
    const long long nn = (long long)d.mx * d.my * d.mz;
    const double is = r32 ? inv_s[0] : 0.0;
    double acc = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nn;
         q += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(d, q, i, j, k);
        double ssig, ss;
        node_sums<double>(d, x, sg, i, j, k, ssig, ss);
        const double r = b[q] - (4.0 * ssig * x[q] - ss) * inv_h12;
        if (r32) r32[q] = (float)(r * is);
        acc = fma(r, r, acc);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_nd_resid64(const NDims& d, const double* x, const double* b, const double* sg, double inv_h12,
                       float* r32, const double* inv_s, double* partials, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_nd_resid64, dim3(nb), dim3(kBlock), 0, s, d, x, b, sg, inv_h12, r32, inv_s, partials);
}

// y = M x = -(A x) on every node, FP64.
__global__ __launch_bounds__(256) void k_nd_apply64(NDims d, const double* __restrict__ x,
                                                    const double* __restrict__ sg, double inv_h12,
                                                    double* __restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= d.mx || j >= d.my || k >= d.mz) return;
    double ssig, ss;
    node_sums<double>(d, x, sg, i, j, k, ssig, ss);
    const long long q = node_index(d, i, j, k);
    y[q] = (ss - 4.0 * ssig * x[q]) * inv_h12;
}

void launch_nd_apply64(const NDims& d, const double* x, const double* sg, double inv_h12, double* y, hipStream_t s)
{
    const Shape3 sh = cells3(d.mx, d.my, d.mz);
    hipLaunchKernelGGL(k_nd_apply64, sh.grid, sh.block, 0, s, d, x, sg, inv_h12, y);
}

// U_e -= (sigma_e / beta0_e) (G phi)_e with (G phi)_e,d = (1/(4h)) sum_B s_d(B) phi_B.
__global__ __launch_bounds__(256) void k_nd_correct(NDims d, double inv4h, const double* __restrict__ sg,
                                                    const double* __restrict__ beta0, const double* __restrict__ phi,
                                                    double* __restrict__ ux, double* __restrict__ uy,
                                                    double* __restrict__ uz)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= d.nx || j >= d.ny || k >= d.nz) return;
    const int i1 = i + 1 == d.mx ? 0 : i + 1;  // periodic: node nx is node 0
    const int j1 = j + 1 == d.my ? 0 : j + 1;
    const int k1 = k + 1 == d.mz ? 0 : k + 1;
    const long long sy = d.mx, sz = (long long)d.mx * d.my;
    const double p000 = phi[k * sz + j * sy + i], p001 = phi[k * sz + j * sy + i1];
    const double p010 = phi[k * sz + j1 * sy + i], p011 = phi[k * sz + j1 * sy + i1];
    const double p100 = phi[k1 * sz + j * sy + i], p101 = phi[k1 * sz + j * sy + i1];
    const double p110 = phi[k1 * sz + j1 * sy + i], p111 = phi[k1 * sz + j1 * sy + i1];
    const double gx = ((p001 - p000) + (p011 - p010) + (p101 - p100) + (p111 - p110)) * inv4h;
    const double gy = ((p010 - p000) + (p011 - p001) + (p110 - p100) + (p111 - p101)) * inv4h;
    const double gz = ((p100 - p000) + (p101 - p001) + (p110 - p010) + (p111 - p011)) * inv4h;
    const long long e = ((long long)k * d.ny + j) * d.nx + i;
    const double w = sg[e] / beta0[e];
    ux[e] -= w * gx;
    uy[e] -= w * gy;
    uz[e] -= w * gz;
}

void launch_nd_correct(const NDims& d, double inv4h, const double* sg, const double* beta0, const double* phi,
                       double* ux, double* uy, double* uz, hipStream_t s)
{
    const Shape3 sh = cells3(d.nx, d.ny, d.nz);
    hipLaunchKernelGGL(k_nd_correct, sh.grid, sh.block, 0, s, d, inv4h, sg, beta0, phi, ux, uy, uz);
}

// ------------------------------------------------------------- bottom solve

// Conjugate gradients in FP64 on the coarsest node grid, one workgroup:
// b is made mean-zero (constants are the null space) and the residual is kept
// mean-zero; x starts at zero, or at the x passed in when use_x0 (the
// tolerance is then relative to the initial residual), and is returned
// mean-zero.  Stops at ||r|| <= rtol ||r0|| or maxit.  work holds 4 n doubles.
// WAVE: run by the first wavefront alone (n <= 64), synchronised within it
// (the other wavefronts of the workgroup wait at a later barrier); a sum is
// lane 0's wavefront sum either way, so both forms give the same bits.
template <typename T, bool WAVE = false>
__device__ void nd_block_cg(const NDims& d, const T* __restrict__ bin, T* __restrict__ xout, const T* __restrict__ sg,
                            double inv_h12, double rtol, int maxit, int use_x0, double* __restrict__ work, double* sh,
                            double* __restrict__ iters = nullptr)
{
    const int n = d.mx * d.my * d.mz;
    const int tid = WAVE ? (int)(threadIdx.x & (kWave - 1)) : (int)threadIdx.x;
    const int nt = WAVE ? kWave : (int)blockDim.x;
    auto sync = [&]() {
        if constexpr (WAVE) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        } else {
            __syncthreads();
        }
    };
    auto total = [&](double v) {
        if constexpr (WAVE) return wave_sum_bcast(v);
        else return block_sum(v, sh);
    };
    double* x = work;
    double* r = work + n;
    double* p = work + 2 * n;
    double* ap = work + 3 * n;
    const long long sy = d.mx, sz = (long long)d.mx * d.my, cy = d.nx, cz = (long long)d.nx * d.ny;
    // out = A y (sigma in T, y in FP64); returns sum of y . out
    auto apply = [&](const double* y, double* out) {
        sync();
        double acc = 0.0;
        for (int q = tid; q < n; q += nt) {
            int i, j, k;
            node_ijk(d, q, i, j, k);
            const Axis ax = axis_of(i, d.nx, d.px), ay = axis_of(j, d.ny, d.py), az = axis_of(k, d.nz, d.pz);
            double ssig = 0.0, ss = 0.0;
            for (int oz = 0; oz < 2; oz++)
                for (int oy = 0; oy < 2; oy++)
                    for (int ox = 0; ox < 2; ox++) {
                        if (!(ax.cok[ox] && ay.cok[oy] && az.cok[oz])) continue;
                        const double se = (double)sg[az.ce[oz] * cz + ay.ce[oy] * cy + ax.ce[ox]];
                        const int a = ox * 2, b = oy * 2, c = oz * 2;
                        const double sum = y[az.nd[1] * sz + ay.nd[b] * sy + ax.nd[a]] +
                                           y[az.nd[c] * sz + ay.nd[1] * sy + ax.nd[a]] +
                                           y[az.nd[c] * sz + ay.nd[b] * sy + ax.nd[1]] +
                                           y[az.nd[c] * sz + ay.nd[b] * sy + ax.nd[a]];
                        ssig += se;
                        ss = fma(se, sum, ss);
                    }
            const double v = (4.0 * ssig * y[q] - ss) * inv_h12;
            out[q] = v;
            acc = fma(y[q], v, acc);
        }
        return total(acc);
    };
    double part = 0.0;
    for (int q = tid; q < n; q += nt) part += (double)bin[q];
    const double mb = total(part) / n;
    for (int q = tid; q < n; q += nt) x[q] = use_x0 ? (double)xout[q] : 0.0;
    if (use_x0) (void)apply(x, ap);
    part = 0.0;
    for (int q = tid; q < n; q += nt) part += ((double)bin[q] - mb) - (use_x0 ? ap[q] : 0.0);
    const double m0 = total(part) / n;
    part = 0.0;
    for (int q = tid; q < n; q += nt) {
        const double rq = ((double)bin[q] - mb) - (use_x0 ? ap[q] : 0.0) - m0;
        r[q] = rq;
        p[q] = rq;
        part = fma(rq, rq, part);
    }
    double rr = total(part);
    const double tol2 = rtol * rtol * rr;
    int it = 0;
    for (; it < maxit && rr > tol2 && rr > 0.0; it++) {
        const double pap = apply(p, ap);
        if (!(pap > 0.0)) break;
        const double alpha = rr / pap;
        part = 0.0;
        for (int q = tid; q < n; q += nt) {
            x[q] = fma(alpha, p[q], x[q]);
            r[q] = fma(-alpha, ap[q], r[q]);
            part += r[q];
        }
        const double mr = total(part) / n;
        part = 0.0;
        for (int q = tid; q < n; q += nt) {
            const double rq = r[q] - mr;
            r[q] = rq;
            part = fma(rq, rq, part);
        }
        const double rr1 = total(part);
        const double beta = rr1 / rr;
        rr = rr1;
        for (int q = tid; q < n; q += nt) p[q] = fma(beta, p[q], r[q]);
    }
    // iterations of this solve added to the caller's running count
    if (iters && tid == 0) iters[0] += (double)it;
    sync();
    part = 0.0;
    for (int q = tid; q < n; q += nt) part += x[q];
    const double mx = total(part) / n;
    for (int q = tid; q < n; q += nt) xout[q] = (T)(x[q] - mx);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_nd_bottom(NDims d, const T* __restrict__ bin, T* __restrict__ xout,
                                                    const T* __restrict__ sg, double inv_h12, double rtol, int maxit,
                                                    int use_x0, double* __restrict__ work, double* __restrict__ iters)
{
    __shared__ double sh[16];
    nd_block_cg<T>(d, bin, xout, sg, inv_h12, rtol, maxit, use_x0, work, sh, iters);
}

template <typename T>
void launch_nd_bottom(const NDims& d, const T* b, T* x, const T* sg, double inv_h12, double rtol, int maxit,
                      int use_x0, double* work, double* iters, hipStream_t s)
{
    const int n = d.mx * d.my * d.mz;
    int nt = ((n + 63) / 64) * 64;
    if (nt > 1024) nt = 1024;
    hipLaunchKernelGGL((k_nd_bottom<T>), dim3(1), dim3(nt), 0, s, d, b, x, sg, inv_h12, rtol, maxit, use_x0, work,
                       iters);
}

// ------------------------------------------------------------- coarse cycle

// The coarse end of a nodal V-cycle in one 1024-thread workgroup with every
// array in LDS: per level the iterate, right-hand side and residual on the
// nodes and sigma on the cells, then the FP64 work of the bottom solve.  The
// per-node arithmetic is that of the one-launch kernels (node_sums,
// nd_restrict_node, nd_prolong_node, nd_block_cg), so both agree bit for bit.
template <typename T>
__device__ __forceinline__ long long nd_lds_off(const NdCoarseArgs<T>& a, int l)
{
    long long off = 0;
    for (int q = 0; q < l; q++) {
        const NDims& d = a.lv[q].d;
        off += 3LL * d.mx * d.my * d.mz + (long long)d.nx * d.ny * d.nz;
    }
    return off;
}

template <typename T>
__device__ __forceinline__ void nd_cc_gs(const NDims& d, T* x, const T* b, const T* sg, T h12, int colour)
{
    const int cx = colour & 1, cy = colour >> 1;
    const int ni = (d.mx - cx + 1) / 2, nj = (d.my - cy + 1) / 2;
    const int cnt = ni * nj * d.mz;
    const FastDiv fi((unsigned)ni), fj((unsigned)nj);
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        int ti, tj, k;
        split3((unsigned)e, fi, fj, ti, tj, k);
        const int i = 2 * ti + cx, j = 2 * tj + cy;
        T ssig, ss;
        node_sums<T>(d, x, sg, i, j, k, ssig, ss);
        const long long q = node_index(d, i, j, k);
        x[q] = (ss + h12 * b[q]) / (T(4) * ssig);
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(1024) void k_nd_coarse(NdCoarseArgs<T> a)
{
    __shared__ T lds[kCoarseLdsBytes / sizeof(T)];
    __shared__ double sh[16];
    const int nl = a.nlev;
    // stage sigma of every level and the right-hand side of the top level;
    // every level starts from zero
    for (int l = 0; l < nl; l++) {
        const NDims& d = a.lv[l].d;
        const int nn = d.mx * d.my * d.mz, nc = d.nx * d.ny * d.nz;
        T* base = lds + nd_lds_off(a, l);
        for (int e = threadIdx.x; e < nn; e += blockDim.x) {
            base[e] = T(0);
            base[nn + e] = l == 0 ? a.lv[0].b[e] : T(0);
        }
        for (int e = threadIdx.x; e < nc; e += blockDim.x) base[3 * nn + e] = a.lv[l].sig[e];
    }
    __syncthreads();
    // down
    for (int l = 0; l < nl - 1; l++) {
        const NDims& d = a.lv[l].d;
        const int nn = d.mx * d.my * d.mz;
        T* x = lds + nd_lds_off(a, l);
        T* b = x + nn;
        T* r = b + nn;
        const T* sg = r + nn;
        for (int s = 0; s < a.nu1; s++)
            for (int colour = 0; colour < 4; colour++) nd_cc_gs<T>(d, x, b, sg, a.lv[l].h12, colour);
        const FastDiv fx((unsigned)d.mx), fy((unsigned)d.my);
        for (int e = threadIdx.x; e < nn; e += blockDim.x) {
            int i, j, k;
            split3((unsigned)e, fx, fy, i, j, k);
            T ssig, ss;
            node_sums<T>(d, x, sg, i, j, k, ssig, ss);
            r[e] = b[e] - (T(4) * ssig * x[e] - ss) * a.lv[l].inv_h12;
        }
        __syncthreads();
        const NDims& c = a.lv[l + 1].d;
        const int nnc = c.mx * c.my * c.mz;
        T* bc = lds + nd_lds_off(a, l + 1) + nnc;
        const FastDiv fxc((unsigned)c.mx), fyc((unsigned)c.my);
        for (int e = threadIdx.x; e < nnc; e += blockDim.x) {
            int I, J, K;
            split3((unsigned)e, fxc, fyc, I, J, K);
            bc[e] = nd_restrict_node<T>(d, r, I, J, K);
        }
        __syncthreads();
    }
    // bottom: FP64 conjugate gradients by the whole workgroup, work in LDS
    {
        const NDims& d = a.lv[nl - 1].d;
        const int nn = d.mx * d.my * d.mz;
        T* x = lds + nd_lds_off(a, nl - 1);
        long long wo = nd_lds_off(a, nl) * (long long)sizeof(T);
        wo = (wo + 7) / 8;  // in doubles, 8-byte aligned
        double* work = reinterpret_cast<double*>(lds) + wo;
        // a bottom of one wavefront's nodes runs in the first wavefront alone
        // (no workgroup barriers inside the iteration)
        if (nn <= kWave) {
            if (threadIdx.x < kWave)
                nd_block_cg<T, true>(d, x + nn, x, x + 3 * nn, a.bottom_inv_h12, a.bottom_rtol, a.bottom_maxit, 0,
                                     work, sh, a.bottom_iters);
        } else {
            nd_block_cg<T>(d, x + nn, x, x + 3 * nn, a.bottom_inv_h12, a.bottom_rtol, a.bottom_maxit, 0, work, sh,
                           a.bottom_iters);
        }
        __syncthreads();
    }
    // up
    for (int l = nl - 2; l >= 0; l--) {
        const NDims& d = a.lv[l].d;
        const int nn = d.mx * d.my * d.mz;
        T* x = lds + nd_lds_off(a, l);
        const T* b = x + nn;
        const T* sg = x + 3 * nn;
        const T* xc = lds + nd_lds_off(a, l + 1);
        const FastDiv fx((unsigned)d.mx), fy((unsigned)d.my);
        for (int e = threadIdx.x; e < nn; e += blockDim.x) {
            int i, j, k;
            split3((unsigned)e, fx, fy, i, j, k);
            x[e] += nd_prolong_node<T>(a.lv[l + 1].d, xc, i, j, k);
        }
        __syncthreads();
        for (int s = 0; s < a.nu2; s++)
            for (int colour = 3; colour >= 0; colour--) nd_cc_gs<T>(d, x, b, sg, a.lv[l].h12, colour);
    }
    {
        const NDims& d = a.lv[0].d;
        const int nn = d.mx * d.my * d.mz;
        const T* x = lds;
        for (int e = threadIdx.x; e < nn; e += blockDim.x) a.lv[0].x[e] = x[e];
    }
}

template <typename T>
long long nd_coarse_lds_bytes(const NDims* lv, int nlev)
{
    long long words = 0;
    for (int q = 0; q < nlev; q++) words += 3LL * lv[q].mx * lv[q].my * lv[q].mz + (long long)lv[q].nx * lv[q].ny * lv[q].nz;
    long long bytes = ((words * (long long)sizeof(T) + 7) / 8) * 8;
    const NDims& bt = lv[nlev - 1];
    return bytes + 4LL * bt.mx * bt.my * bt.mz * 8;
}

template <typename T>
void launch_nd_coarse(const NdCoarseArgs<T>& a, hipStream_t s)
{
    hipLaunchKernelGGL((k_nd_coarse<T>), dim3(1), dim3(1024), 0, s, a);
}

template long long nd_coarse_lds_bytes<float>(const NDims*, int);
template long long nd_coarse_lds_bytes<double>(const NDims*, int);
template void launch_nd_coarse<float>(const NdCoarseArgs<float>&, hipStream_t);
template void launch_nd_coarse<double>(const NdCoarseArgs<double>&, hipStream_t);

#define ND_INST(T)                                                                                        \
    template void launch_nd_gs<T>(const NDims&, T*, const T*, const T*, T, int, hipStream_t);             \
    template void launch_nd_resid<T>(const NDims&, const T*, const T*, const T*, T, T*, hipStream_t);     \
    template void launch_nd_restrict<T>(const NDims&, const NDims&, const T*, T*, hipStream_t);           \
    template void launch_nd_prolong<T>(const NDims&, const NDims&, T*, const T*, int, hipStream_t);       \
    template void launch_nd_bottom<T>(const NDims&, const T*, T*, const T*, double, double, int, int,     \
                                      double*, double*, hipStream_t);
ND_INST(float)
ND_INST(double)
template void launch_nd_sigma<double, float>(int, int, int, const double*, float*, int, hipStream_t);
template void launch_nd_sigma<double, double>(int, int, int, const double*, double*, int, hipStream_t);
template void launch_nd_sigma<float, float>(int, int, int, const float*, float*, int, hipStream_t);

}  // namespace mp
