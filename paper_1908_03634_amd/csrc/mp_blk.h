// mp_blk.h -- device helpers of the register-blocked finest-level kernels
// (strips of 2M x cells per lane, R rows per wavefront, z-marching; see
// k_blk.hip).  Included by the kernel files only.
#pragma once
#include "mp_device.h"

namespace mp {

constexpr int BK_W = 4;  // wavefronts per block
constexpr int BK_T = 64 * BK_W;  // threads per block

template <typename T>
struct V2;
template <>
struct V2<float> {
    using type = float2;
};
template <>
struct V2<double> {
    using type = double2;
};

// Whole-wavefront rotations: lane l receives lane l-1's value (lane 0 gets
// lane 63's), or lane l+1's (lane 63 gets lane 0's).  Every lane reads a
// valid source, so the DPP move needs no "old" value (mov_dpp: no register
// is zeroed first).
__device__ __forceinline__ float from_prev(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x13C, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_next(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x134, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_prev(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x13C, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x13C, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_next(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x134, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x134, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}


// 2M consecutive cells of one row.
template <typename T, int M>
struct Strip {
    T v[2 * M];
};

template <typename T, int M>
__device__ __forceinline__ Strip<T, M> ld_strip(const T* __restrict__ p, long long off)
{
    Strip<T, M> s;
    if constexpr (sizeof(T) == 4 && M % 2 == 0) {
#pragma unroll
        for (int q = 0; q < M / 2; q++) {
            const float4 f = *reinterpret_cast<const float4*>(p + off + 4 * q);
            s.v[4 * q] = f.x;
            s.v[4 * q + 1] = f.y;
            s.v[4 * q + 2] = f.z;
            s.v[4 * q + 3] = f.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < M; q++) {
            const typename V2<T>::type f = *reinterpret_cast<const typename V2<T>::type*>(p + off + 2 * q);
            s.v[2 * q] = f.x;
            s.v[2 * q + 1] = f.y;
        }
    }
    return s;
}

template <typename T, int M>
__device__ __forceinline__ void st_strip(T* __restrict__ p, long long off, const Strip<T, M>& s)
{
    if constexpr (sizeof(T) == 4 && M % 2 == 0) {
#pragma unroll
        for (int q = 0; q < M / 2; q++)
            *reinterpret_cast<float4*>(p + off + 4 * q) =
                make_float4(s.v[4 * q], s.v[4 * q + 1], s.v[4 * q + 2], s.v[4 * q + 3]);
    } else {
#pragma unroll
        for (int q = 0; q < M; q++)
            *reinterpret_cast<typename V2<T>::type*>(p + off + 2 * q) =
                typename V2<T>::type{s.v[2 * q], s.v[2 * q + 1]};
    }
}

template <typename T, int M>
__device__ __forceinline__ Strip<T, M> zero_strip()
{
    Strip<T, M> s;
#pragma unroll
    for (int c = 0; c < 2 * M; c++) s.v[c] = T(0);
    return s;
}

struct BlkGeo {
    int lane, xi, j0, z0, z1;
    bool hal;     // lane 0 or 63 of a wavefront that does not span the row: loads a halo column
    int hcol;     // that column (the wrap partner when periodic)
    bool wl, wr;  // the strip's first / last cell touches a Neumann wall
    bool live;    // the wavefront's rows lie inside the grid
    bool yfirst;  // row j0 has a face below
    bool ylast;   // row j0 + R - 1 has a face above
};

// Workgroups are dealt to the 8 XCDs in turn (workgroup p runs on XCD p % 8),
// and each XCD has its own L2.  Renumbering so that every XCD receives one
// contiguous run of (x tile, row block, plane chunk) keeps the halo rows and
// planes shared by neighbouring blocks inside one L2.
__device__ __forceinline__ void blk_tile(unsigned& bx, unsigned& by, unsigned& bz)
{
    const unsigned gx = gridDim.x, gy = gridDim.y, n = gridDim.x * gridDim.y * gridDim.z;
    unsigned p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    if (n % 8 == 0) p = (p % 8) * (n / 8) + p / 8;
    bx = p % gx;
    by = (p / gx) % gy;
    bz = p / (gx * gy);
}

template <int M, int R>
__device__ __forceinline__ BlkGeo blk_geo(const Dims& d, int lz)
{
    constexpr int W = 128 * M;  // columns per wavefront
    unsigned bx, by, bz;
    blk_tile(bx, by, bz);
    BlkGeo g;
    g.lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int x0 = (int)bx * W;
    g.xi = x0 + 2 * M * g.lane;
    g.j0 = ((int)by * BK_W + w) * R;
    g.live = g.j0 < d.ny;
    g.z0 = (int)bz * lz;
    g.z1 = min(g.z0 + lz, d.nz);
    const bool whole = W == d.nx;
    g.hal = !whole && (g.lane == 0 || g.lane == kWave - 1);
    g.hcol = g.lane == 0 ? (x0 > 0 ? x0 - 1 : d.nx - 1) : (x0 + W < d.nx ? x0 + W : 0);
    g.wl = g.xi == 0 && !d.px;
    g.wr = g.xi + 2 * M == d.nx && !d.px;
    g.yfirst = g.j0 > 0 || d.py;
    g.ylast = g.j0 + R < d.ny || d.py;
    return g;
}

// Row jj wrapped (periodic) or clamped to the wall row (Neumann; such a row
// only ever meets a zero coefficient).
__device__ __forceinline__ int wrap_row(const Dims& d, int jj)
{
    if (jj < 0) return d.py ? jj + d.ny : 0;
    if (jj >= d.ny) return d.py ? jj - d.ny : d.ny - 1;
    return jj;
}
__device__ __forceinline__ int wrap_plane(const Dims& d, int k)
{
    if (k < 0) return d.pz ? k + d.nz : 0;
    if (k >= d.nz) return d.pz ? k - d.nz : d.nz - 1;
    return k;
}

// x faces of a strip: f[0] left of cell 0, f[q] between cells q-1 and q,
// f[2M] right of the last cell (0 at walls).  hc: halo cell value (lanes 0/63
// of a partial-row wavefront).  All lanes must call (DPP).
template <typename T, int M>
__device__ __forceinline__ void x_faces(const BlkGeo& g, const Strip<T, M>& c, T hc, T (&f)[2 * M + 1])
{
    const T pl = from_prev(c.v[2 * M - 1]), nr = from_next(c.v[0]);
    const T cl = (g.hal && g.lane == 0) ? hc : pl;
    const T cr = (g.hal && g.lane == kWave - 1) ? hc : nr;
    f[0] = g.wl ? T(0) : harm(cl, c.v[0]);
#pragma unroll
    for (int q = 1; q < 2 * M; q++) f[q] = harm(c.v[q - 1], c.v[q]);
    f[2 * M] = g.wr ? T(0) : harm(c.v[2 * M - 1], cr);
}

// Values just outside the strip (left of cell 0, right of the last cell) as
// the neighbours see them.  All lanes must call (DPP).
template <typename T, int M>
__device__ __forceinline__ void x_edges(const BlkGeo& g, const Strip<T, M>& v, T hv, T& vl, T& vr)
{
    const T pl = from_prev(v.v[2 * M - 1]), nr = from_next(v.v[0]);
    vl = (g.hal && g.lane == 0) ? hv : pl;
    vr = (g.hal && g.lane == kWave - 1) ? hv : nr;
}

// y faces between rows t-1 and t (t = 0..R) of one plane.
template <typename T, int M, int R>
__device__ __forceinline__ void y_faces(const BlkGeo& g, const Strip<T, M> (&c)[R], const Strip<T, M>& clo,
                                        const Strip<T, M>& chi, T (&f)[R + 1][2 * M])
{
#pragma unroll
    for (int t = 0; t <= R; t++) {
        const Strip<T, M>& lo = t > 0 ? c[t > 0 ? t - 1 : 0] : clo;
        const Strip<T, M>& hi = t < R ? c[t < R ? t : 0] : chi;
        const bool has = (t > 0 || g.yfirst) && (t < R || g.ylast);
#pragma unroll
        for (int q = 0; q < 2 * M; q++) f[t][q] = has ? harm(lo.v[q], hi.v[q]) : T(0);
    }
}

// The 6 coefficients and 6 neighbour values of cell q of row t, in stencil
// order (x low, x high, y low, y high, z low, z high).  A neighbour behind a
// wall (coefficient 0) takes the cell's own value, as in the one-cell kernels.
template <typename T>
struct CellIn {
    T c[6], v[6];
};

template <typename T, int M, int R>
__device__ __forceinline__ CellIn<T> cell_in(int q, int t, const BlkGeo& g, bool hzm, bool hzp,
                                             const T (&fx)[2 * M + 1], const T (&fy)[R + 1][2 * M],
                                             const Strip<T, M>& c, const Strip<T, M>& czl, const Strip<T, M>& czh,
                                             const Strip<T, M>& nv, T vl, T vr, const Strip<T, M>& ylo,
                                             const Strip<T, M>& yhi, const Strip<T, M>& zlo, const Strip<T, M>& zhi,
                                             T own)
{
    CellIn<T> s;
    s.c[0] = fx[q];
    s.c[1] = fx[q + 1];
    s.c[2] = fy[t][q];
    s.c[3] = fy[t + 1][q];
    s.c[4] = hzm ? harm(czl.v[q], c.v[q]) : T(0);
    s.c[5] = hzp ? harm(c.v[q], czh.v[q]) : T(0);
    s.v[0] = q > 0 ? nv.v[q > 0 ? q - 1 : 0] : (g.wl ? own : vl);
    s.v[1] = q < 2 * M - 1 ? nv.v[q < 2 * M - 1 ? q + 1 : 0] : (g.wr ? own : vr);
    s.v[2] = (t == 0 && !g.yfirst) ? own : ylo.v[q];
    s.v[3] = (t == R - 1 && !g.ylast) ? own : yhi.v[q];
    s.v[4] = hzm ? zlo.v[q] : own;
    s.v[5] = hzp ? zhi.v[q] : own;
    return s;
}

// Parent corrections of a strip (one coarse value per pair of cells).
template <typename T, int M>
struct EStrip {
    T e[M];
};

template <typename T, int M>
__device__ __forceinline__ Strip<T, M> add_e(const Strip<T, M>& x, const EStrip<T, M>& e)
{
    Strip<T, M> r;
#pragma unroll
    for (int q = 0; q < 2 * M; q++) r.v[q] = x.v[q] + e.e[q >> 1];
    return r;
}

// ------------------------------------------------------------ launch shape

// Strip width M (pairs per lane): the whole row in one wavefront when
// nx / 128 <= 4, else the largest of 4, 3, 2, 1 that divides nx / 128.
inline int strip_pairs(const Dims& d)
{
    const int t = d.nx / 128;
    if (t <= 4) return t;
    for (int m = 4; m > 1; m--)
        if (t % m == 0) return m;
    return 1;
}

// Rows per wavefront (register budget): 4 for FP32 pairs, else 2.
template <typename T>
constexpr int rows_for(int M)
{
    return sizeof(T) == 4 && M == 1 ? 4 : 2;
}

// Planes per block: even, halved from 16 until the grid has at least
// `min_blocks` blocks, then doubled while it has more than `max_blocks`.
inline dim3 blk_grid(const Dims& d, int M, int rows, long long min_blocks, long long max_blocks, int& lz)
{
    const long long gx = d.nx / (128 * M), gy = (d.ny + rows * BK_W - 1) / (rows * BK_W);
    auto nb = [&](int l) { return gx * gy * ((d.nz + l - 1) / l); };
    lz = 16;
    while (lz > 2 && nb(lz) < min_blocks) lz >>= 1;
    while (lz < d.nz && nb(lz) > max_blocks) lz <<= 1;
    return dim3((unsigned)gx, (unsigned)gy, (unsigned)((d.nz + lz - 1) / lz));
}

constexpr long long kBlkMinBlocks = 512;

}  // namespace mp
