// k_blk.hip -- register-blocked finest-level kernels (cell-value coefficients).
//
// A 7-point stencil with one cell per thread issues about eleven memory
// instructions per cell (centre and in-plane neighbours of the iterate and of
// the coefficients, the right-hand side, the store), most of them misaligned
// by one element; on gfx950 that instruction stream, not HBM bandwidth, is
// what limits such kernels.  Here every lane owns a pair of x-adjacent cells
// (one 2-element vector access per row) in R consecutive rows and marches
// along z:
//   * x neighbours come from the adjacent lanes through whole-wavefront DPP
//     shifts; only lanes 0 and 63 load one halo column;
//   * y neighbours are the lane's own rows plus one halo row on each side;
//   * z neighbours stay in registers from the previous and next planes.
// About three row-contiguous memory instructions per cell remain.  Every cell
// is evaluated with the shared per-cell arithmetic of the one-cell-per-thread
// kernels (same operands, same order), so results agree bit for bit.
//
// Shape: 256-thread blocks of 4 wavefronts; block (bx, by, bz) covers columns
// [128 bx, 128 bx + 128), rows [4R by, 4R by + 4R) (R per wavefront: 4 in
// FP32, 2 for the FP64 residual) and planes [lz bz, lz bz + lz).  Requires nx % 128 == 0, ny % 4 == 0 and an even nz >= 4.
#include "mp_device.h"
#include "mp_kernels.h"

namespace mp {

constexpr int BK_W = 4;     // wavefronts per block
constexpr int BK_XW = 128;  // columns per wavefront (2 per lane)

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

// Lane l receives lane l-1's value (from_left) or lane l+1's (from_right);
// the lane at the wavefront's edge receives 0 and must substitute its halo.
__device__ __forceinline__ float dpp_from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double dpp_from_left(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_from_right(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

bool blk_supported(const Dims& d) { return d.nx % BK_XW == 0 && d.ny % 4 == 0 && d.nz >= 4 && d.nz % 2 == 0; }

struct BlkGeo {
    int lane, xi, j0, z0, z1;
    bool hasL, hasR;  // lane 0 / 63 couples to a cell beyond the wavefront
    int hcol;         // column of that cell
    bool live;        // the wavefront's rows lie inside the grid
    bool yfirst;      // row j0 has a face below
    bool ylast;       // row j0 + R - 1 has a face above
};

template <int R>
__device__ __forceinline__ BlkGeo blk_geo(const Dims& d, int lz)
{
    BlkGeo g;
    g.lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int x0 = blockIdx.x * BK_XW;
    g.xi = x0 + 2 * g.lane;
    g.j0 = (blockIdx.y * BK_W + w) * R;
    g.live = g.j0 < d.ny;
    g.z0 = blockIdx.z * lz;
    g.z1 = min(g.z0 + lz, d.nz);
    g.hasL = g.lane == 0 && (x0 > 0 || d.px);
    g.hasR = g.lane == kWave - 1 && (x0 + BK_XW < d.nx || d.px);
    g.hcol = g.lane == 0 ? (x0 > 0 ? x0 - 1 : d.nx - 1) : (x0 + BK_XW < d.nx ? x0 + BK_XW : 0);
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

template <typename T>
__device__ __forceinline__ typename V2<T>::type ld2(const T* p, long long q)
{
    return *reinterpret_cast<const typename V2<T>::type*>(p + q);
}

// The two cells (a = column xi, b = column xi + 1) of one row of a lane's
// pair: the 6 face coefficients and 6 neighbour values of each, in stencil
// order (x low, x high, y low, y high, z low, z high).
template <typename T>
struct PairSt {
    T ca[6], cb[6], va[6], vb[6];
};

// c, cz_lo, cz_hi: cell values of the row on planes k, k-1, k+1; hc: halo
// cell value (lanes 0/63); fy*: y faces below/above cells a and b; v: the
// row's values as neighbours see them, hv: halo value, y_lo/y_hi: rows
// below/above, z_lo/z_hi: planes below/above; own_a/own_b: the cells' own
// values, used in place of a neighbour behind a wall (coefficient 0), as the
// one-cell kernels do.
template <typename T>
__device__ __forceinline__ void pair_stencil(const BlkGeo& g, bool hzm, bool hzp, bool ywl, bool ywh,
                                             typename V2<T>::type c, typename V2<T>::type cz_lo,
                                             typename V2<T>::type cz_hi, T hc, T fyla, T fyha, T fylb, T fyhb,
                                             typename V2<T>::type v, T hv, typename V2<T>::type y_lo,
                                             typename V2<T>::type y_hi, typename V2<T>::type z_lo,
                                             typename V2<T>::type z_hi, T own_a, T own_b, PairSt<T>& s)
{
    // DPP before any lane-dependent selection (all lanes take part)
    const T cl_d = dpp_from_left(c.y), cr_d = dpp_from_right(c.x);
    const T vl_d = dpp_from_left(v.y), vr_d = dpp_from_right(v.x);
    const bool hl = g.lane > 0 || g.hasL, hr = g.lane < kWave - 1 || g.hasR;
    const T cl = g.lane == 0 ? hc : cl_d, cr = g.lane == kWave - 1 ? hc : cr_d;
    const T vl = g.lane == 0 ? hv : vl_d, vr = g.lane == kWave - 1 ? hv : vr_d;
    const T fab = harm(c.x, c.y);
    s.ca[0] = hl ? harm(cl, c.x) : T(0);
    s.ca[1] = fab;
    s.ca[2] = fyla;
    s.ca[3] = fyha;
    s.ca[4] = hzm ? harm(cz_lo.x, c.x) : T(0);
    s.ca[5] = hzp ? harm(c.x, cz_hi.x) : T(0);
    s.cb[0] = fab;
    s.cb[1] = hr ? harm(c.y, cr) : T(0);
    s.cb[2] = fylb;
    s.cb[3] = fyhb;
    s.cb[4] = hzm ? harm(cz_lo.y, c.y) : T(0);
    s.cb[5] = hzp ? harm(c.y, cz_hi.y) : T(0);
    s.va[0] = hl ? vl : own_a;
    s.va[1] = v.y;
    s.va[2] = ywl ? own_a : y_lo.x;
    s.va[3] = ywh ? own_a : y_hi.x;
    s.va[4] = hzm ? z_lo.x : own_a;
    s.va[5] = hzp ? z_hi.x : own_a;
    s.vb[0] = v.x;
    s.vb[1] = hr ? vr : own_b;
    s.vb[2] = ywl ? own_b : y_lo.y;
    s.vb[3] = ywh ? own_b : y_hi.y;
    s.vb[4] = hzm ? z_lo.y : own_b;
    s.vb[5] = hzp ? z_hi.y : own_b;
}

// y faces between rows t-1 and t (t = 0..R) of one plane, per cell of the pair.
template <typename T, int R>
__device__ __forceinline__ void y_faces(const BlkGeo& g, const typename V2<T>::type (&c)[R],
                                        typename V2<T>::type clo, typename V2<T>::type chi, T (&fa)[R + 1],
                                        T (&fb)[R + 1])
{
#pragma unroll
    for (int t = 0; t <= R; t++) {
        const typename V2<T>::type lo = t > 0 ? c[t - 1] : clo;
        const typename V2<T>::type hi = t < R ? c[t] : chi;
        const bool has = (t > 0 || g.yfirst) && (t < R || g.ylast);
        fa[t] = has ? harm(lo.x, hi.x) : T(0);
        fb[t] = has ? harm(lo.y, hi.y) : T(0);
    }
}

// ------------------------------------------------------------------ smoother

// One colour of red-black Gauss-Seidel, in place (modes: mp_kernels.h).  In
// GS_E_ALL the other cell of each pair is written back as read (without the
// correction): only the updated cell keeps x + e, and GS_E_OWN adds e to the
// cells of the second colour, so every cell receives e exactly once.

// IRU (FP32 only, last pass of a V-cycle): also phi += s[0] * x for both
// cells of every pair (the refinement update, otherwise a separate pass).
template <typename T, int MODE, int R, bool IRU>
__global__ __launch_bounds__(256) void k_gs_blk(Dims d, int lz, T* __restrict__ x, const T* __restrict__ b,
                                                const T* __restrict__ cc, T h2, int colour, const T* __restrict__ ec,
                                                double* __restrict__ phi, const double* __restrict__ irs)
{
    using P = typename V2<T>::type;
    constexpr bool ZI = MODE == GS_ZERO;
    constexpr bool EA = MODE == GS_E_ALL;
    constexpr bool EO = MODE == GS_E_ALL || MODE == GS_E_OWN;
    const BlkGeo g = blk_geo<R>(d, lz);
    if (!g.live) return;
    const long long sz = (long long)d.nx * d.ny;
    const int nxc = d.nx >> 1;
    const long long szc = (long long)nxc * (d.ny >> 1);
    int rows[R + 2];
    long long roff[R + 2];
#pragma unroll
    for (int t = 0; t < R + 2; t++) {
        rows[t] = wrap_row(d, g.j0 - 1 + t);
        roff[t] = (long long)rows[t] * d.nx;
    }
    auto epar = [&](int kk, int jj, int col) -> T {
        return ec[(long long)(kk >> 1) * szc + (long long)(jj >> 1) * nxc + (col >> 1)];
    };
    auto addp = [](P v, T e) -> P { return P{v.x + e, v.y + e}; };
    const P z2 = P{T(0), T(0)};

    // rings over planes k-1, k: raw x (not in GS_ZERO), parent corrections
    // (GS_E_ALL), cell values
    P xm[R], x0[R], cm[R], c0[R];
    T em[R], e0[R];
    {
        const int km = wrap_plane(d, g.z0 - 1);
        const long long bm = (long long)km * sz, b0 = (long long)g.z0 * sz;
#pragma unroll
        for (int t = 0; t < R; t++) {
            if constexpr (!ZI) {
                xm[t] = ld2(x, bm + roff[t + 1] + g.xi);
                x0[t] = ld2(x, b0 + roff[t + 1] + g.xi);
            } else {
                xm[t] = z2;
                x0[t] = z2;
            }
            if constexpr (EA) {
                em[t] = epar(km, rows[t + 1], g.xi);
                e0[t] = epar(g.z0, rows[t + 1], g.xi);
            }
            cm[t] = ld2(cc, bm + roff[t + 1] + g.xi);
            c0[t] = ld2(cc, b0 + roff[t + 1] + g.xi);
        }
    }
    for (int k = g.z0; k < g.z1; k++) {
        const bool hzm = k > 0 || d.pz, hzp = k < d.nz - 1 || d.pz;
        const int kp = wrap_plane(d, k + 1);
        const long long bk = (long long)k * sz, bp = (long long)kp * sz;
        P xp[R], cp[R], bq[R];
        T ep[R], hx[R], hc[R];
        P xlo = z2, xhi = z2;
        const P clo = ld2(cc, bk + roff[0] + g.xi);
        const P chi = ld2(cc, bk + roff[R + 1] + g.xi);
        if constexpr (!ZI) {
            xlo = ld2(x, bk + roff[0] + g.xi);
            xhi = ld2(x, bk + roff[R + 1] + g.xi);
            if constexpr (EA) {
                xlo = addp(xlo, epar(k, rows[0], g.xi));
                xhi = addp(xhi, epar(k, rows[R + 1], g.xi));
            }
        }
#pragma unroll
        for (int t = 0; t < R; t++) {
            xp[t] = ZI ? z2 : ld2(x, bp + roff[t + 1] + g.xi);
            if constexpr (EA) ep[t] = epar(kp, rows[t + 1], g.xi);
            if constexpr (MODE == GS_E_OWN) e0[t] = epar(k, rows[t + 1], g.xi);
            cp[t] = ld2(cc, bp + roff[t + 1] + g.xi);
            bq[t] = ld2(b, bk + roff[t + 1] + g.xi);
            hx[t] = T(0);
            hc[t] = T(0);
            if (g.hasL || g.hasR) {
                hc[t] = cc[bk + roff[t + 1] + g.hcol];
                if constexpr (!ZI) {
                    hx[t] = x[bk + roff[t + 1] + g.hcol];
                    if constexpr (EA) hx[t] += epar(k, rows[t + 1], g.hcol);
                }
            }
        }
        T fya[R + 1], fyb[R + 1];
        y_faces<T, R>(g, c0, clo, chi, fya, fyb);
        // rows as their neighbours see them
        P nv[R];
#pragma unroll
        for (int t = 0; t < R; t++) nv[t] = EA ? addp(x0[t], e0[t]) : x0[t];
#pragma unroll
        for (int t = 0; t < R; t++) {
            const int jj = g.j0 + t;
            const bool a_upd = ((jj + k) & 1) == colour;
            const T own_a = EO ? x0[t].x + e0[t] : x0[t].x;
            const T own_b = EO ? x0[t].y + e0[t] : x0[t].y;
            const P zl = EA ? addp(xm[t], em[t]) : xm[t];
            const P zh = EA ? addp(xp[t], ep[t]) : xp[t];
            PairSt<T> s;
            pair_stencil<T>(g, hzm, hzp, t == 0 && !g.yfirst, t == R - 1 && !g.ylast, c0[t], cm[t], cp[t], hc[t],
                            fya[t], fya[t + 1], fyb[t], fyb[t + 1], nv[t], hx[t], t > 0 ? nv[t - 1] : xlo,
                            t < R - 1 ? nv[t + 1] : xhi, zl, zh, own_a, own_b, s);
            P out = x0[t];
            if (a_upd)
                out.x = gs_value<T>(s.ca[0], s.ca[1], s.ca[2], s.ca[3], s.ca[4], s.ca[5], s.va[0], s.va[1], s.va[2],
                                    s.va[3], s.va[4], s.va[5], bq[t].x, h2, own_a);
            else
                out.y = gs_value<T>(s.cb[0], s.cb[1], s.cb[2], s.cb[3], s.cb[4], s.cb[5], s.vb[0], s.vb[1], s.vb[2],
                                    s.vb[3], s.vb[4], s.vb[5], bq[t].y, h2, own_b);
            *reinterpret_cast<P*>(x + bk + roff[t + 1] + g.xi) = out;
            if constexpr (IRU) {
                const double sc = irs[0];
                double2* pp = reinterpret_cast<double2*>(phi + bk + roff[t + 1] + g.xi);
                const double2 pv = *pp;
                *pp = make_double2(fma(sc, (double)out.x, pv.x), fma(sc, (double)out.y, pv.y));
            }
        }
#pragma unroll
        for (int t = 0; t < R; t++) {
            xm[t] = x0[t];
            x0[t] = xp[t];
            cm[t] = c0[t];
            c0[t] = cp[t];
            if constexpr (EA) {
                em[t] = e0[t];
                e0[t] = ep[t];
            }
        }
    }
}

// ------------------------------------------------- residual and restriction

// One plane's loads shared by the residual kernels (no prolongation terms).
template <typename T, int R>
struct PlaneIn {
    typename V2<T>::type xp[R], cp[R], bq[R], xlo, xhi, clo, chi;
    T hx[R], hc[R];
};

template <typename T, int R>
__device__ __forceinline__ void load_plane(const BlkGeo& g, const T* __restrict__ x, const T* __restrict__ b,
                                           const T* __restrict__ cc, const long long (&roff)[R + 2], long long bk,
                                           long long bp, PlaneIn<T, R>& q)
{
    q.xlo = ld2(x, bk + roff[0] + g.xi);
    q.xhi = ld2(x, bk + roff[R + 1] + g.xi);
    q.clo = ld2(cc, bk + roff[0] + g.xi);
    q.chi = ld2(cc, bk + roff[R + 1] + g.xi);
#pragma unroll
    for (int t = 0; t < R; t++) {
        q.xp[t] = ld2(x, bp + roff[t + 1] + g.xi);
        q.cp[t] = ld2(cc, bp + roff[t + 1] + g.xi);
        q.bq[t] = ld2(b, bk + roff[t + 1] + g.xi);
        q.hx[t] = T(0);
        q.hc[t] = T(0);
        if (g.hasL || g.hasR) {
            q.hx[t] = x[bk + roff[t + 1] + g.hcol];
            q.hc[t] = cc[bk + roff[t + 1] + g.hcol];
        }
    }
}

// Residuals b - A x of the pair in every row of plane k.
template <typename T, int R>
__device__ __forceinline__ void plane_resid(const BlkGeo& g, bool hzm, bool hzp, const typename V2<T>::type (&xm)[R],
                                            const typename V2<T>::type (&x0)[R],
                                            const typename V2<T>::type (&cm)[R],
                                            const typename V2<T>::type (&c0)[R], const PlaneIn<T, R>& q, T inv_h2,
                                            T (&ra)[R], T (&rb)[R])
{
    T fya[R + 1], fyb[R + 1];
    y_faces<T, R>(g, c0, q.clo, q.chi, fya, fyb);
#pragma unroll
    for (int t = 0; t < R; t++) {
        PairSt<T> s;
        pair_stencil<T>(g, hzm, hzp, t == 0 && !g.yfirst, t == R - 1 && !g.ylast, c0[t], cm[t], q.cp[t], q.hc[t],
                        fya[t], fya[t + 1], fyb[t], fyb[t + 1], x0[t], q.hx[t], t > 0 ? x0[t - 1] : q.xlo,
                        t < R - 1 ? x0[t + 1] : q.xhi, xm[t], q.xp[t], x0[t].x, x0[t].y, s);
        ra[t] = resid_value<T>(s.ca[0], s.ca[1], s.ca[2], s.ca[3], s.ca[4], s.ca[5], s.va[0], s.va[1], s.va[2],
                               s.va[3], s.va[4], s.va[5], x0[t].x, q.bq[t].x, inv_h2);
        rb[t] = resid_value<T>(s.cb[0], s.cb[1], s.cb[2], s.cb[3], s.cb[4], s.cb[5], s.vb[0], s.vb[1], s.vb[2],
                               s.vb[3], s.vb[4], s.vb[5], x0[t].y, q.bq[t].y, inv_h2);
    }
}

template <typename T, int R>
__device__ __forceinline__ void ring_start(const Dims& d, const BlkGeo& g, const T* __restrict__ x,
                                           const T* __restrict__ cc, const long long (&roff)[R + 2], long long sz,
                                           typename V2<T>::type (&xm)[R], typename V2<T>::type (&x0)[R],
                                           typename V2<T>::type (&cm)[R], typename V2<T>::type (&c0)[R])
{
    const long long bm = (long long)wrap_plane(d, g.z0 - 1) * sz, b0 = (long long)g.z0 * sz;
#pragma unroll
    for (int t = 0; t < R; t++) {
        xm[t] = ld2(x, bm + roff[t + 1] + g.xi);
        x0[t] = ld2(x, b0 + roff[t + 1] + g.xi);
        cm[t] = ld2(cc, bm + roff[t + 1] + g.xi);
        c0[t] = ld2(cc, b0 + roff[t + 1] + g.xi);
    }
}

template <typename T, int R>
__device__ __forceinline__ void ring_shift(typename V2<T>::type (&xm)[R], typename V2<T>::type (&x0)[R],
                                           typename V2<T>::type (&cm)[R], typename V2<T>::type (&c0)[R],
                                           const PlaneIn<T, R>& q)
{
#pragma unroll
    for (int t = 0; t < R; t++) {
        xm[t] = x0[t];
        x0[t] = q.xp[t];
        cm[t] = c0[t];
        c0[t] = q.cp[t];
    }
}

// Coarse right-hand side = mean of the 8 fine residuals of each coarse cell,
// summed in the order of restrict_cell (z, then y, then x child).  A lane's
// pair is the two x children of one coarse cell; planes are taken in pairs
// (chunks start on even planes), rows in pairs (j0 is a multiple of 4).
template <typename T, int R>
__global__ __launch_bounds__(256) void k_rr_blk(Dims d, int lz, const T* __restrict__ x, const T* __restrict__ b,
                                                const T* __restrict__ cc, T inv_h2, T* __restrict__ bc)
{
    using P = typename V2<T>::type;
    const BlkGeo g = blk_geo<R>(d, lz);
    if (!g.live) return;
    const long long sz = (long long)d.nx * d.ny;
    const int nxc = d.nx >> 1;
    const long long szc = (long long)nxc * (d.ny >> 1);
    long long roff[R + 2];
#pragma unroll
    for (int t = 0; t < R + 2; t++) roff[t] = (long long)wrap_row(d, g.j0 - 1 + t) * d.nx;
    P xm[R], x0[R], cm[R], c0[R];
    ring_start<T, R>(d, g, x, cc, roff, sz, xm, x0, cm, c0);
    for (int k = g.z0; k < g.z1; k += 2) {
        T r[2][R][2];  // [z child][row][x child]
#pragma unroll
        for (int cz = 0; cz < 2; cz++) {
            const int kk = k + cz;
            const bool hzm = kk > 0 || d.pz, hzp = kk < d.nz - 1 || d.pz;
            PlaneIn<T, R> q;
            load_plane<T, R>(g, x, b, cc, roff, (long long)kk * sz, (long long)wrap_plane(d, kk + 1) * sz, q);
            T ra[R], rb[R];
            plane_resid<T, R>(g, hzm, hzp, xm, x0, cm, c0, q, inv_h2, ra, rb);
#pragma unroll
            for (int t = 0; t < R; t++) {
                r[cz][t][0] = ra[t];
                r[cz][t][1] = rb[t];
            }
            ring_shift<T, R>(xm, x0, cm, c0, q);
        }
        const long long base = (long long)(k >> 1) * szc + (g.xi >> 1);
#pragma unroll
        for (int u = 0; u < R / 2; u++) {
            T acc = T(0);
#pragma unroll
            for (int cz = 0; cz < 2; cz++)
#pragma unroll
                for (int bb = 0; bb < 2; bb++)
#pragma unroll
                    for (int a = 0; a < 2; a++) acc += r[cz][2 * u + bb][a];
            bc[base + (long long)((g.j0 >> 1) + u) * nxc] = T(0.125) * acc;
        }
    }
}

// FP64 refinement residual r = b - A x, its scaled FP32 copy
// r32 = float(r * inv_s[0]) (when r32 != nullptr) and per-block sums of r^2.
template <int R>
__global__ __launch_bounds__(256) void k_resid64_blk(Dims d, int lz, const double* __restrict__ x,
                                                     const double* __restrict__ b, const double* __restrict__ cc,
                                                     double inv_h2, float* __restrict__ r32,
                                                     const double* __restrict__ inv_s, double* partials)
{
    using P = double2;
    __shared__ double sh[BK_W];
    const BlkGeo g = blk_geo<R>(d, lz);
    double acc = 0.0;
    if (g.live) {
        const double is = r32 ? inv_s[0] : 0.0;
        const long long sz = (long long)d.nx * d.ny;
        long long roff[R + 2];
#pragma unroll
        for (int t = 0; t < R + 2; t++) roff[t] = (long long)wrap_row(d, g.j0 - 1 + t) * d.nx;
        P xm[R], x0[R], cm[R], c0[R];
        ring_start<double, R>(d, g, x, cc, roff, sz, xm, x0, cm, c0);
        for (int k = g.z0; k < g.z1; k++) {
            const bool hzm = k > 0 || d.pz, hzp = k < d.nz - 1 || d.pz;
            const long long bk = (long long)k * sz;
            PlaneIn<double, R> q;
            load_plane<double, R>(g, x, b, cc, roff, bk, (long long)wrap_plane(d, k + 1) * sz, q);
            double ra[R], rb[R];
            plane_resid<double, R>(g, hzm, hzp, xm, x0, cm, c0, q, inv_h2, ra, rb);
#pragma unroll
            for (int t = 0; t < R; t++) {
                acc = fma(ra[t], ra[t], acc);
                acc = fma(rb[t], rb[t], acc);
                if (r32)
                    *reinterpret_cast<float2*>(r32 + bk + roff[t + 1] + g.xi) =
                        make_float2((float)(ra[t] * is), (float)(rb[t] * is));
            }
            ring_shift<double, R>(xm, x0, cm, c0, q);
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// ------------------------------------------------------------------ launches

// Rows per wavefront: 4 in FP32, 2 in FP64 (register budget).
constexpr int kRowsF = 4;
constexpr int kRowsD = 2;
template <typename T>
constexpr int rows_of() { return sizeof(T) == 4 ? kRowsF : kRowsD; }

// Planes per block: even, halved from 16 until the grid has at least
// `min_blocks` blocks, then doubled while it has more than `max_blocks`.
static dim3 blk_grid(const Dims& d, int rows, long long min_blocks, long long max_blocks, int& lz)
{
    const long long gx = d.nx / BK_XW, gy = (d.ny + rows * BK_W - 1) / (rows * BK_W);
    auto nb = [&](int l) { return gx * gy * ((d.nz + l - 1) / l); };
    lz = 16;
    while (lz > 2 && nb(lz) < min_blocks) lz >>= 1;
    while (lz < d.nz && nb(lz) > max_blocks) lz <<= 1;
    return dim3((unsigned)gx, (unsigned)gy, (unsigned)((d.nz + lz - 1) / lz));
}

constexpr long long kBlkMinBlocks = 512;

int blk_reduce_blocks(const Dims& d)
{
    int lz;
    const dim3 g = blk_grid(d, kRowsD, kBlkMinBlocks, kMaxRedBlocks, lz);
    return (int)(g.x * g.y * g.z);
}

template <typename T, int MODE, bool IRU>
static void gs_launch(const dim3& grid, const Dims& d, int lz, T* x, const T* b, const T* cc, T h2, int colour,
                      const T* ec, double* phi, const double* irs, hipStream_t s)
{
    hipLaunchKernelGGL((k_gs_blk<T, MODE, rows_of<T>(), IRU>), grid, dim3(256), 0, s, d, lz, x, b, cc, h2, colour,
                       ec, phi, irs);
}

template <typename T, bool IRU>
static void gs_mode(int mode, const dim3& grid, const Dims& d, int lz, T* x, const T* b, const T* cc, T h2,
                    int colour, const T* ec, double* phi, const double* irs, hipStream_t s)
{
    if constexpr (IRU) {
        // the refinement update rides on the last pass of a V-cycle: colour 1
        // of a plain sweep, or of the first sweep after prolongation
        if (mode == GS_E_OWN) gs_launch<T, GS_E_OWN, true>(grid, d, lz, x, b, cc, h2, colour, ec, phi, irs, s);
        else gs_launch<T, GS_PLAIN, true>(grid, d, lz, x, b, cc, h2, colour, ec, phi, irs, s);
        return;
    }
    switch (mode) {
    case GS_ZERO: gs_launch<T, GS_ZERO, IRU>(grid, d, lz, x, b, cc, h2, colour, ec, phi, irs, s); break;
    case GS_E_ALL: gs_launch<T, GS_E_ALL, IRU>(grid, d, lz, x, b, cc, h2, colour, ec, phi, irs, s); break;
    case GS_E_OWN: gs_launch<T, GS_E_OWN, IRU>(grid, d, lz, x, b, cc, h2, colour, ec, phi, irs, s); break;
    default: gs_launch<T, GS_PLAIN, IRU>(grid, d, lz, x, b, cc, h2, colour, ec, phi, irs, s); break;
    }
}

template <typename T>
void launch_gs_blk(const Dims& d, T* x, const T* b, const T* cc, T h2, int colour, int mode, const T* ec,
                   double* phi, const double* irs, hipStream_t s)
{
    int lz;
    const dim3 grid = blk_grid(d, rows_of<T>(), kBlkMinBlocks, 1LL << 30, lz);
    if constexpr (sizeof(T) == 4) {
        if (phi) {
            gs_mode<T, true>(mode, grid, d, lz, x, b, cc, h2, colour, ec, phi, irs, s);
            return;
        }
    }
    gs_mode<T, false>(mode, grid, d, lz, x, b, cc, h2, colour, ec, nullptr, nullptr, s);
}

template <typename T>
void launch_rr_blk(const Dims& d, const T* x, const T* b, const T* cc, T inv_h2, T* bc, hipStream_t s)
{
    int lz;
    const dim3 grid = blk_grid(d, rows_of<T>(), kBlkMinBlocks, 1LL << 30, lz);
    hipLaunchKernelGGL((k_rr_blk<T, rows_of<T>()>), grid, dim3(256), 0, s, d, lz, x, b, cc, inv_h2, bc);
}

void launch_resid64_blk(const Dims& d, const double* x, const double* b, const double* cc, double inv_h2, float* r32,
                        const double* inv_s, double* partials, int* nb_out, hipStream_t s)
{
    int lz;
    const dim3 grid = blk_grid(d, kRowsD, kBlkMinBlocks, kMaxRedBlocks, lz);
    *nb_out = (int)(grid.x * grid.y * grid.z);
    hipLaunchKernelGGL((k_resid64_blk<kRowsD>), grid, dim3(256), 0, s, d, lz, x, b, cc, inv_h2, r32, inv_s,
                       partials);
}

template void launch_gs_blk<float>(const Dims&, float*, const float*, const float*, float, int, int, const float*,
                                   double*, const double*, hipStream_t);
template void launch_gs_blk<double>(const Dims&, double*, const double*, const double*, double, int, int,
                                    const double*, double*, const double*, hipStream_t);
template void launch_rr_blk<float>(const Dims&, const float*, const float*, const float*, float, float*, hipStream_t);
template void launch_rr_blk<double>(const Dims&, const double*, const double*, const double*, double, double*,
                                    hipStream_t);

}  // namespace mp
