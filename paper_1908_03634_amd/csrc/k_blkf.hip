// k_blkf.hip -- register-blocked kernels for levels with stored face
// coefficients (the coarse levels of the hierarchy, and a finest level whose
// coefficients the caller set).
//
// The layout and the march are those of k_blk.hip (strips of 2M x cells per
// lane, R rows per wavefront, z-marching, DPP rotations across lanes); the
// coefficients are the level's three low-face arrays instead of cell values:
// the x faces of a strip are its own row segment plus the first face of the
// next strip, the y faces its own rows plus one row above, the z faces the
// current and next plane.  Every cell is evaluated with the shared per-cell
// arithmetic in the operand order of the one-cell kernels, so results agree
// bit for bit.
#include "mp_blk.h"
#include "mp_device.h"
#include "mp_kernels.h"

namespace mp {

// Face coefficients of the strip in row t: fx[0..2M], fy (low, high) and fz
// (low, high) per cell; walls 0.
template <typename T, int M>
struct FaceRow {
    T fx[2 * M + 1];
    T fyl[2 * M], fyh[2 * M], fzl[2 * M], fzh[2 * M];
};

// cx, cyl, cyh, czl, czh: strips of the x faces (plane k), the low y faces of
// the row and of the row above, the z faces of planes k and k+1; hcx: the x
// face beyond lane 63's strip (partial-row wavefronts); yh, zh: the row above
// and the plane above are inside the domain or across a wrap.
template <typename T, int M>
__device__ __forceinline__ FaceRow<T, M> face_row(const BlkGeo& g, const Strip<T, M>& cx, T hcx,
                                                  const Strip<T, M>& cyl, const Strip<T, M>& cyh, bool yh,
                                                  const Strip<T, M>& czl, const Strip<T, M>& czh, bool zh)
{
    FaceRow<T, M> f;
    const T nr = from_next(cx.v[0]);
#pragma unroll
    for (int q = 0; q < 2 * M; q++) f.fx[q] = cx.v[q];
    f.fx[2 * M] = g.wr ? T(0) : ((g.hal && g.lane == kWave - 1) ? hcx : nr);
#pragma unroll
    for (int q = 0; q < 2 * M; q++) {
        f.fyl[q] = cyl.v[q];
        f.fyh[q] = yh ? cyh.v[q] : T(0);
        f.fzl[q] = czl.v[q];
        f.fzh[q] = zh ? czh.v[q] : T(0);
    }
    return f;
}

template <typename T, int MODE, int M, int R>
__global__ __launch_bounds__(BK_T) void k_gs_blkf(Dims d, int lz, T* __restrict__ x, const T* __restrict__ b,
                                                  const T* __restrict__ cxa, const T* __restrict__ cya,
                                                  const T* __restrict__ cza, T h2, int colour,
                                                  const T* __restrict__ ec)
{
    using S = Strip<T, M>;
    using E = EStrip<T, M>;
    constexpr bool ZI = MODE == GS_ZERO;
    constexpr bool EA = MODE == GS_E_ALL;
    constexpr bool EO = MODE == GS_E_ALL || MODE == GS_E_OWN;
    const BlkGeo g = blk_geo<M, R>(d, lz);
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
    auto epar = [&](int kk, int jj) -> E {
        E e;
        const long long o = (long long)(kk >> 1) * szc + (long long)(jj >> 1) * nxc + (g.xi >> 1);
#pragma unroll
        for (int q = 0; q < M; q++) e.e[q] = ec[o + q];
        return e;
    };
    auto epar1 = [&](int kk, int jj, int col) -> T {
        return ec[(long long)(kk >> 1) * szc + (long long)(jj >> 1) * nxc + (col >> 1)];
    };

    S xm[R], x0[R], cz0[R];
    E em[R], e0[R];
    {
        const int km = wrap_plane(d, g.z0 - 1);
        const long long bm = (long long)km * sz, b0 = (long long)g.z0 * sz;
#pragma unroll
        for (int t = 0; t < R; t++) {
            if constexpr (!ZI) {
                xm[t] = ld_strip<T, M>(x, bm + roff[t + 1] + g.xi);
                x0[t] = ld_strip<T, M>(x, b0 + roff[t + 1] + g.xi);
            } else {
                xm[t] = zero_strip<T, M>();
                x0[t] = zero_strip<T, M>();
            }
            if constexpr (EA) {
                em[t] = epar(km, rows[t + 1]);
                e0[t] = epar(g.z0, rows[t + 1]);
            }
            cz0[t] = ld_strip<T, M>(cza, b0 + roff[t + 1] + g.xi);
        }
    }
    // loads of plane k (b, x and y faces, halo rows / column) and of plane k+1
    // (x, z faces), issued one plane ahead of their use
    struct Ld {
        S xp[R], czp[R], bq[R], cx[R], cy[R + 1], xlo, xhi;
        E ep[R], eo[R];
        T hx[R], hcx[R];
    };
    auto load = [&](int k) -> Ld {
        Ld L;
        const int kp = wrap_plane(d, k + 1);
        const long long bk = (long long)k * sz, bp = (long long)kp * sz;
        L.xlo = zero_strip<T, M>();
        L.xhi = zero_strip<T, M>();
        if constexpr (!ZI) {
            L.xlo = ld_strip<T, M>(x, bk + roff[0] + g.xi);
            L.xhi = ld_strip<T, M>(x, bk + roff[R + 1] + g.xi);
            if constexpr (EA) {
                L.xlo = add_e(L.xlo, epar(k, rows[0]));
                L.xhi = add_e(L.xhi, epar(k, rows[R + 1]));
            }
        }
        L.cy[R] = ld_strip<T, M>(cya, bk + roff[R + 1] + g.xi);
#pragma unroll
        for (int t = 0; t < R; t++) {
            L.xp[t] = ZI ? zero_strip<T, M>() : ld_strip<T, M>(x, bp + roff[t + 1] + g.xi);
            if constexpr (EA) L.ep[t] = epar(kp, rows[t + 1]);
            if constexpr (MODE == GS_E_OWN) L.eo[t] = epar(k, rows[t + 1]);
            L.czp[t] = ld_strip<T, M>(cza, bp + roff[t + 1] + g.xi);
            L.bq[t] = ld_strip<T, M>(b, bk + roff[t + 1] + g.xi);
            L.cx[t] = ld_strip<T, M>(cxa, bk + roff[t + 1] + g.xi);
            L.cy[t] = ld_strip<T, M>(cya, bk + roff[t + 1] + g.xi);
            L.hx[t] = T(0);
            L.hcx[t] = T(0);
            if (g.hal) {
                L.hcx[t] = cxa[bk + roff[t + 1] + g.hcol];
                if constexpr (!ZI) {
                    L.hx[t] = x[bk + roff[t + 1] + g.hcol];
                    if constexpr (EA) L.hx[t] += epar1(k, rows[t + 1], g.hcol);
                }
            }
        }
        return L;
    };
    Ld cur = load(g.z0);
    for (int k = g.z0; k < g.z1; k++) {
        const bool hzm = k > 0 || d.pz, hzp = k < d.nz - 1 || d.pz;
        const long long bk = (long long)k * sz;
        Ld nxt;
        if (k + 1 < g.z1) nxt = load(k + 1);
        if constexpr (MODE == GS_E_OWN) {
#pragma unroll
            for (int t = 0; t < R; t++) e0[t] = cur.eo[t];
        }
        S nv[R];
#pragma unroll
        for (int t = 0; t < R; t++) nv[t] = EA ? add_e(x0[t], e0[t]) : x0[t];
#pragma unroll
        for (int t = 0; t < R; t++) {
            const FaceRow<T, M> f = face_row<T, M>(g, cur.cx[t], cur.hcx[t], cur.cy[t], cur.cy[t + 1],
                                                   t < R - 1 || g.ylast, cz0[t], cur.czp[t], hzp);
            T vl, vr;
            x_edges<T, M>(g, nv[t], cur.hx[t], vl, vr);
            const S zl = EA ? add_e(xm[t], em[t]) : xm[t];
            const S zh = EA ? add_e(cur.xp[t], cur.ep[t]) : cur.xp[t];
            const S& ylo = t > 0 ? nv[t > 0 ? t - 1 : 0] : cur.xlo;
            const S& yhi = t < R - 1 ? nv[t < R - 1 ? t + 1 : 0] : cur.xhi;
            const bool ywl = t == 0 && !g.yfirst, ywh = t == R - 1 && !g.ylast;
            S out = x0[t];
            auto upd = [&](int q) {
                const T own = EO ? x0[t].v[q] + e0[t].e[q >> 1] : x0[t].v[q];
                const T xm_ = q > 0 ? nv[t].v[q > 0 ? q - 1 : 0] : (g.wl ? own : vl);
                const T xp_ = q < 2 * M - 1 ? nv[t].v[q < 2 * M - 1 ? q + 1 : 0] : (g.wr ? own : vr);
                const T ym = ywl ? own : ylo.v[q];
                const T yp = ywh ? own : yhi.v[q];
                const T zm = hzm ? zl.v[q] : own;
                const T zp = hzp ? zh.v[q] : own;
                out.v[q] = gs_value<T>(f.fx[q], f.fx[q + 1], f.fyl[q], f.fyh[q], f.fzl[q], f.fzh[q], xm_, xp_, ym, yp,
                                       zm, zp, cur.bq[t].v[q], h2, own);
            };
            if (((colour + g.j0 + t + k) & 1) == 0) {
#pragma unroll
                for (int q = 0; q < 2 * M; q += 2) upd(q);
            } else {
#pragma unroll
                for (int q = 1; q < 2 * M; q += 2) upd(q);
            }
            st_strip<T, M>(x, bk + roff[t + 1] + g.xi, out);
        }
#pragma unroll
        for (int t = 0; t < R; t++) {
            xm[t] = x0[t];
            x0[t] = cur.xp[t];
            cz0[t] = cur.czp[t];
            if constexpr (EA) {
                em[t] = e0[t];
                e0[t] = cur.ep[t];
            }
        }
        cur = nxt;
    }
}

// Coarse right-hand side = mean of the 8 fine residuals (restrict_cell order).
template <typename T, int M, int R>
__global__ __launch_bounds__(BK_T) void k_rr_blkf(Dims d, int lz, const T* __restrict__ x, const T* __restrict__ b,
                                                  const T* __restrict__ cxa, const T* __restrict__ cya,
                                                  const T* __restrict__ cza, T inv_h2, T* __restrict__ bc)
{
    using S = Strip<T, M>;
    const BlkGeo g = blk_geo<M, R>(d, lz);
    if (!g.live) return;
    const long long sz = (long long)d.nx * d.ny;
    const int nxc = d.nx >> 1;
    const long long szc = (long long)nxc * (d.ny >> 1);
    long long roff[R + 2];
#pragma unroll
    for (int t = 0; t < R + 2; t++) roff[t] = (long long)wrap_row(d, g.j0 - 1 + t) * d.nx;
    S xm[R], x0[R], cz0[R];
    {
        const long long bm = (long long)wrap_plane(d, g.z0 - 1) * sz, b0 = (long long)g.z0 * sz;
#pragma unroll
        for (int t = 0; t < R; t++) {
            xm[t] = ld_strip<T, M>(x, bm + roff[t + 1] + g.xi);
            x0[t] = ld_strip<T, M>(x, b0 + roff[t + 1] + g.xi);
            cz0[t] = ld_strip<T, M>(cza, b0 + roff[t + 1] + g.xi);
        }
    }
    struct Ld {
        S xp[R], czp[R], bq[R], cx[R], cy[R + 1], xlo, xhi;
        T hx[R], hcx[R];
    };
    auto load = [&](int k) -> Ld {
        Ld L;
        const long long bk = (long long)k * sz, bp = (long long)wrap_plane(d, k + 1) * sz;
        L.xlo = ld_strip<T, M>(x, bk + roff[0] + g.xi);
        L.xhi = ld_strip<T, M>(x, bk + roff[R + 1] + g.xi);
        L.cy[R] = ld_strip<T, M>(cya, bk + roff[R + 1] + g.xi);
#pragma unroll
        for (int t = 0; t < R; t++) {
            L.xp[t] = ld_strip<T, M>(x, bp + roff[t + 1] + g.xi);
            L.czp[t] = ld_strip<T, M>(cza, bp + roff[t + 1] + g.xi);
            L.bq[t] = ld_strip<T, M>(b, bk + roff[t + 1] + g.xi);
            L.cx[t] = ld_strip<T, M>(cxa, bk + roff[t + 1] + g.xi);
            L.cy[t] = ld_strip<T, M>(cya, bk + roff[t + 1] + g.xi);
            L.hx[t] = T(0);
            L.hcx[t] = T(0);
            if (g.hal) {
                L.hx[t] = x[bk + roff[t + 1] + g.hcol];
                L.hcx[t] = cxa[bk + roff[t + 1] + g.hcol];
            }
        }
        return L;
    };
    Ld cur = load(g.z0);
    for (int k = g.z0; k < g.z1; k += 2) {
        S r[2][R];  // [z child][row]
#pragma unroll
        for (int cz = 0; cz < 2; cz++) {
            const int kk = k + cz;
            const bool hzm = kk > 0 || d.pz, hzp = kk < d.nz - 1 || d.pz;
            Ld nxt;
            if (kk + 1 < g.z1) nxt = load(kk + 1);
#pragma unroll
            for (int t = 0; t < R; t++) {
                const FaceRow<T, M> f = face_row<T, M>(g, cur.cx[t], cur.hcx[t], cur.cy[t], cur.cy[t + 1],
                                                       t < R - 1 || g.ylast, cz0[t], cur.czp[t], hzp);
                T vl, vr;
                x_edges<T, M>(g, x0[t], cur.hx[t], vl, vr);
                const S& ylo = t > 0 ? x0[t > 0 ? t - 1 : 0] : cur.xlo;
                const S& yhi = t < R - 1 ? x0[t < R - 1 ? t + 1 : 0] : cur.xhi;
                const bool ywl = t == 0 && !g.yfirst, ywh = t == R - 1 && !g.ylast;
#pragma unroll
                for (int q = 0; q < 2 * M; q++) {
                    const T own = x0[t].v[q];
                    const T xm_ = q > 0 ? x0[t].v[q > 0 ? q - 1 : 0] : (g.wl ? own : vl);
                    const T xp_ = q < 2 * M - 1 ? x0[t].v[q < 2 * M - 1 ? q + 1 : 0] : (g.wr ? own : vr);
                    const T ym = ywl ? own : ylo.v[q];
                    const T yp = ywh ? own : yhi.v[q];
                    const T zm = hzm ? xm[t].v[q] : own;
                    const T zp = hzp ? cur.xp[t].v[q] : own;
                    r[cz][t].v[q] = resid_value<T>(f.fx[q], f.fx[q + 1], f.fyl[q], f.fyh[q], f.fzl[q], f.fzh[q], xm_,
                                                   xp_, ym, yp, zm, zp, own, cur.bq[t].v[q], inv_h2);
                }
            }
#pragma unroll
            for (int t = 0; t < R; t++) {
                xm[t] = x0[t];
                x0[t] = cur.xp[t];
                cz0[t] = cur.czp[t];
            }
            cur = nxt;
        }
        const long long base = (long long)(k >> 1) * szc + (g.xi >> 1);
#pragma unroll
        for (int u = 0; u < R / 2; u++) {
            T* o = bc + base + (long long)((g.j0 >> 1) + u) * nxc;
#pragma unroll
            for (int m = 0; m < M; m++) {
                T acc = T(0);
#pragma unroll
                for (int cz = 0; cz < 2; cz++)
#pragma unroll
                    for (int bb = 0; bb < 2; bb++)
#pragma unroll
                        for (int a = 0; a < 2; a++) acc += r[cz][2 * u + bb].v[2 * m + a];
                o[m] = T(0.125) * acc;
            }
        }
    }
}

// ------------------------------------------------------------------ launches

template <typename T, int MODE, int M>
static void gsf_launch(const Dims& d, T* x, const T* b, const Coef<T>& c, T h2, int colour, const T* ec,
                       hipStream_t s)
{
    constexpr int R = rows_for<T>(M);
    int lz;
    const dim3 grid = blk_grid(d, M, R, kBlkMinBlocks, 1LL << 30, lz);
    hipLaunchKernelGGL((k_gs_blkf<T, MODE, M, R>), grid, dim3(BK_T), 0, s, d, lz, x, b, c.x, c.y, c.z, h2, colour,
                       ec);
}

template <typename T, int M>
static void gsf_mode(int mode, const Dims& d, T* x, const T* b, const Coef<T>& c, T h2, int colour, const T* ec,
                     hipStream_t s)
{
    switch (mode) {
    case GS_ZERO: gsf_launch<T, GS_ZERO, M>(d, x, b, c, h2, colour, ec, s); break;
    case GS_E_ALL: gsf_launch<T, GS_E_ALL, M>(d, x, b, c, h2, colour, ec, s); break;
    case GS_E_OWN: gsf_launch<T, GS_E_OWN, M>(d, x, b, c, h2, colour, ec, s); break;
    default: gsf_launch<T, GS_PLAIN, M>(d, x, b, c, h2, colour, ec, s); break;
    }
}

// Strip width: pairs in FP64 and when nx / 128 is odd, else strips of 4.
template <typename T>
static bool face_pairs(const Dims& d)
{
    return sizeof(T) == 8 || (d.nx / 128) % 2 != 0;
}

template <typename T>
void launch_gs_blkf(const Dims& d, T* x, const T* b, const Coef<T>& c, T h2, int colour, int mode, const T* ec,
                    hipStream_t s)
{
    if (face_pairs<T>(d)) gsf_mode<T, 1>(mode, d, x, b, c, h2, colour, ec, s);
    else gsf_mode<T, 2>(mode, d, x, b, c, h2, colour, ec, s);
}

template <typename T>
void launch_rr_blkf(const Dims& d, const T* x, const T* b, const Coef<T>& c, T inv_h2, T* bc, hipStream_t s)
{
    // pairs in two rows per wavefront: the residuals of two planes stay live
    constexpr int R = 2;
    int lz;
    const dim3 grid = blk_grid(d, 1, R, kBlkMinBlocks, 1LL << 30, lz);
    hipLaunchKernelGGL((k_rr_blkf<T, 1, R>), grid, dim3(BK_T), 0, s, d, lz, x, b, c.x, c.y, c.z, inv_h2, bc);
}

template void launch_gs_blkf<float>(const Dims&, float*, const float*, const Coef<float>&, float, int, int,
                                    const float*, hipStream_t);
template void launch_gs_blkf<double>(const Dims&, double*, const double*, const Coef<double>&, double, int, int,
                                     const double*, hipStream_t);
template void launch_rr_blkf<float>(const Dims&, const float*, const float*, const Coef<float>&, float, float*,
                                    hipStream_t);
template void launch_rr_blkf<double>(const Dims&, const double*, const double*, const Coef<double>&, double, double*,
                                     hipStream_t);

}  // namespace mp
