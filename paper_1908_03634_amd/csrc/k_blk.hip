// k_blk.hip -- register-blocked finest-level kernels (cell-value coefficients).
//
// A 7-point stencil with one cell per thread issues about eleven memory
// instructions per cell (centre and in-plane neighbours of the iterate and of
// the coefficients, the right-hand side, the store), most of them misaligned
// by one element; on gfx950 that instruction stream, not HBM bandwidth, is
// what limits such kernels.  Here every lane owns a strip of 2M consecutive
// cells of a row (M = 1..4: one or two 8/16-byte accesses per row) in R
// consecutive rows, and marches along z:
//   * x neighbours inside the strip are registers; across strips they come
//     from the adjacent lanes by whole-wavefront DPP rotations.  A wavefront
//     covers 128 M columns: when that is the whole row the rotation also
//     closes a periodic wrap; otherwise lanes 0 and 63 load one halo column;
//   * y neighbours are the lane's own rows plus one halo row on each side;
//   * z neighbours stay in registers from the previous and next planes.
// Every cell is evaluated with the shared per-cell arithmetic of the
// one-cell-per-thread kernels (same operands, same order), so results agree
// bit for bit.
//
// Shape: 256-thread blocks of 4 wavefronts; block (bx, by, bz) covers columns
// [128 M bx, 128 M (bx + 1)), rows [4R by, 4R (by + 1)) (R per wavefront) and
// planes [lz bz, lz (bz + 1)).  Requires nx % 128 == 0, ny % 4 == 0 and an
// even nz >= 4; arrays 16-byte aligned.
#include "mp_blk.h"
#include "mp_device.h"
#include "mp_kernels.h"

#include <hip/hip_ext.h>

namespace mp {

bool blk_supported(const Dims& d) { return d.nx % 128 == 0 && d.ny % 4 == 0 && d.nz >= 4 && d.nz % 2 == 0; }

// ------------------------------------------------------------------ smoother

// One colour of red-black Gauss-Seidel, in place (modes: mp_kernels.h).  In
// GS_E_ALL the cells of the other colour are written back as read (without
// the correction): only the updated cells keep x + e, and GS_E_OWN adds e to
// the cells of the second colour, so every cell receives e exactly once.
// IRU (FP32 only, last pass of a V-cycle): also phi += s[0] * x on every
// cell (the refinement update, otherwise a separate pass).
template <typename T, int MODE, int M, int R, bool IRU>
__global__ __launch_bounds__(BK_T) void k_gs_blk(Dims d, int lz, T* __restrict__ x, const T* __restrict__ b,
                                                const T* __restrict__ cc, T h2, int colour, const T* __restrict__ ec,
                                                double* __restrict__ phi, const double* __restrict__ irs)
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
    // parent corrections of a strip / of one column
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

    S xm[R], x0[R], cm[R], c0[R];
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
            cm[t] = ld_strip<T, M>(cc, bm + roff[t + 1] + g.xi);
            c0[t] = ld_strip<T, M>(cc, b0 + roff[t + 1] + g.xi);
        }
    }
    // Loads for plane k (b, halo rows and column) and k+1 (z+ neighbours),
    // issued one plane ahead of their use.
    struct Ld {
        S xp[R], cp[R], bq[R], xlo, xhi, clo, chi;
        E ep[R], eo[R];
        T hx[R], hc[R];
    };
    auto load = [&](int k) -> Ld {
        Ld L;
        const int kp = wrap_plane(d, k + 1);
        const long long bk = (long long)k * sz, bp = (long long)kp * sz;
        L.clo = ld_strip<T, M>(cc, bk + roff[0] + g.xi);
        L.chi = ld_strip<T, M>(cc, bk + roff[R + 1] + g.xi);
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
#pragma unroll
        for (int t = 0; t < R; t++) {
            L.xp[t] = ZI ? zero_strip<T, M>() : ld_strip<T, M>(x, bp + roff[t + 1] + g.xi);
            if constexpr (EA) L.ep[t] = epar(kp, rows[t + 1]);
            if constexpr (MODE == GS_E_OWN) L.eo[t] = epar(k, rows[t + 1]);
            L.cp[t] = ld_strip<T, M>(cc, bp + roff[t + 1] + g.xi);
            L.bq[t] = ld_strip<T, M>(b, bk + roff[t + 1] + g.xi);
            L.hx[t] = T(0);
            L.hc[t] = T(0);
            if (g.hal) {
                L.hc[t] = cc[bk + roff[t + 1] + g.hcol];
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
        const S(&xp)[R] = cur.xp;
        const S(&cp)[R] = cur.cp;
        const S(&bq)[R] = cur.bq;
        const E(&ep)[R] = cur.ep;
        const T(&hx)[R] = cur.hx;
        const T(&hc)[R] = cur.hc;
        const S &xlo = cur.xlo, &xhi = cur.xhi, &clo = cur.clo, &chi = cur.chi;
        if constexpr (MODE == GS_E_OWN) {
#pragma unroll
            for (int t = 0; t < R; t++) e0[t] = cur.eo[t];
        }
        T fy[R + 1][2 * M];
        y_faces<T, M, R>(g, c0, clo, chi, fy);
        // rows as their neighbours see them
        S nv[R];
#pragma unroll
        for (int t = 0; t < R; t++) nv[t] = EA ? add_e(x0[t], e0[t]) : x0[t];
#pragma unroll
        for (int t = 0; t < R; t++) {
            T fx[2 * M + 1];
            x_faces<T, M>(g, c0[t], hc[t], fx);
            T vl, vr;
            x_edges<T, M>(g, nv[t], hx[t], vl, vr);
            const S zl = EA ? add_e(xm[t], em[t]) : xm[t];
            const S zh = EA ? add_e(xp[t], ep[t]) : xp[t];
            const S& ylo = t > 0 ? nv[t > 0 ? t - 1 : 0] : xlo;
            const S& yhi = t < R - 1 ? nv[t < R - 1 ? t + 1 : 0] : xhi;
            S out = x0[t];
            const int first = (colour + g.j0 + t + k) & 1;  // first updated cell of the strip
            auto upd = [&](int q) {
                const T own = EO ? x0[t].v[q] + e0[t].e[q >> 1] : x0[t].v[q];
                const CellIn<T> s = cell_in<T, M, R>(q, t, g, hzm, hzp, fx, fy, c0[t], cm[t], cp[t], nv[t], vl, vr,
                                                     ylo, yhi, zl, zh, own);
                out.v[q] = gs_value<T>(s.c[0], s.c[1], s.c[2], s.c[3], s.c[4], s.c[5], s.v[0], s.v[1], s.v[2], s.v[3],
                                       s.v[4], s.v[5], bq[t].v[q], h2, own);
            };
            if (first == 0) {
#pragma unroll
                for (int q = 0; q < 2 * M; q += 2) upd(q);
            } else {
#pragma unroll
                for (int q = 1; q < 2 * M; q += 2) upd(q);
            }
            st_strip<T, M>(x, bk + roff[t + 1] + g.xi, out);
            if constexpr (IRU) {
                const double sc = irs[0];
                double* pp = phi + bk + roff[t + 1] + g.xi;
#pragma unroll
                for (int q = 0; q < M; q++) {
                    const double2 pv = *reinterpret_cast<const double2*>(pp + 2 * q);
                    *reinterpret_cast<double2*>(pp + 2 * q) = make_double2(fma(sc, (double)out.v[2 * q], pv.x),
                                                                           fma(sc, (double)out.v[2 * q + 1], pv.y));
                }
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
        cur = nxt;
    }
}

// ------------------------------------------------- residual and restriction

// One plane's loads shared by the residual kernels.
template <typename T, int M, int R>
struct PlaneIn {
    Strip<T, M> xp[R], cp[R], bq[R], xlo, xhi, clo, chi;
    T hx[R], hc[R];
};

template <typename T, int M, int R>
__device__ __forceinline__ void load_plane(const BlkGeo& g, const T* __restrict__ x, const T* __restrict__ b,
                                           const T* __restrict__ cc, const long long (&roff)[R + 2], long long bk,
                                           long long bp, PlaneIn<T, M, R>& q)
{
    q.xlo = ld_strip<T, M>(x, bk + roff[0] + g.xi);
    q.xhi = ld_strip<T, M>(x, bk + roff[R + 1] + g.xi);
    q.clo = ld_strip<T, M>(cc, bk + roff[0] + g.xi);
    q.chi = ld_strip<T, M>(cc, bk + roff[R + 1] + g.xi);
#pragma unroll
    for (int t = 0; t < R; t++) {
        q.xp[t] = ld_strip<T, M>(x, bp + roff[t + 1] + g.xi);
        q.cp[t] = ld_strip<T, M>(cc, bp + roff[t + 1] + g.xi);
        q.bq[t] = ld_strip<T, M>(b, bk + roff[t + 1] + g.xi);
        q.hx[t] = T(0);
        q.hc[t] = T(0);
        if (g.hal) {
            q.hx[t] = x[bk + roff[t + 1] + g.hcol];
            q.hc[t] = cc[bk + roff[t + 1] + g.hcol];
        }
    }
}

// Residuals b - A x of the strip in every row of plane k.
template <typename T, int M, int R>
__device__ __forceinline__ void plane_resid(const BlkGeo& g, bool hzm, bool hzp, const Strip<T, M> (&xm)[R],
                                            const Strip<T, M> (&x0)[R], const Strip<T, M> (&cm)[R],
                                            const Strip<T, M> (&c0)[R], const PlaneIn<T, M, R>& q, T inv_h2,
                                            Strip<T, M> (&r)[R])
{
    T fy[R + 1][2 * M];
    y_faces<T, M, R>(g, c0, q.clo, q.chi, fy);
#pragma unroll
    for (int t = 0; t < R; t++) {
        T fx[2 * M + 1];
        x_faces<T, M>(g, c0[t], q.hc[t], fx);
        T vl, vr;
        x_edges<T, M>(g, x0[t], q.hx[t], vl, vr);
        const Strip<T, M>& ylo = t > 0 ? x0[t > 0 ? t - 1 : 0] : q.xlo;
        const Strip<T, M>& yhi = t < R - 1 ? x0[t < R - 1 ? t + 1 : 0] : q.xhi;
#pragma unroll
        for (int c = 0; c < 2 * M; c++) {
            const T own = x0[t].v[c];
            const CellIn<T> s = cell_in<T, M, R>(c, t, g, hzm, hzp, fx, fy, c0[t], cm[t], q.cp[t], x0[t], vl, vr, ylo,
                                                 yhi, xm[t], q.xp[t], own);
            r[t].v[c] = resid_value<T>(s.c[0], s.c[1], s.c[2], s.c[3], s.c[4], s.c[5], s.v[0], s.v[1], s.v[2], s.v[3],
                                       s.v[4], s.v[5], own, q.bq[t].v[c], inv_h2);
        }
    }
}

template <typename T, int M, int R>
__device__ __forceinline__ void ring_start(const Dims& d, const BlkGeo& g, const T* __restrict__ x,
                                           const T* __restrict__ cc, const long long (&roff)[R + 2], long long sz,
                                           Strip<T, M> (&xm)[R], Strip<T, M> (&x0)[R], Strip<T, M> (&cm)[R],
                                           Strip<T, M> (&c0)[R])
{
    const long long bm = (long long)wrap_plane(d, g.z0 - 1) * sz, b0 = (long long)g.z0 * sz;
#pragma unroll
    for (int t = 0; t < R; t++) {
        xm[t] = ld_strip<T, M>(x, bm + roff[t + 1] + g.xi);
        x0[t] = ld_strip<T, M>(x, b0 + roff[t + 1] + g.xi);
        cm[t] = ld_strip<T, M>(cc, bm + roff[t + 1] + g.xi);
        c0[t] = ld_strip<T, M>(cc, b0 + roff[t + 1] + g.xi);
    }
}

template <typename T, int M, int R>
__device__ __forceinline__ void ring_shift(Strip<T, M> (&xm)[R], Strip<T, M> (&x0)[R], Strip<T, M> (&cm)[R],
                                           Strip<T, M> (&c0)[R], const PlaneIn<T, M, R>& q)
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
// summed in the order of restrict_cell (z, then y, then x child).  A strip
// holds the x children of M coarse cells; planes are taken in pairs (chunks
// start on even planes), rows in pairs (j0 is even).
template <typename T, int M, int R>
__global__ __launch_bounds__(BK_T) void k_rr_blk(Dims d, int lz, const T* __restrict__ x, const T* __restrict__ b,
                                                const T* __restrict__ cc, T inv_h2, T* __restrict__ bc)
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
    S xm[R], x0[R], cm[R], c0[R];
    ring_start<T, M, R>(d, g, x, cc, roff, sz, xm, x0, cm, c0);
    // each plane's loads are issued one plane ahead of their use
    PlaneIn<T, M, R> cur;
    load_plane<T, M, R>(g, x, b, cc, roff, (long long)g.z0 * sz, (long long)wrap_plane(d, g.z0 + 1) * sz, cur);
    for (int k = g.z0; k < g.z1; k += 2) {
        S r[2][R];  // [z child][row]
#pragma unroll
        for (int cz = 0; cz < 2; cz++) {
            const int kk = k + cz;
            const bool hzm = kk > 0 || d.pz, hzp = kk < d.nz - 1 || d.pz;
            PlaneIn<T, M, R> nxt;
            if (kk + 1 < g.z1)
                load_plane<T, M, R>(g, x, b, cc, roff, (long long)(kk + 1) * sz, (long long)wrap_plane(d, kk + 2) * sz,
                                    nxt);
            plane_resid<T, M, R>(g, hzm, hzp, xm, x0, cm, c0, cur, inv_h2, r[cz]);
            ring_shift<T, M, R>(xm, x0, cm, c0, cur);
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

// FP64 refinement residual r = (b - shift[0]) - A x (shift == nullptr: b as
// stored), its scaled FP32 copy r32 = float(r * inv_s[0]) (when r32 !=
// nullptr) and per-block sums of r^2.
template <int M, int R>
__global__ __launch_bounds__(BK_T) void k_resid64_blk(Dims d, int lz, const double* __restrict__ x,
                                                     const double* __restrict__ b, const double* __restrict__ cc,
                                                     double inv_h2, float* __restrict__ r32,
                                                     const double* __restrict__ inv_s, double* partials,
                                                     const double* __restrict__ shift)
{
    using S = Strip<double, M>;
    __shared__ double sh[BK_W];
    const BlkGeo g = blk_geo<M, R>(d, lz);
    double acc = 0.0;
    if (g.live) {
        const double is = r32 ? inv_s[0] : 0.0;
        const double m = shift ? shift[0] : 0.0;
        const long long sz = (long long)d.nx * d.ny;
        long long roff[R + 2];
#pragma unroll
        for (int t = 0; t < R + 2; t++) roff[t] = (long long)wrap_row(d, g.j0 - 1 + t) * d.nx;
        S xm[R], x0[R], cm[R], c0[R];
        ring_start<double, M, R>(d, g, x, cc, roff, sz, xm, x0, cm, c0);
        PlaneIn<double, M, R> q;  // loads issued one plane ahead of their use
        load_plane<double, M, R>(g, x, b, cc, roff, (long long)g.z0 * sz, (long long)wrap_plane(d, g.z0 + 1) * sz, q);
        for (int k = g.z0; k < g.z1; k++) {
            const bool hzm = k > 0 || d.pz, hzp = k < d.nz - 1 || d.pz;
            const long long bk = (long long)k * sz;
            PlaneIn<double, M, R> nxt;
            if (k + 1 < g.z1)
                load_plane<double, M, R>(g, x, b, cc, roff, (long long)(k + 1) * sz, (long long)wrap_plane(d, k + 2) * sz,
                                         nxt);
            // b - m: the bits of a right-hand side stored with its mean removed
#pragma unroll
            for (int t = 0; t < R; t++)
#pragma unroll
                for (int c = 0; c < 2 * M; c++) q.bq[t].v[c] = q.bq[t].v[c] - m;
            S r[R];
            plane_resid<double, M, R>(g, hzm, hzp, xm, x0, cm, c0, q, inv_h2, r);
#pragma unroll
            for (int t = 0; t < R; t++) {
                Strip<float, M> f;
#pragma unroll
                for (int c = 0; c < 2 * M; c++) {
                    acc = fma(r[t].v[c], r[t].v[c], acc);
                    f.v[c] = (float)(r[t].v[c] * is);
                }
                if (r32) st_strip<float, M>(r32, bk + roff[t + 1] + g.xi, f);
            }
            ring_shift<double, M, R>(xm, x0, cm, c0, q);
            q = nxt;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// ------------------------------------------------------------------ launches

constexpr int kResidPairs = 1;  // FP64 residual strip width (pairs)

int blk_reduce_blocks(const Dims& d)
{
    int lz;
    const dim3 g = blk_grid(d, kResidPairs, rows_for<double>(kResidPairs), kBlkMinBlocks, kMaxRedBlocks, lz);
    return (int)(g.x * g.y * g.z);
}

// Launch timing: when ev0 != nullptr the launch records its start and end
// in (ev0, ev1) (timestamps of the dispatch itself, no extra stream markers).
struct LaunchEv {
    hipEvent_t ev0, ev1;
};

template <typename T, int MODE, int M, bool IRU>
static void gs_launch(const Dims& d, T* x, const T* b, const T* cc, T h2, int colour, const T* ec, double* phi,
                      const double* irs, LaunchEv ev, hipStream_t s)
{
    constexpr int R = rows_for<T>(M);
    int lz;
    const dim3 grid = blk_grid(d, M, R, kBlkMinBlocks, 1LL << 30, lz);
    if (ev.ev0)
        hipExtLaunchKernelGGL((k_gs_blk<T, MODE, M, R, IRU>), grid, dim3(BK_T), 0, s, ev.ev0, ev.ev1, 0, d, lz, x, b,
                              cc, h2, colour, ec, phi, irs);
    else
        hipLaunchKernelGGL((k_gs_blk<T, MODE, M, R, IRU>), grid, dim3(BK_T), 0, s, d, lz, x, b, cc, h2, colour, ec,
                           phi, irs);
}

template <typename T, int M, bool IRU>
static void gs_mode(int mode, const Dims& d, T* x, const T* b, const T* cc, T h2, int colour, const T* ec,
                    double* phi, const double* irs, LaunchEv ev, hipStream_t s)
{
    if constexpr (IRU) {
        // the refinement update rides on the last pass of a V-cycle: colour 1
        // of a plain sweep, or of the first sweep after prolongation
        if (mode == GS_E_OWN) gs_launch<T, GS_E_OWN, M, true>(d, x, b, cc, h2, colour, ec, phi, irs, ev, s);
        else gs_launch<T, GS_PLAIN, M, true>(d, x, b, cc, h2, colour, ec, phi, irs, ev, s);
        return;
    }
    switch (mode) {
    case GS_ZERO: gs_launch<T, GS_ZERO, M, false>(d, x, b, cc, h2, colour, ec, phi, irs, ev, s); break;
    case GS_E_ALL: gs_launch<T, GS_E_ALL, M, false>(d, x, b, cc, h2, colour, ec, phi, irs, ev, s); break;
    case GS_E_OWN: gs_launch<T, GS_E_OWN, M, false>(d, x, b, cc, h2, colour, ec, phi, irs, ev, s); break;
    default: gs_launch<T, GS_PLAIN, M, false>(d, x, b, cc, h2, colour, ec, phi, irs, ev, s); break;
    }
}

template <typename T, bool IRU>
static void gs_width(int mode, const Dims& d, T* x, const T* b, const T* cc, T h2, int colour, const T* ec,
                     double* phi, const double* irs, LaunchEv ev, hipStream_t s)
{
    if constexpr (sizeof(T) == 8) {
        gs_mode<T, 1, IRU>(mode, d, x, b, cc, h2, colour, ec, phi, irs, ev, s);  // FP64: pairs
    } else {
        switch (strip_pairs(d)) {
        case 4: gs_mode<T, 4, IRU>(mode, d, x, b, cc, h2, colour, ec, phi, irs, ev, s); break;
        case 3: gs_mode<T, 3, IRU>(mode, d, x, b, cc, h2, colour, ec, phi, irs, ev, s); break;
        case 2: gs_mode<T, 2, IRU>(mode, d, x, b, cc, h2, colour, ec, phi, irs, ev, s); break;
        default: gs_mode<T, 1, IRU>(mode, d, x, b, cc, h2, colour, ec, phi, irs, ev, s); break;
        }
    }
}

template <typename T>
void launch_gs_blk(const Dims& d, T* x, const T* b, const T* cc, T h2, int colour, int mode, const T* ec,
                   double* phi, const double* irs, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s)
{
    const LaunchEv ev{ev0, ev1};
    if constexpr (sizeof(T) == 4) {
        if (phi) {
            gs_width<T, true>(mode, d, x, b, cc, h2, colour, ec, phi, irs, ev, s);
            return;
        }
    }
    gs_width<T, false>(mode, d, x, b, cc, h2, colour, ec, nullptr, nullptr, ev, s);
}

template <typename T, int M>
static void rr_launch(const Dims& d, const T* x, const T* b, const T* cc, T inv_h2, T* bc, hipStream_t s)
{
    constexpr int R = rows_for<T>(M);
    int lz;
    const dim3 grid = blk_grid(d, M, R, kBlkMinBlocks, 1LL << 30, lz);
    hipLaunchKernelGGL((k_rr_blk<T, M, R>), grid, dim3(BK_T), 0, s, d, lz, x, b, cc, inv_h2, bc);
}

template <typename T>
void launch_rr_blk(const Dims& d, const T* x, const T* b, const T* cc, T inv_h2, T* bc, hipStream_t s)
{
    if constexpr (sizeof(T) == 8) {
        rr_launch<T, 1>(d, x, b, cc, inv_h2, bc, s);
    } else {
        switch (strip_pairs(d)) {
        case 4: rr_launch<T, 4>(d, x, b, cc, inv_h2, bc, s); break;
        case 3: rr_launch<T, 3>(d, x, b, cc, inv_h2, bc, s); break;
        case 2: rr_launch<T, 2>(d, x, b, cc, inv_h2, bc, s); break;
        default: rr_launch<T, 1>(d, x, b, cc, inv_h2, bc, s); break;
        }
    }
}

void launch_resid64_blk(const Dims& d, const double* x, const double* b, const double* cc, double inv_h2, float* r32,
                        const double* inv_s, double* partials, int* nb_out, hipStream_t s, const double* shift)
{
    constexpr int R = rows_for<double>(kResidPairs);
    int lz;
    const dim3 grid = blk_grid(d, kResidPairs, R, kBlkMinBlocks, kMaxRedBlocks, lz);
    *nb_out = (int)(grid.x * grid.y * grid.z);
    hipLaunchKernelGGL((k_resid64_blk<kResidPairs, R>), grid, dim3(BK_T), 0, s, d, lz, x, b, cc, inv_h2, r32, inv_s,
                       partials, shift);
}

template void launch_gs_blk<float>(const Dims&, float*, const float*, const float*, float, int, int, const float*,
                                   double*, const double*, hipEvent_t, hipEvent_t, hipStream_t);
template void launch_gs_blk<double>(const Dims&, double*, const double*, const double*, double, int, int,
                                    const double*, double*, const double*, hipEvent_t, hipEvent_t, hipStream_t);
template void launch_rr_blk<float>(const Dims&, const float*, const float*, const float*, float, float*, hipStream_t);
template void launch_rr_blk<double>(const Dims&, const double*, const double*, const double*, double, double*,
                                    hipStream_t);

}  // namespace mp
