// k_fsweep.hip -- both colours of a red-black Gauss-Seidel sweep in one pass
// over the finest level (register-blocked strips, out of place).
//
// A sweep updates every red cell (i + j + k even) from the old black values,
// then every black cell from the new red values.  Done as two passes, each
// pass streams the iterate, the right-hand side and the coefficients through
// HBM once; here one pass does both.  A wavefront owns R rows of a plane and
// marches along z, updating red on plane k+1 and then black on plane k:
//   * black on plane k needs new red values in its own rows, in the rows
//     just outside them (owned by other wavefronts) and on planes k-1 and
//     k+1; the wavefront therefore computes red for R + 2 rows (one halo row
//     on each side, recomputed rather than exchanged), which needs the old
//     values of R + 4 rows;
//   * the planes it keeps in registers are k-1 (final), k (new red), k+1
//     (old, then new red) and k+2 (old, loaded at the top of the step);
//   * a plane chunk starts by computing red on its first two planes.
// The sweep reads the old iterate `xo` and writes `xn`: a wavefront reads
// old values of rows and planes that other wavefronts write.  Every cell is
// evaluated with the shared per-cell arithmetic (`harm`, `gs_value`), in the
// operand order of the one-cell kernels, so the result equals two colour
// passes bit for bit.  Used when one wavefront spans a row (nx = 128 M,
// M <= 2).
#include "mp_blk.h"
#include "mp_device.h"
#include "mp_kernels.h"

#include <hip/hip_ext.h>

namespace mp {

bool fsw_supported(const Dims& d) { return blk_supported(d) && (d.nx == 128 || d.nx == 256); }

// Red (colour 0) update of rows 1 .. R+2 of plane P, in place in x.
// x, c: rows j0-2 .. j0+R+1 of plane P.  xb/cb (below, plane P-1) and xa/ca
// (above, plane P+1) hold row j0-2+t at index t-1+OB / t-1+OA.  bq: rows
// j0-1 .. j0+R.
template <typename T, int M, int R, int OB, int NB, int OA, int NA>
__device__ __forceinline__ void fs_red(const Dims& d, const BlkGeo& g, int P, T h2, Strip<T, M> (&x)[R + 4],
                                       const Strip<T, M> (&c)[R + 4], const Strip<T, M> (&xb)[NB],
                                       const Strip<T, M> (&cb)[NB], const Strip<T, M> (&xa)[NA],
                                       const Strip<T, M> (&ca)[NA], const Strip<T, M> (&bq)[R + 2])
{
    constexpr int NH = R + 4;
    const bool hzm = P > 0 || d.pz, hzp = P < d.nz - 1 || d.pz;
    T fy[NH][2 * M];  // fy[t]: face between rows t-1 and t
#pragma unroll
    for (int t = 1; t < NH; t++) {
        const int j = g.j0 - 2 + t;
        const bool has = (j > 0 || d.py) && (j < d.ny || d.py);
#pragma unroll
        for (int q = 0; q < 2 * M; q++) fy[t][q] = has ? harm(c[t - 1].v[q], c[t].v[q]) : T(0);
    }
#pragma unroll
    for (int t = 1; t <= R + 2; t++) {
        const int j = g.j0 - 2 + t;
        T fx[2 * M + 1];
        x_faces<T, M>(g, c[t], T(0), fx);
        T vl, vr;
        x_edges<T, M>(g, x[t], T(0), vl, vr);
        const bool ywl = !(j > 0 || d.py), ywh = !(j < d.ny - 1 || d.py);
        Strip<T, M> out = x[t];
        auto upd = [&](int q) {
            const T own = x[t].v[q];
            const T c4 = hzm ? harm(cb[t - 1 + OB].v[q], c[t].v[q]) : T(0);
            const T c5 = hzp ? harm(c[t].v[q], ca[t - 1 + OA].v[q]) : T(0);
            const T xm = q > 0 ? x[t].v[q > 0 ? q - 1 : 0] : (g.wl ? own : vl);
            const T xp = q < 2 * M - 1 ? x[t].v[q < 2 * M - 1 ? q + 1 : 0] : (g.wr ? own : vr);
            const T ym = ywl ? own : x[t - 1].v[q];
            const T yp = ywh ? own : x[t + 1].v[q];
            const T zm = hzm ? xb[t - 1 + OB].v[q] : own;
            const T zp = hzp ? xa[t - 1 + OA].v[q] : own;
            out.v[q] = gs_value<T>(fx[q], fx[q + 1], fy[t][q], fy[t + 1][q], c4, c5, xm, xp, ym, yp, zm, zp,
                                   bq[t - 1].v[q], h2, own);
        };
        if (((j + P) & 1) == 0) {
#pragma unroll
            for (int q = 0; q < 2 * M; q += 2) upd(q);
        } else {
#pragma unroll
            for (int q = 1; q < 2 * M; q += 2) upd(q);
        }
        x[t] = out;  // rows t+1.. read only black cells of row t
    }
}

// FS_ZERO: the old iterate is zero (not read).  FS_PROLONG: every old value
// is taken as x + e of its parent coarse cell (ec: coarse correction), i.e.
// the prolongation is applied on the fly.  IRU (FP32): also phi += irs[0] x.
template <typename T, int MODE, int M, int R, bool IRU>
__global__ __launch_bounds__(BK_T) void k_fsw_blk(Dims d, int lz, const T* __restrict__ xo, T* __restrict__ xn,
                                                  const T* __restrict__ b, const T* __restrict__ cc, T h2,
                                                  const T* __restrict__ ec, double* __restrict__ phi,
                                                  const double* __restrict__ irs)
{
    using S = Strip<T, M>;
    constexpr bool ZI = MODE == FS_ZERO;
    constexpr bool EC = MODE == FS_PROLONG;
    constexpr int NH = R + 4;
    const BlkGeo g = blk_geo<M, R>(d, lz);
    if (!g.live) return;
    const long long sz = (long long)d.nx * d.ny;
    const int nxc = d.nx >> 1;
    const long long szc = (long long)nxc * (d.ny >> 1);
    int rows[NH];
    long long roff[NH];
#pragma unroll
    for (int t = 0; t < NH; t++) {
        rows[t] = wrap_row(d, g.j0 - 2 + t);
        roff[t] = (long long)rows[t] * d.nx;
    }
    auto ldx = [&](int kk, int t) -> S {
        if constexpr (ZI) {
            return zero_strip<T, M>();
        } else {
            S v = ld_strip<T, M>(xo, (long long)kk * sz + roff[t] + g.xi);
            if constexpr (EC) {
                const long long o = (long long)(kk >> 1) * szc + (long long)(rows[t] >> 1) * nxc + (g.xi >> 1);
#pragma unroll
                for (int q = 0; q < 2 * M; q++) v.v[q] = v.v[q] + ec[o + (q >> 1)];
            }
            return v;
        }
    };
    auto ldc = [&](int kk, int t) -> S { return ld_strip<T, M>(cc, (long long)kk * sz + roff[t] + g.xi); };
    auto ldb = [&](int kk, int t) -> S { return ld_strip<T, M>(b, (long long)kk * sz + roff[t] + g.xi); };

    // ---- prologue: red on planes z0-1 and z0
    S xC[R], cC[R], xB[R + 2], cB[R + 2], bB[R], xA[NH], cA[NH];
    {
        const int pm2 = wrap_plane(d, g.z0 - 2), pm1 = wrap_plane(d, g.z0 - 1), p0 = g.z0,
                  p1 = wrap_plane(d, g.z0 + 1);
        S x2[R + 2], c2[R + 2], x1[NH], c1[NH], b1[R + 2], x0[NH], c0[NH], b0[R + 2];
#pragma unroll
        for (int t = 0; t < R + 2; t++) {
            x2[t] = ldx(pm2, t + 1);
            c2[t] = ldc(pm2, t + 1);
            b1[t] = ldb(pm1, t + 1);
            b0[t] = ldb(p0, t + 1);
        }
#pragma unroll
        for (int t = 0; t < NH; t++) {
            x1[t] = ldx(pm1, t);
            c1[t] = ldc(pm1, t);
            x0[t] = ldx(p0, t);
            c0[t] = ldc(p0, t);
            xA[t] = ldx(p1, t);
            cA[t] = ldc(p1, t);
        }
        fs_red<T, M, R, 0, R + 2, 1, NH>(d, g, g.z0 - 1, h2, x1, c1, x2, c2, x0, c0, b1);
        fs_red<T, M, R, 1, NH, 1, NH>(d, g, g.z0, h2, x0, c0, x1, c1, xA, cA, b0);
#pragma unroll
        for (int t = 0; t < R; t++) {
            xC[t] = x1[t + 2];
            cC[t] = c1[t + 2];
            bB[t] = b0[t + 1];
        }
#pragma unroll
        for (int t = 0; t < R + 2; t++) {
            xB[t] = x0[t + 1];
            cB[t] = c0[t + 1];
        }
    }

    for (int k = g.z0; k < g.z1; k++) {
        const int k1 = wrap_plane(d, k + 1), k2 = wrap_plane(d, k + 2);
        S xD[NH], cD[NH], bA[R + 2];
#pragma unroll
        for (int t = 0; t < NH; t++) {
            xD[t] = ldx(k2, t);
            cD[t] = ldc(k2, t);
        }
#pragma unroll
        for (int t = 0; t < R + 2; t++) bA[t] = ldb(k1, t + 1);
        // red on plane k+1 (old black of planes k, k+1, k+2)
        fs_red<T, M, R, 0, R + 2, 1, NH>(d, g, k + 1, h2, xA, cA, xB, cB, xD, cD, bA);
        // black on plane k (new red of planes k-1, k, k+1)
        const bool hzm = k > 0 || d.pz, hzp = k < d.nz - 1 || d.pz;
        const long long bk = (long long)k * sz;
        T fy[R + 2][2 * M];  // fy[t]: face between rows t-1 and t of xB (row j0-1+t)
#pragma unroll
        for (int t = 1; t <= R + 1; t++) {
            const int j = g.j0 - 1 + t;
            const bool has = (j > 0 || d.py) && (j < d.ny || d.py);
#pragma unroll
            for (int q = 0; q < 2 * M; q++) fy[t][q] = has ? harm(cB[t - 1].v[q], cB[t].v[q]) : T(0);
        }
#pragma unroll
        for (int t = 1; t <= R; t++) {
            const int j = g.j0 - 1 + t;
            T fx[2 * M + 1];
            x_faces<T, M>(g, cB[t], T(0), fx);
            T vl, vr;
            x_edges<T, M>(g, xB[t], T(0), vl, vr);
            const bool ywl = !(j > 0 || d.py), ywh = !(j < d.ny - 1 || d.py);
            S out = xB[t];
            auto upd = [&](int q) {
                const T own = xB[t].v[q];
                const T c4 = hzm ? harm(cC[t - 1].v[q], cB[t].v[q]) : T(0);
                const T c5 = hzp ? harm(cB[t].v[q], cA[t + 1].v[q]) : T(0);
                const T xm = q > 0 ? xB[t].v[q > 0 ? q - 1 : 0] : (g.wl ? own : vl);
                const T xp = q < 2 * M - 1 ? xB[t].v[q < 2 * M - 1 ? q + 1 : 0] : (g.wr ? own : vr);
                const T ym = ywl ? own : xB[t - 1].v[q];
                const T yp = ywh ? own : xB[t + 1].v[q];
                const T zm = hzm ? xC[t - 1].v[q] : own;
                const T zp = hzp ? xA[t + 1].v[q] : own;
                out.v[q] = gs_value<T>(fx[q], fx[q + 1], fy[t][q], fy[t + 1][q], c4, c5, xm,
                                       xp, ym, yp, zm, zp, bB[t - 1].v[q], h2, own);
            };
            if (((1 + j + k) & 1) == 0) {
#pragma unroll
                for (int q = 0; q < 2 * M; q += 2) upd(q);
            } else {
#pragma unroll
                for (int q = 1; q < 2 * M; q += 2) upd(q);
            }
            xB[t] = out;
            st_strip<T, M>(xn, bk + roff[t + 1] + g.xi, out);
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
        // rotate: k-1 <- k (own rows, final), k <- k+1, k+1 <- k+2
#pragma unroll
        for (int t = 0; t < R; t++) {
            xC[t] = xB[t + 1];
            cC[t] = cB[t + 1];
            bB[t] = bA[t + 1];
        }
#pragma unroll
        for (int t = 0; t < R + 2; t++) {
            xB[t] = xA[t + 1];
            cB[t] = cA[t + 1];
        }
#pragma unroll
        for (int t = 0; t < NH; t++) {
            xA[t] = xD[t];
            cA[t] = cD[t];
        }
    }
}

// Rows per wavefront: 2 for pairs, 1 for strips of 4 (register budget).
template <int M>
constexpr int fsw_rows()
{
    return M == 1 ? 2 : 1;
}

template <typename T, int MODE, int M, bool IRU>
static void fsw_launch(const Dims& d, const T* xo, T* xn, const T* b, const T* cc, T h2, const T* ec, double* phi,
                       const double* irs, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s)
{
    constexpr int R = fsw_rows<M>();
    int lz;
    const dim3 grid = blk_grid(d, M, R, kBlkMinBlocks, 1LL << 30, lz);
    if (ev0)
        hipExtLaunchKernelGGL((k_fsw_blk<T, MODE, M, R, IRU>), grid, dim3(BK_T), 0, s, ev0, ev1, 0, d, lz, xo, xn, b,
                              cc, h2, ec, phi, irs);
    else
        hipLaunchKernelGGL((k_fsw_blk<T, MODE, M, R, IRU>), grid, dim3(BK_T), 0, s, d, lz, xo, xn, b, cc, h2, ec, phi,
                           irs);
}

template <typename T, int M>
static void fsw_mode(int mode, const Dims& d, const T* xo, T* xn, const T* b, const T* cc, T h2, const T* ec,
                     double* phi, const double* irs, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s)
{
    if constexpr (sizeof(T) == 4) {
        if (phi) {
            // the refinement update rides on the last sweep of a V-cycle
            if (mode == FS_PROLONG)
                fsw_launch<T, FS_PROLONG, M, true>(d, xo, xn, b, cc, h2, ec, phi, irs, ev0, ev1, s);
            else
                fsw_launch<T, FS_PLAIN, M, true>(d, xo, xn, b, cc, h2, ec, phi, irs, ev0, ev1, s);
            return;
        }
    }
    switch (mode) {
    case FS_ZERO: fsw_launch<T, FS_ZERO, M, false>(d, xo, xn, b, cc, h2, ec, nullptr, nullptr, ev0, ev1, s); break;
    case FS_PROLONG:
        fsw_launch<T, FS_PROLONG, M, false>(d, xo, xn, b, cc, h2, ec, nullptr, nullptr, ev0, ev1, s);
        break;
    default: fsw_launch<T, FS_PLAIN, M, false>(d, xo, xn, b, cc, h2, ec, nullptr, nullptr, ev0, ev1, s); break;
    }
}

template <typename T>
void launch_fsw_blk(const Dims& d, const T* xo, T* xn, const T* b, const T* cc, T h2, int mode, const T* ec,
                    double* phi, const double* irs, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s)
{
    if (d.nx == 256) fsw_mode<T, 2>(mode, d, xo, xn, b, cc, h2, ec, phi, irs, ev0, ev1, s);
    else fsw_mode<T, 1>(mode, d, xo, xn, b, cc, h2, ec, phi, irs, ev0, ev1, s);
}

template void launch_fsw_blk<float>(const Dims&, const float*, float*, const float*, const float*, float, int,
                                    const float*, double*, const double*, hipEvent_t, hipEvent_t, hipStream_t);

}  // namespace mp
