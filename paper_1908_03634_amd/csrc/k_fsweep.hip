// k_fsweep.hip -- both colours of a red-black Gauss-Seidel sweep in one pass
// over the finest level (whole rows, out of place, rows exchanged in LDS).
//
// A sweep updates every red cell (i + j + k even) from the old black values,
// then every black cell from the new red values.  As two colour passes it
// streams the iterate, the right-hand side and the coefficients through HBM
// twice (32 bytes per cell in FP32); here one pass does both (16 bytes).
//
// Wavefront w of a workgroup holds row j0 - 2 + w of every plane (a whole
// row: nx = 128 M, 2M cells per lane), so the R + 4 wavefronts span the R
// owned rows, one row on each side whose red is recomputed and one more on
// each side that only supplies old values.  The workgroup marches along z
// through a chunk of planes; each wavefront keeps its own cells of planes
// k-1 .. k+2 (and the planes being prefetched) in registers, and a row's y
// neighbours come from the other wavefronts through three LDS plane buffers
// (x and c), used in turn.  Plane step k (planes z0-2 .. z1-1 of the chunk):
//   1. prefetch x and c of plane k+2+D and b of plane k+1+D;
//   2. publish the old x and c of plane k+1 in its buffer; barrier;
//   3. red on plane k+1 (rows j0-1 .. j0+R), written back to the buffer: the
//      other red rows read only the black cells of the row, which keep their
//      values;
//   4. black on plane k (rows j0 .. j0+R-1) from the new red of plane k (the
//      neighbour rows, published in step 3 of the previous plane step and
//      made visible by this step's barrier) and of planes k-1 and k+1 (own
//      registers); stored to xn.
// A buffer is filled again two plane steps after its black reads, with a
// barrier between, so one barrier per plane step suffices.  The chunk starts
// two planes early (red only on planes z0-1 and z0).  The sweep reads the old
// iterate xo and writes xn: other workgroups read old values of the rows and
// planes this one writes.  Each cell is evaluated with the shared per-cell
// arithmetic (harm, gs_value) in the operand order of the colour passes, so
// the result equals two colour passes bit for bit.
#include "mp_blk.h"
#include "mp_device.h"
#include "mp_kernels.h"

#include <hip/hip_ext.h>

namespace mp {

bool fsw_supported(const Dims& d)
{
    return blk_supported(d) && (d.nx == 128 || d.nx == 256 || d.nx == 384 || d.nx == 512);
}

// Rows of 192 cells between walls in x (the 384^3 box's second level): the
// strips of 256-cell rows, lanes 48-63 past the row's end idle (they load the
// row's first cells, and store nothing).
bool fsw_narrow_supported(const Dims& d)
{
    return d.nx == 192 && !d.px && d.ny % 4 == 0 && d.nz >= 4 && d.nz % 2 == 0;
}

// The M cells of one parity (q even or q odd) of a lane's strip.
template <typename T, int M>
struct Half {
    T v[M];
};

// One colour (par 0: red, 1: black) of row j of plane P, in place in x.
// xlo/xhi: the cells of the colour's parity in rows j-1 and j+1 of plane P
// (the update of cell q reads element q / 2); xb and xa: this row on planes
// P-1 and P+1; fx: the x faces of the row.
// CELL (cell coefficients): c is the row's coefficients, clo/chi those of
// rows j-1 and j+1 (colour parity), fzl/fzh the z faces below and above
// (z_faces of planes P-1 and P).
// Stored faces: c is the row's low y faces, chi the low y faces of row j+1
// (colour parity), fzl/fzh the low z faces of planes P and P+1; a high face
// across a wall is 0 (fyh, zh), the low faces are taken as stored.
// PXY: x and y periodic (no wall in the row or between rows; the selects
// for walls drop out at compile time).
template <typename T, int M, bool CELL, bool PXY>
__device__ __forceinline__ void fs_row(const Dims& d, const BlkGeo& g, int j, int P, int par, T h2, Strip<T, M>& x,
                                       const Half<T, M>& xlo, const Half<T, M>& xhi, const Strip<T, M>& xb,
                                       const Strip<T, M>& xa, const T (&fx)[2 * M + 1], const Strip<T, M>& c,
                                       const Half<T, M>& clo, const Half<T, M>& chi, const Strip<T, M>& fzl,
                                       const Strip<T, M>& fzh, const Strip<T, M>& bq)
{
    const bool hzm = P > 0 || d.pz, hzp = P < d.nz - 1 || d.pz;
    const bool fyl = PXY || ((j > 0 || d.py) && (j < d.ny || d.py));
    const bool fyh = PXY || ((j + 1 > 0 || d.py) && (j + 1 < d.ny || d.py));
    const bool ywl = !PXY && !(j > 0 || d.py), ywh = !PXY && !(j < d.ny - 1 || d.py);
    T vl, vr;
    x_edges<T, M>(g, x, T(0), vl, vr);
    Strip<T, M> out = x;
    auto upd = [&](int q) {
        const T own = x.v[q];
        T fl, fh, c5;
        if constexpr (CELL) {
            fl = fyl ? harm(clo.v[q >> 1], c.v[q]) : T(0);
            fh = fyh ? harm(c.v[q], chi.v[q >> 1]) : T(0);
            c5 = fzh.v[q];
        } else {
            fl = c.v[q];
            fh = fyh ? chi.v[q >> 1] : T(0);
            c5 = hzp ? fzh.v[q] : T(0);
        }
        const T xm = q > 0 ? x.v[q > 0 ? q - 1 : 0] : (!PXY && g.wl ? own : vl);
        const T xp = q < 2 * M - 1 ? x.v[q < 2 * M - 1 ? q + 1 : 0] : (!PXY && g.wr ? own : vr);
        const T ym = ywl ? own : xlo.v[q >> 1];
        const T yp = ywh ? own : xhi.v[q >> 1];
        const T zm = hzm ? xb.v[q] : own;
        const T zp = hzp ? xa.v[q] : own;
        out.v[q] = gs_value<T>(fx[q], fx[q + 1], fl, fh, fzl.v[q], c5, xm, xp, ym, yp, zm, zp, bq.v[q], h2, own);
    };
    if (((j + P + par) & 1) == 0) {
#pragma unroll
        for (int q = 0; q < 2 * M; q += 2) upd(q);
    } else {
#pragma unroll
        for (int q = 1; q < 2 * M; q += 2) upd(q);
    }
    x = out;
}

// x faces of a row from its stored low x faces: the face above the strip's
// last cell is the next strip's first (0 at a wall).  All lanes must call (DPP).
template <typename T, int M, bool PXY>
__device__ __forceinline__ void x_faces_stored(const BlkGeo& g, const Strip<T, M>& cx, T (&f)[2 * M + 1])
{
    const T nr = from_next(cx.v[0]);
#pragma unroll
    for (int q = 0; q < 2 * M; q++) f[q] = cx.v[q];
    f[2 * M] = !PXY && g.wr ? T(0) : nr;
}

// x faces of a row from cell coefficients (x_faces).  Periodic in x, the
// face above the strip's last cell is the next lane's face below its first
// cell, the harmonic mean of the same two values in the same order: it is
// taken from that lane instead of formed again.  All lanes must call (DPP).
template <typename T, int M, bool PXY>
__device__ __forceinline__ void x_faces_cell(const BlkGeo& g, const Strip<T, M>& c, T (&f)[2 * M + 1])
{
    if constexpr (PXY) {
        f[0] = harm(from_prev(c.v[2 * M - 1]), c.v[0]);
#pragma unroll
        for (int q = 1; q < 2 * M; q++) f[q] = harm(c.v[q - 1], c.v[q]);
        f[2 * M] = from_next(f[0]);
    } else {
        x_faces<T, M>(g, c, T(0), f);
    }
}

// Coefficients of the z faces between planes P and P+1 of a row (0 where
// either side lies beyond a wall).  A cell of plane P takes them as its face
// above, a cell of plane P+1 as its face below: in the colour passes the same
// harmonic mean of the same two values.
template <typename T, int M>
__device__ __forceinline__ Strip<T, M> z_faces(const Dims& d, int P, const Strip<T, M>& lo, const Strip<T, M>& hi)
{
    const bool has = (P >= 0 || d.pz) && (P < d.nz - 1 || d.pz);
    Strip<T, M> f;
#pragma unroll
    for (int q = 0; q < 2 * M; q++) f.v[q] = has ? harm(lo.v[q], hi.v[q]) : T(0);
    return f;
}

// A row of a plane buffer holds the even cells of every lane's strip, then
// the odd ones: lane l's cells 2e (e < M) at l M + e, its cells 2e + 1 at
// NX / 2 + l M + e.  A colour reads the cells of one parity of a neighbour
// row in one access of M consecutive words per lane, free of bank conflicts.
// (par selects by value: an index computed at run time would move the
// caller's register slots to scratch memory)
template <typename T, int M>
__device__ __forceinline__ void lds_put_half(T* p, const Strip<T, M>& s, int par)
{
    T h[M];
#pragma unroll
    for (int e = 0; e < M; e++) h[e] = par ? s.v[2 * e + 1] : s.v[2 * e];
    if constexpr (M == 2) {
        *reinterpret_cast<typename V2<T>::type*>(p) = typename V2<T>::type{h[0], h[1]};
    } else if constexpr (M == 4 && sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(h[0], h[1], h[2], h[3]);
    } else {
#pragma unroll
        for (int e = 0; e < M; e++) p[e] = h[e];
    }
}
// p: the row's first word plus lane l M.
template <typename T, int M, int NX>
__device__ __forceinline__ void lds_put_row(T* p, const Strip<T, M>& s)
{
    lds_put_half<T, M>(p, s, 0);
    lds_put_half<T, M>(p + NX / 2, s, 1);
}
template <typename T, int M>
__device__ __forceinline__ Half<T, M> lds_get_half(const T* p)
{
    Half<T, M> h;
    if constexpr (M == 2) {
        const typename V2<T>::type v = *reinterpret_cast<const typename V2<T>::type*>(p);
        h.v[0] = v.x;
        h.v[1] = v.y;
    } else if constexpr (M == 4 && sizeof(T) == 4) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        h.v[0] = v.x;
        h.v[1] = v.y;
        h.v[2] = v.z;
        h.v[3] = v.w;
    } else {
#pragma unroll
        for (int e = 0; e < M; e++) h.v[e] = p[e];
    }
    return h;
}

// Per-wavefront state of the LDS-tiled sweep.  Plane p of the chunk lives in
// register slot (p - z0 + 2) mod NS of x, c and b, so that a plane step
// names its planes by compile-time slots and no values move between
// registers (a move would wait for the prefetch in flight).  The x faces of
// a plane and the z faces above it are computed once, for its red update,
// and kept for the black update of the same plane and the red update of the
// next (slots of fx and fz).
// With stored faces, c holds the low y faces and cx, cz the low x and z faces.
template <typename T, int M, int NS>
struct FsCol {
    Strip<T, M> x[NS], c[NS], b[NS], fz[NS], cx[NS], cz[NS];
    T fx[NS][2 * M + 1];
};

template <typename T, int MODE, int M, int R, int D, bool IRU, bool CELL, bool PXY>
struct FsLds {
    static constexpr int NW = R + 4, NX = 128 * M, NS = D + 4;
    static_assert(D >= 0 && D <= 3, "the plane loop is unrolled for at most 7 slots");
    using S = Strip<T, M>;
    using H = Half<T, M>;
    const Dims& d;
    const BlkGeo& g;
    int j, jw;
    bool red_row, black_row;
    long long sz, roff;
    int nxc;
    long long szc;
    int so;
    const T* __restrict__ xo;
    T* __restrict__ xn;
    const T* __restrict__ b;
    const T* __restrict__ cc;  // cell coefficients, or the low y faces
    const T* __restrict__ cxa;  // low x and z faces (stored faces only)
    const T* __restrict__ cza;
    const T* __restrict__ ec;
    double* __restrict__ phi;
    const double* __restrict__ irs;
    bool phi_fresh;  // phi is zero on entry: written, not read
    bool lane_live;  // the lane's strip lies in the row (rows narrower than 2 M x 64 cells)
    int xe;          // the strip's first column, 0 for a lane past the row's end
    T h2;
    T (*sx)[NW * NX];
    T (*sc)[NW * NX];

    __device__ __forceinline__ S ldx(int kk) const
    {
        if constexpr (MODE == FS_ZERO) {
            return zero_strip<T, M>();
        } else {
            S v = ld_strip<T, M>(xo, (long long)kk * sz + roff);
            if constexpr (MODE == FS_PROLONG) {
                const long long o = (long long)(kk >> 1) * szc + (long long)(jw >> 1) * nxc + (xe >> 1);
#pragma unroll
                for (int q = 0; q < 2 * M; q++) v.v[q] = v.v[q] + ec[o + (q >> 1)];
            }
            return v;
        }
    }
    __device__ __forceinline__ S ldc(int kk) const { return ld_strip<T, M>(cc, (long long)kk * sz + roff); }
    __device__ __forceinline__ S ldb(int kk) const { return ld_strip<T, M>(b, (long long)kk * sz + roff); }
    // everything of plane kk a plane step needs, into slot Q
    template <int Q>
    __device__ __forceinline__ void ld_plane(FsCol<T, M, NS>& s, int kk) const
    {
        s.x[Q] = ldx(kk);
        s.c[Q] = ldc(kk);
        if constexpr (!CELL) {
            s.cx[Q] = ld_strip<T, M>(cxa, (long long)kk * sz + roff);
            s.cz[Q] = ld_strip<T, M>(cza, (long long)kk * sz + roff);
        }
    }

    // Plane step k; P0 is the slot of plane k.  i0, i1: LDS buffers of planes
    // k and k+1.
    template <int P0>
    __device__ __forceinline__ void step(FsCol<T, M, NS>& s, int k, int i0, int i1) const
    {
        constexpr int PM = (P0 + NS - 1) % NS, P1 = (P0 + 1) % NS, P2 = (P0 + 2) % NS;
        constexpr int PL = (P0 + 2 + D) % NS, PB = (P0 + 1 + D) % NS;
        // unconditional loads (the last planes of a chunk load the last
        // plane it needs again): a skipped load would leave the count of
        // loads in flight unknown to the compiler, which then waits for all
        ld_plane<PL>(s, wrap_plane(d, min(k + 2 + D, g.z1 + 1)));
        s.b[PB] = ldb(wrap_plane(d, min(k + 1 + D, g.z1)));

        lds_put_row<T, M, NX>(&sx[i1][so], s.x[P1]);
        lds_put_row<T, M, NX>(&sc[i1][so], s.c[P1]);
        __syncthreads();
        // red cells of row j on plane k+1 and black cells on plane k: cell q
        // with (q + j + k + 1) even, the same half of a buffer row
        const int ho = ((j + k + 1) & 1) * (NX / 2);
        const bool blk = black_row && k >= g.z0;
        // the black update's neighbour rows first, so that their LDS latency
        // overlaps the red update (it writes only plane k+1's buffer).  Every
        // wavefront reads (rows without a black update read their own row, in
        // bounds, and drop the values): no branch and no zeroed registers.
        const int blo = black_row ? so + ho - NX : so + ho, bhi = black_row ? so + ho + NX : so + ho;
        const H bxlo = lds_get_half<T, M>(&sx[i0][blo]);
        const H bxhi = lds_get_half<T, M>(&sx[i0][bhi]);
        const H bclo = CELL ? lds_get_half<T, M>(&sc[i0][blo]) : H{};
        const H bchi = lds_get_half<T, M>(&sc[i0][bhi]);
        if (red_row) {
            if constexpr (CELL) {
                x_faces_cell<T, M, PXY>(g, s.c[P1], s.fx[P1]);
                s.fz[P1] = z_faces<T, M>(d, k + 1, s.c[P1], s.c[P2]);
            } else {
                x_faces_stored<T, M, PXY>(g, s.cx[P1], s.fx[P1]);
            }
            const H xlo = lds_get_half<T, M>(&sx[i1][so + ho - NX]), xhi = lds_get_half<T, M>(&sx[i1][so + ho + NX]);
            const H clo = CELL ? lds_get_half<T, M>(&sc[i1][so + ho - NX]) : H{};
            const H chi = lds_get_half<T, M>(&sc[i1][so + ho + NX]);
            fs_row<T, M, CELL, PXY>(d, g, j, k + 1, 0, h2, s.x[P1], xlo, xhi, s.x[P0], s.x[P2], s.fx[P1], s.c[P1], clo,
                               chi, CELL ? s.fz[P0] : s.cz[P1], CELL ? s.fz[P1] : s.cz[P2], s.b[P1]);
            // only the red half changed
            lds_put_half<T, M>(&sx[i1][so + ho], s.x[P1], (j + k + 1) & 1);
        }
        if (blk) {
            fs_row<T, M, CELL, PXY>(d, g, j, k, 1, h2, s.x[P0], bxlo, bxhi, s.x[PM], s.x[P1], s.fx[P0], s.c[P0], bclo,
                               bchi, CELL ? s.fz[PM] : s.cz[P0], CELL ? s.fz[P0] : s.cz[P1], s.b[P0]);
            const long long o = (long long)k * sz + roff;
            if (lane_live) st_strip<T, M>(xn, o, s.x[P0]);
            if constexpr (IRU) {
                if (lane_live) {
                    const double sc0 = irs[0];
                    double* pp = phi + o;
#pragma unroll
                    for (int q = 0; q < M; q++) {
                        const double2 pv =
                            phi_fresh ? make_double2(0.0, 0.0) : *reinterpret_cast<const double2*>(pp + 2 * q);
                        *reinterpret_cast<double2*>(pp + 2 * q) = make_double2(
                            fma(sc0, (double)s.x[P0].v[2 * q], pv.x), fma(sc0, (double)s.x[P0].v[2 * q + 1], pv.y));
                    }
                }
            }
        }
    }
};

// D: planes loaded ahead of the three a plane step works on (x, c), and of
// the two it takes b from.
// CELL: cc holds cell coefficients; otherwise cc, cxa, cza hold the low y,
// x and z faces.  PXY: x and y periodic.
template <typename T, int MODE, int M, int R, int D, bool IRU, bool CELL, bool PXY>
__global__ __launch_bounds__(kWave*(R + 4)) void k_fsw_lds(Dims d, int lz, const T* __restrict__ xo,
                                                            T* __restrict__ xn, const T* __restrict__ b,
                                                            const T* __restrict__ cc, const T* __restrict__ cxa,
                                                            const T* __restrict__ cza, T h2,
                                                            const T* __restrict__ ec, double* __restrict__ phi,
                                                            const double* __restrict__ irs, int irf)
{
    using F = FsLds<T, MODE, M, R, D, IRU, CELL, PXY>;
    constexpr int NS = F::NS;
    __shared__ __align__(16) T sx[3][F::NW * F::NX];
    __shared__ __align__(16) T sc[3][F::NW * F::NX];
    unsigned bx, by, bz;
    blk_tile(bx, by, bz);
    BlkGeo g;
    g.lane = threadIdx.x & (kWave - 1);
    g.xi = 2 * M * g.lane;
    g.j0 = (int)by * R;
    g.z0 = (int)bz * lz;
    g.z1 = min(g.z0 + lz, d.nz);
    g.hal = false;
    g.hcol = 0;
    g.wl = !PXY && g.xi == 0 && !d.px;
    g.wr = !PXY && g.xi + 2 * M == d.nx && !d.px;
    g.live = true;
    g.yfirst = g.ylast = true;
    const int t = threadIdx.x / kWave;  // row of the workgroup
    F f{d, g};
    f.j = g.j0 - 2 + t;
    f.jw = wrap_row(d, f.j);
    f.red_row = t >= 1 && t <= R + 2;
    f.black_row = t >= 2 && t <= R + 1 && f.j < d.ny;
    f.sz = (long long)d.nx * d.ny;
    f.lane_live = g.xi < d.nx;
    f.xe = f.lane_live ? g.xi : 0;
    f.roff = (long long)f.jw * d.nx + f.xe;
    f.nxc = d.nx >> 1;
    f.szc = (long long)f.nxc * (d.ny >> 1);
    f.so = t * F::NX + M * g.lane;  // the lane's words in row t of a buffer
    f.xo = xo;
    f.xn = xn;
    f.b = b;
    f.cc = cc;
    f.cxa = cxa;
    f.cza = cza;
    f.ec = ec;
    f.phi = phi;
    f.irs = irs;
    f.phi_fresh = (irf & 1) != 0;
    f.h2 = h2;
    f.sx = sx;
    f.sc = sc;

    // planes z0-2 .. z0+D-1 (x and coefficients) and z0-1 .. z0+D-2 (b)
    // before the first step
    const int zs = g.z0 - 2;
    FsCol<T, M, NS> s;
#pragma unroll
    for (int q = 0; q < NS; q++) {
        s.x[q] = s.c[q] = s.b[q] = s.fz[q] = s.cx[q] = s.cz[q] = zero_strip<T, M>();
#pragma unroll
        for (int e = 0; e <= 2 * M; e++) s.fx[q][e] = T(0);
    }
    f.template ld_plane<0>(s, wrap_plane(d, zs));
    f.template ld_plane<1 % NS>(s, wrap_plane(d, zs + 1));
    if constexpr (D >= 1) f.template ld_plane<2 % NS>(s, wrap_plane(d, zs + 2));
    if constexpr (D >= 2) f.template ld_plane<3 % NS>(s, wrap_plane(d, zs + 3));
    if constexpr (D >= 3) f.template ld_plane<4 % NS>(s, wrap_plane(d, zs + 4));
#pragma unroll
    for (int q = 1; q <= D; q++) s.b[q] = f.ldb(wrap_plane(d, zs + q));
    if constexpr (CELL) s.fz[0] = z_faces<T, M>(d, zs, s.c[0], s.c[1]);  // below the first red plane
    int i0 = 0, i1 = 1;  // LDS buffers of planes k and k+1
    auto adv = [&]() {
        i0 = i1;
        i1 = i1 == 2 ? 0 : i1 + 1;
    };
    // whole groups of NS plane steps, then the rest one at a time
    int k = zs;
    for (; k + NS <= g.z1; k += NS) {
        f.template step<0>(s, k, i0, i1);
        adv();
        f.template step<1>(s, k + 1, i0, i1);
        adv();
        f.template step<2>(s, k + 2, i0, i1);
        adv();
        f.template step<3>(s, k + 3, i0, i1);
        adv();
        if constexpr (NS > 4) {
            f.template step<4 % NS>(s, k + 4, i0, i1);
            adv();
        }
        if constexpr (NS > 5) {
            f.template step<5 % NS>(s, k + 5, i0, i1);
            adv();
        }
        if constexpr (NS > 6) {
            f.template step<6 % NS>(s, k + 6, i0, i1);
            adv();
        }
    }
    if (k < g.z1) f.template step<0>(s, k, i0, i1);
    adv();
    if (k + 1 < g.z1) f.template step<1>(s, k + 1, i0, i1);
    adv();
    if (k + 2 < g.z1) f.template step<2>(s, k + 2, i0, i1);
    adv();
    if constexpr (NS > 4) {
        if (k + 3 < g.z1) f.template step<3 % NS>(s, k + 3, i0, i1);
        adv();
    }
    if constexpr (NS > 5) {
        if (k + 4 < g.z1) f.template step<4 % NS>(s, k + 4, i0, i1);
        adv();
    }
    if constexpr (NS > 6) {
        if (k + 5 < g.z1) f.template step<5 % NS>(s, k + 5, i0, i1);
        adv();
    }
}

// Launch shape by strip width M (2M cells per lane, rows of 128 M cells):
// rows owned by a workgroup (R + 4 wavefronts) and planes loaded ahead (D).
// Rows of up to 256 cells: 8 rows, 12 wavefronts, three per SIMD.  Rows of
// 384 and 512 cells hold 6 or 8 cells per lane in every plane slot: 4 rows,
// 8 wavefronts, two per SIMD, which the larger strips need for registers.
template <int M, int MODE, bool IRU, bool CELL>
struct FswShape {
    static constexpr int R = M <= 2 ? 8 : 4;
    static constexpr int D = M <= 3 ? 1 : 0;
};
constexpr int kFswMinPlanes = 8;

// Planes per chunk.  Each workgroup marches lz + 2 plane steps, and the
// per-plane critical path (barrier, LDS round trips, the two updates) rather
// than HBM bounds a workgroup, so the sweep takes about (rounds of resident
// workgroups) x (lz + 2) plane steps: the chunk count minimising that is
// taken (at least kFswMinPlanes planes, which bounds the share of the four
// planes a chunk reads beyond its own), each chunk lengthened until its plane
// steps are whole groups of the unrolled plane loop.  256^3 (32 row blocks):
// 8 chunks of 33 planes in one round; 512^3 (128 row blocks): 2 of 258;
// 384^3 (96 row blocks): 8 chunks of 48 planes in three rounds rather than 2
// chunks of 192 on three quarters of the CUs.
template <typename T, int MODE, int M, bool IRU, bool CELL, bool PXY>
static int fsw_chunk(const Dims& d, long long gy)
{
    constexpr int R = FswShape<M, MODE, IRU, CELL>::R, D = FswShape<M, MODE, IRU, CELL>::D, NS = D + 4;
    static int resident = 0;  // workgroups resident on the device at once
    if (resident == 0) {
        int dev = 0, ncu = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void*>(k_fsw_lds<T, MODE, M, R, D, IRU, CELL, PXY>), kWave * (R + 4),
                0) != hipSuccess)
            return 16;
        resident = max(1, ncu * max(per_cu, 1));
    }
    int best = d.nz;
    long long best_cost = -1;
    for (int c = 1; c == 1 || d.nz / c >= kFswMinPlanes; c++) {
        int lz = max((d.nz + c - 1) / c, kFswMinPlanes);
        lz += (NS - (lz + 2) % NS) % NS;
        const long long wgs = gy * ((d.nz + lz - 1) / lz);
        const long long cost = (wgs + resident - 1) / resident * (lz + 2);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = lz;
        }
    }
    return best;
}

template <typename T, int MODE, int M, bool IRU, bool CELL, bool PXY>
static void fsw_launch_p(const Dims& d, const T* xo, T* xn, const T* b, const T* cc, const T* cxa, const T* cza,
                         T h2, const T* ec, double* phi, const double* irs, int irf, hipEvent_t ev0, hipEvent_t ev1,
                         hipStream_t s)
{
    constexpr int R = FswShape<M, MODE, IRU, CELL>::R, D = FswShape<M, MODE, IRU, CELL>::D;
    const long long gy = (d.ny + R - 1) / R;
    const int lz = fsw_chunk<T, MODE, M, IRU, CELL, PXY>(d, gy);
    const dim3 grid(1, (unsigned)gy, (unsigned)((d.nz + lz - 1) / lz));
    const dim3 block(kWave * (R + 4));
    if (ev0)
        hipExtLaunchKernelGGL((k_fsw_lds<T, MODE, M, R, D, IRU, CELL, PXY>), grid, block, 0, s, ev0, ev1, 0, d,
                              lz, xo, xn, b, cc, cxa, cza, h2, ec, phi, irs, irf);
    else
        hipLaunchKernelGGL((k_fsw_lds<T, MODE, M, R, D, IRU, CELL, PXY>), grid, block, 0, s, d, lz, xo, xn, b,
                           cc, cxa, cza, h2, ec, phi, irs, irf);
}

// the variant without wall selects when x and y are both periodic
template <typename T, int MODE, int M, bool IRU, bool CELL>
static void fsw_launch(const Dims& d, const T* xo, T* xn, const T* b, const T* cc, const T* cxa, const T* cza, T h2,
                       const T* ec, double* phi, const double* irs, int irf, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s)
{
    if (d.px && d.py)
        fsw_launch_p<T, MODE, M, IRU, CELL, true>(d, xo, xn, b, cc, cxa, cza, h2, ec, phi, irs, irf, ev0, ev1, s);
    else
        fsw_launch_p<T, MODE, M, IRU, CELL, false>(d, xo, xn, b, cc, cxa, cza, h2, ec, phi, irs, irf, ev0, ev1, s);
}

template <typename T, int M>
static void fsw_mode(int mode, const Dims& d, const T* xo, T* xn, const T* b, const T* cc, T h2, const T* ec,
                     double* phi, const double* irs, int irf, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s)
{
    if (phi) {
        // the refinement update rides on the last sweep of a V-cycle
        if (mode == FS_PROLONG)
            fsw_launch<T, FS_PROLONG, M, true, true>(d, xo, xn, b, cc, nullptr, nullptr, h2, ec, phi, irs, irf, ev0, ev1,
                                                     s);
        else
            fsw_launch<T, FS_PLAIN, M, true, true>(d, xo, xn, b, cc, nullptr, nullptr, h2, ec, phi, irs, irf, ev0, ev1, s);
        return;
    }
    switch (mode) {
    case FS_ZERO:
        fsw_launch<T, FS_ZERO, M, false, true>(d, xo, xn, b, cc, nullptr, nullptr, h2, ec, nullptr, nullptr, 0, ev0, ev1,
                                               s);
        break;
    case FS_PROLONG:
        fsw_launch<T, FS_PROLONG, M, false, true>(d, xo, xn, b, cc, nullptr, nullptr, h2, ec, nullptr, nullptr, 0, ev0,
                                                  ev1, s);
        break;
    default:
        fsw_launch<T, FS_PLAIN, M, false, true>(d, xo, xn, b, cc, nullptr, nullptr, h2, ec, nullptr, nullptr, 0, ev0, ev1,
                                                s);
        break;
    }
}

template <typename T>
void launch_fsw_blk(const Dims& d, const T* xo, T* xn, const T* b, const T* cc, T h2, int mode, const T* ec,
                    double* phi, const double* irs, int irf, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s)
{
    switch (d.nx) {
    case 512: fsw_mode<T, 4>(mode, d, xo, xn, b, cc, h2, ec, phi, irs, irf, ev0, ev1, s); break;
    case 384: fsw_mode<T, 3>(mode, d, xo, xn, b, cc, h2, ec, phi, irs, irf, ev0, ev1, s); break;
    case 256: fsw_mode<T, 2>(mode, d, xo, xn, b, cc, h2, ec, phi, irs, irf, ev0, ev1, s); break;
    default: fsw_mode<T, 1>(mode, d, xo, xn, b, cc, h2, ec, phi, irs, irf, ev0, ev1, s); break;
    }
}

template <typename T, int M>
static void fswf_mode(int mode, const Dims& d, const T* xo, T* xn, const T* b, const Coef<T>& c, T h2, const T* ec,
                      hipStream_t s)
{
    switch (mode) {
    case FS_ZERO:
        fsw_launch<T, FS_ZERO, M, false, false>(d, xo, xn, b, c.y, c.x, c.z, h2, ec, nullptr, nullptr, 0, nullptr,
                                                nullptr, s);
        break;
    case FS_PROLONG:
        fsw_launch<T, FS_PROLONG, M, false, false>(d, xo, xn, b, c.y, c.x, c.z, h2, ec, nullptr, nullptr, 0, nullptr,
                                                   nullptr, s);
        break;
    default:
        fsw_launch<T, FS_PLAIN, M, false, false>(d, xo, xn, b, c.y, c.x, c.z, h2, ec, nullptr, nullptr, 0, nullptr,
                                                 nullptr, s);
        break;
    }
}

template <typename T>
void launch_fsw_blkf(const Dims& d, const T* xo, T* xn, const T* b, const Coef<T>& c, T h2, int mode, const T* ec,
                     hipStream_t s)
{
    switch (d.nx) {
    case 512: fswf_mode<T, 4>(mode, d, xo, xn, b, c, h2, ec, s); break;
    case 384: fswf_mode<T, 3>(mode, d, xo, xn, b, c, h2, ec, s); break;
    case 256:
    case 192: fswf_mode<T, 2>(mode, d, xo, xn, b, c, h2, ec, s); break;
    default: fswf_mode<T, 1>(mode, d, xo, xn, b, c, h2, ec, s); break;
    }
}

template void launch_fsw_blk<float>(const Dims&, const float*, float*, const float*, const float*, float, int,
                                    const float*, double*, const double*, int, hipEvent_t, hipEvent_t, hipStream_t);
template void launch_fsw_blkf<float>(const Dims&, const float*, float*, const float*, const Coef<float>&, float, int,
                                     const float*, hipStream_t);

}  // namespace mp
