// k_sweep.hip -- one full red-black Gauss-Seidel sweep (red, then black) in a
// single launch, out of place: reads x_old, writes x_new.
//
// Why: with one launch per colour every sweep streams the iterate, the three
// face coefficients and the right-hand side through HBM twice (10 words per
// cell).  Fusing the colours reads them once (6 words).  The black update
// needs the new red values of its in-plane neighbours, which live partly in
// neighbouring tiles; instead of synchronising tiles, each workgroup
// recomputes the red values of a one-cell ring around its tile from x_old
// (a two-cell ring of x_old is staged in LDS).  Because x_old is never
// written, tiles are independent and the result is, cell for cell, the same
// arithmetic as the two-launch sweep (bitwise equal).
//
// Data flow per workgroup: a 64 x 8 tile of columns marches along z.  At
// step s it stages plane s of x_old (68 x 12 with halo) in an LDS ring of 3
// planes, computes red on plane s-1 over the 66 x 10 ring (LDS ring of 3
// planes of red values), then black on plane s-2 over the tile and writes
// both colours of plane s-2 to x_new.  Coefficients and b are read straight
// from global memory (each is touched by at most two consecutive steps, so
// the second touch hits L2).  Tiles are ordered so that each XCD (own L2)
// gets a contiguous slab of tiles; halo rows then mostly hit the same L2.
//
// Optional fusions: zero_init (x_old = 0, nothing read) for the first
// pre-smoothing sweep, and ec != nullptr (x_old = x + P e_coarse,
// piecewise-constant prolongation added while staging) for the first
// post-smoothing sweep.
#include "mp_device.h"
#include "mp_kernels.h"

namespace mp {

constexpr int SW_TX = 64, SW_TY = 8;
constexpr int SW_HX = SW_TX + 4, SW_HY = SW_TY + 4;  // x_old frame, halo 2
constexpr int SW_RX = SW_TX + 2, SW_RY = SW_TY + 2;  // red frame, halo 1
constexpr int SW_THREADS = 256;

// Global index of a frame position: in range, wrapped (periodic; a tile may
// extend past a short axis, so the wrap is a true modulo), or outside
// (Neumann).
__device__ __forceinline__ int frame_wrap(int g, int n, int per, bool& ok)
{
    if (g >= 0 && g < n) {
        ok = true;
        return g;
    }
    if (per) {
        ok = true;
        int r = g % n;
        return r < 0 ? r + n : r;
    }
    ok = false;
    return 0;
}

__device__ __forceinline__ int ring(int v) { return (v + 3) % 3; }  // v >= -3

// In-plane geometry of one frame position, fixed for the whole z-march.
struct PlanePos {
    int off;   // in-plane element offset (gy * nx + gx), -1 outside the grid
    int dxp;   // offset of the high-x face coefficient, 0 = wall
    int dyp;   // offset of the high-y face coefficient, 0 = wall
    int coff;  // in-plane offset of the parent cell one level coarser
};

__device__ __forceinline__ PlanePos plane_pos(const Dims& d, int gxu, int gyu)
{
    PlanePos p;
    bool okx, oky;
    const int gx = frame_wrap(gxu, d.nx, d.px, okx);
    const int gy = frame_wrap(gyu, d.ny, d.py, oky);
    if (!(okx && oky)) {
        p.off = -1;
        p.dxp = p.dyp = p.coff = 0;
        return p;
    }
    p.off = gy * d.nx + gx;
    p.dxp = gx < d.nx - 1 ? 1 : (d.px ? -(d.nx - 1) : 0);
    p.dyp = gy < d.ny - 1 ? d.nx : (d.py ? -(d.ny - 1) * d.nx : 0);
    p.coff = (gy >> 1) * (d.nx >> 1) + (gx >> 1);
    return p;
}

template <typename T>
__global__ __launch_bounds__(SW_THREADS) void k_sweep(Dims d, int lz, int tiles_x, int tiles_y, int nblk,
                                                      const T* __restrict__ xo, T* __restrict__ xn,
                                                      const T* __restrict__ b, const T* __restrict__ cx,
                                                      const T* __restrict__ cy, const T* __restrict__ cz, T h2,
                                                      int zero_init, const T* __restrict__ ec)
{
    constexpr int NSTG = (SW_HX * SW_HY + SW_THREADS - 1) / SW_THREADS;        // staging values per thread
    constexpr int NRED = (SW_RY * (SW_RX / 2) + SW_THREADS - 1) / SW_THREADS;  // red cells per thread
    constexpr int PLANE_O = SW_HY * SW_HX, PLANE_R = SW_RY * SW_RX;
    __shared__ T so[3 * PLANE_O];
    __shared__ T sr[3 * PLANE_R];
    const int tid = threadIdx.x;
    // XCD-aware order: consecutive dispatches go to different XCDs, so give
    // XCD x the contiguous logical range [x * full/8, (x+1) * full/8).
    const int bid = blockIdx.x;
    const int full = (nblk / 8) * 8;
    const int lin = bid < full ? (bid % 8) * (full / 8) + bid / 8 : bid;
    const int tx = lin % tiles_x;
    const int t2 = lin / tiles_x;
    const int ty = t2 % tiles_y;
    const int zc = t2 / tiles_y;
    const int x0 = tx * SW_TX, y0 = ty * SW_TY;
    const int z0 = zc * lz, z1 = min(z0 + lz, d.nz);
    const long long sz = (long long)d.nx * d.ny;
    const long long szc = (long long)(d.nx >> 1) * (d.ny >> 1);

    // ---- per-thread geometry, fixed along z ----
    PlanePos stp[NSTG];
#pragma unroll
    for (int u = 0; u < NSTG; u++) {
        const int e = tid + SW_THREADS * u;
        const int ly = e / SW_HX, lx = e - ly * SW_HX;
        stp[u] = e < PLANE_O ? plane_pos(d, x0 + lx - 2, y0 + ly - 2) : PlanePos{-1, 0, 0, 0};
    }
    // red cells for the two parities of the plane index; frame index in the
    // red frame (rr) and in the x_old frame (ro)
    PlanePos rp[2][NRED];
    int rr[2][NRED], ro[2][NRED];
#pragma unroll
    for (int par = 0; par < 2; par++)
#pragma unroll
        for (int u = 0; u < NRED; u++) {
            const int e = tid + SW_THREADS * u;
            const int ly = e / (SW_RX / 2), hq = e - ly * (SW_RX / 2);
            const int lx = 2 * hq + ((x0 - 1 + y0 + ly - 1 + par) & 1);
            const bool in = e < SW_RY * (SW_RX / 2);
            rp[par][u] = in ? plane_pos(d, x0 + lx - 1, y0 + ly - 1) : PlanePos{-1, 0, 0, 0};
            rr[par][u] = in ? ly * SW_RX + lx : -1;
            ro[par][u] = (ly + 1) * SW_HX + lx + 1;
        }
    // this thread's black cell (row bly, pair bp) for the two plane parities
    const int bly = tid >> 5, bp = tid & 31;
    const int bgy = y0 + bly;
    const int blx0 = 2 * bp + ((x0 + bgy + 1) & 1), blx1 = blx0 ^ 1;
    const PlanePos bpp0 = (bgy < d.ny && x0 + blx0 < d.nx) ? plane_pos(d, x0 + blx0, bgy) : PlanePos{-1, 0, 0, 0};
    const PlanePos bpp1 = (bgy < d.ny && x0 + blx1 < d.nx) ? plane_pos(d, x0 + blx1, bgy) : PlanePos{-1, 0, 0, 0};
    auto bsel = [&](bool odd) {
        PlanePos p;
        p.off = odd ? bpp1.off : bpp0.off;
        p.dxp = odd ? bpp1.dxp : bpp0.dxp;
        p.dyp = odd ? bpp1.dyp : bpp0.dyp;
        p.coff = odd ? bpp1.coff : bpp0.coff;
        return p;
    };

    // Plane z of the grid (wrapped / outside) and its z-face data.
    struct PlaneZ {
        bool ok;
        long long base;   // gz * sz
        long long cbase;  // (gz >> 1) * szc
        long long hzp;    // base of the high-z face plane, -1 = wall
    };
    auto plane_z = [&](int s) {
        PlaneZ pz;
        bool ok;
        const int gz = frame_wrap(s, d.nz, d.pz, ok);
        pz.ok = ok;
        pz.base = (long long)gz * sz;
        pz.cbase = (long long)(gz >> 1) * szc;
        pz.hzp = gz < d.nz - 1 ? pz.base + sz : (d.pz ? 0 : -1);
        return pz;
    };

    // Software pipeline: every global load is issued one z-step before its
    // use, into registers, so its latency overlaps the current step's work.
    T stg[NSTG];
    T rcf[NRED][7];  // red cells of the next plane: 6 coefficients and b
    T bcf[7];        // black cell of the next plane

    auto load_stage = [&](int s) {
        const PlaneZ pz = plane_z(s);
#pragma unroll
        for (int u = 0; u < NSTG; u++) {
            T v = T(0);
            if (stp[u].off >= 0 && pz.ok && !zero_init) {
                v = xo[pz.base + stp[u].off];
                if (ec) v += ec[pz.cbase + stp[u].coff];
            }
            stg[u] = v;
        }
    };
    auto load_coefs = [&](const PlaneZ& pz, const PlanePos& pp, T* out) {
        const long long q = pz.base + pp.off;
        out[0] = cx[q];
        out[1] = pp.dxp ? cx[q + pp.dxp] : T(0);
        out[2] = cy[q];
        out[3] = pp.dyp ? cy[q + pp.dyp] : T(0);
        out[4] = cz[q];
        out[5] = pz.hzp >= 0 ? cz[pz.hzp + pp.off] : T(0);
        out[6] = b[q];
    };
    // (register arrays are only ever indexed by compile-time constants, so
    // the parity is resolved by branching on it)
    auto load_red_p = [&](const PlaneZ& pz, const PlanePos (&RP)[NRED]) {
#pragma unroll
        for (int u = 0; u < NRED; u++)
            if (RP[u].off >= 0) load_coefs(pz, RP[u], rcf[u]);
    };
    auto load_red = [&](int m) {
        if (m < z0 - 1 || m > z1) return;
        const PlaneZ pz = plane_z(m);
        if (!pz.ok) return;
        if (m & 1)
            load_red_p(pz, rp[1]);
        else
            load_red_p(pz, rp[0]);
    };
    auto load_black = [&](int k) {
        if (k < z0 || k >= z1) return;
        const PlanePos pp = bsel(k & 1);
        if (pp.off >= 0) load_coefs(plane_z(k), pp, bcf);
    };
    auto red_p = [&](bool okz, const T* om, const T* omm, const T* omp, T* rm, const PlanePos (&RP)[NRED],
                     const int (&RR)[NRED], const int (&RO)[NRED]) {
#pragma unroll
        for (int u = 0; u < NRED; u++) {
            if (RR[u] >= 0) {
                T v = T(0);
                if (okz && RP[u].off >= 0) {
                    const int o = RO[u];
                    v = gs_value<T>(rcf[u][0], rcf[u][1], rcf[u][2], rcf[u][3], rcf[u][4], rcf[u][5], om[o - 1],
                                    om[o + 1], om[o - SW_HX], om[o + SW_HX], omm[o], omp[o], rcf[u][6], h2, om[o]);
                }
                rm[RR[u]] = v;
            }
        }
    };

    load_stage(z0 - 2);
    for (int s = z0 - 2; s <= z1 + 1; s++) {
        // (1) plane s of x_old into the LDS ring; prefetch plane s+1
        {
            T* dst = so + ring(s) * PLANE_O;
#pragma unroll
            for (int u = 0; u < NSTG; u++) {
                const int e = tid + SW_THREADS * u;
                if (e < PLANE_O) dst[e] = stg[u];
            }
            if (s + 1 <= z1 + 1) load_stage(s + 1);
        }
        __syncthreads();
        // (2) red ((i+j+k) even) on plane m = s-1 over the halo-1 frame
        const int m = s - 1;
        if (m >= z0 - 1 && m <= z1) {
            const bool okz = plane_z(m).ok;
            const T* om = so + ring(m) * PLANE_O;
            const T* omm = so + ring(m - 1) * PLANE_O;
            const T* omp = so + ring(m + 1) * PLANE_O;
            T* rm = sr + ring(m) * PLANE_R;
            if (m & 1)
                red_p(okz, om, omm, omp, rm, rp[1], rr[1], ro[1]);
            else
                red_p(okz, om, omm, omp, rm, rp[0], rr[0], ro[0]);
        }
        load_red(s);
        __syncthreads();
        // (3) black on plane k = s-2 over the tile; write both colours
        const int k = s - 2;
        if (k >= z0 && k < z1) {
            const bool odd = k & 1;
            const PlanePos pp = bsel(odd);
            const int lxb = odd ? blx1 : blx0, lxr = lxb ^ 1;
            const T* rk = sr + ring(k) * PLANE_R;
            const T* rkm = sr + ring(k - 1) * PLANE_R;
            const T* rkp = sr + ring(k + 1) * PLANE_R;
            const long long base = (long long)k * sz;
            if (pp.off >= 0) {
                const int o = (bly + 1) * SW_RX + lxb + 1;
                // The old value is read from x_old in global memory: the LDS
                // slot of plane k is being restaged by threads that have
                // moved on to the next step.
                T old = T(0);
                if (!zero_init) {
                    old = xo[base + pp.off];
                    if (ec) old += ec[(long long)(k >> 1) * szc + pp.coff];
                }
                xn[base + pp.off] = gs_value<T>(bcf[0], bcf[1], bcf[2], bcf[3], bcf[4], bcf[5], rk[o - 1], rk[o + 1],
                                                rk[o - SW_RX], rk[o + SW_RX], rkm[o], rkp[o], bcf[6], h2, old);
            }
            if (bgy < d.ny && x0 + lxr < d.nx)
                xn[base + (long long)bgy * d.nx + x0 + lxr] = rk[(bly + 1) * SW_RX + lxr + 1];
        }
        load_black(s - 1);
    }
}

bool sweep_supported(const Dims& d)
{
    // colours must be consistent across periodic wraps
    if (d.px && d.nx % 2) return false;
    if (d.py && d.ny % 2) return false;
    if (d.pz && d.nz % 2) return false;
    return true;
}

template <typename T>
void launch_sweep(const Dims& d, const T* xo, T* xn, const T* b, const T* cx, const T* cy, const T* cz, T h2,
                  int zero_init, const T* ec, hipStream_t s)
{
    const int tiles_x = (d.nx + SW_TX - 1) / SW_TX, tiles_y = (d.ny + SW_TY - 1) / SW_TY;
    const long long tiles = (long long)tiles_x * tiles_y;
    // at least 8 resident workgroups per CU on 256 CUs when the grid allows,
    // with chunks long enough that the 4 extra halo planes stay cheap
    int lz = d.nz < 8 ? d.nz : 8;
    for (int c = 64; c >= 8; c >>= 1) {
        if (c <= d.nz && tiles * ((d.nz + c - 1) / c) >= 2048) {
            lz = c;
            break;
        }
    }
    const int nblk = (int)(tiles * ((d.nz + lz - 1) / lz));
    hipLaunchKernelGGL((k_sweep<T>), dim3(nblk), dim3(SW_THREADS), 0, s, d, lz, tiles_x, tiles_y, nblk, xo, xn, b,
                       cx, cy, cz, h2, zero_init, ec);
}

template void launch_sweep<float>(const Dims&, const float*, float*, const float*, const float*, const float*,
                                  const float*, float, int, const float*, hipStream_t);
template void launch_sweep<double>(const Dims&, const double*, double*, const double*, const double*, const double*,
                                   const double*, double, int, const double*, hipStream_t);

}  // namespace mp
