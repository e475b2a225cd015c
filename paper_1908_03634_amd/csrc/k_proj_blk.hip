// k_proj_blk.hip -- register-blocked projection kernels on the finest level
// (right-hand side / divergence defect and velocity correction of Sec. 3.2
// Steps 3 and 7, Appendix A).
//
// Same layout as the blocked smoother (mp_blk.h): each lane owns a strip of 2
// consecutive cells (one 16-byte FP64 access per array and row) in R rows and
// marches along z; x neighbours come from the adjacent lanes by DPP rotations
// (lanes 0 and 63 of a wavefront that does not span the row load a halo
// column), y neighbours from the lane's own rows and halo rows, z neighbours
// from the previous plane kept in registers.  Periodic x and y only, so every
// face array has the cell shape and every strip access is aligned.  Every
// face flux and face update uses the expressions of the one-cell kernels in
// the same operand order, so the results are the same bits.
#include "mp_blk.h"
#include "mp_device.h"
#include "mp_kernels.h"

namespace mp {

namespace {

constexpr int PB_M = 1;  // pairs per lane (2 doubles)
constexpr int PB_R = 2;  // rows per wavefront

using S2 = Strip<double, PB_M>;

// Source of a cell (S, or S - Sbar per plane or per irregular radius).
__device__ __forceinline__ double src_of(const Dims& d, double s, const double* __restrict__ sbar, int smode, int i,
                                         int j, int k)
{
    if (smode == 1) return s - sbar[k];
    if (smode == 2) {
        const long long a = 2LL * i + 1 - d.nx, b = 2LL * j + 1 - d.ny, c = 2LL * k + 1 - d.nz;
        return s - sbar[(a * a + b * b + c * c - 3) / 8];
    }
    return s;
}

}  // namespace

bool proj_blk_supported(const Dims& d) { return blk_supported(d) && d.px && d.py; }

// b = beta0 S' - D(beta0 U) (shift == nullptr: written, partials = sum b and,
// when part2 != nullptr, part2 = sum b^2), or the defect sum of
// (b - shift[0])^2 without a write.
__global__ __launch_bounds__(BK_T) void k_rhs_blk(Dims d, int lz, double inv_h, const double* __restrict__ beta0,
                                                  const double* __restrict__ ux, const double* __restrict__ uy,
                                                  const double* __restrict__ uz, const double* __restrict__ S,
                                                  const double* __restrict__ sbar, int smode, double* __restrict__ b,
                                                  double* part, const double* __restrict__ shift,
                                                  double* __restrict__ part2)
{
    constexpr int R = PB_R;
    __shared__ double sh[BK_T / kWave];
    const BlkGeo g = blk_geo<PB_M, R>(d, lz);
    double acc = 0.0, acc2 = 0.0;
    const double sh0 = shift ? shift[0] : 0.0;
    if (g.live) {
        const long long sz = (long long)d.nx * d.ny;
        long long roff[R + 2];  // rows j0-1 .. j0+R (wrapped)
#pragma unroll
        for (int t = 0; t < R + 2; t++) roff[t] = (long long)wrap_row(d, g.j0 - 1 + t) * d.nx;
        // beta0 of the current plane and the z flux through its low face
        S2 bq[R];
        double fzl[R][2];
#pragma unroll
        for (int t = 0; t < R; t++) {
            const long long q = (long long)g.z0 * sz + roff[t + 1] + g.xi;
            bq[t] = ld_strip<double, PB_M>(beta0, q);
            if (g.z0 > 0 || d.pz) {
                const S2 bm = ld_strip<double, PB_M>(beta0, (long long)wrap_plane(d, g.z0 - 1) * sz + roff[t + 1] + g.xi);
                const S2 u = ld_strip<double, PB_M>(uz, q);
#pragma unroll
                for (int c = 0; c < 2; c++) fzl[t][c] = 0.5 * (bm.v[c] + bq[t].v[c]) * u.v[c];
            } else {
                fzl[t][0] = fzl[t][1] = 0.0;
            }
        }
        for (int k = g.z0; k < g.z1; k++) {
            const long long pk = (long long)k * sz;
            const bool hzp = k < d.nz - 1 || d.pz;
            // the high z faces: plane k+1 of uz (the wrap to plane 0 when
            // periodic), beta0 of plane k+1
            const long long pn = (long long)(k < d.nz - 1 ? k + 1 : 0) * sz;
            const long long pu = k < d.nz - 1 || d.pz ? pn : pk;
            const S2 blo = ld_strip<double, PB_M>(beta0, pk + roff[0] + g.xi);
            const S2 bhi = ld_strip<double, PB_M>(beta0, pk + roff[R + 1] + g.xi);
            S2 vy[R + 1], vx[R], sv[R], bn[R], vz[R];
            double hb[R], hu[R];
#pragma unroll
            for (int t = 0; t <= R; t++) vy[t] = ld_strip<double, PB_M>(uy, pk + roff[t + 1] + g.xi);
#pragma unroll
            for (int t = 0; t < R; t++) {
                const long long q = pk + roff[t + 1] + g.xi;
                vx[t] = ld_strip<double, PB_M>(ux, q);
                sv[t] = ld_strip<double, PB_M>(S, q);
                bn[t] = ld_strip<double, PB_M>(beta0, pn + roff[t + 1] + g.xi);
                vz[t] = ld_strip<double, PB_M>(uz, pu + roff[t + 1] + g.xi);
                hb[t] = g.hal ? beta0[pk + roff[t + 1] + g.hcol] : 0.0;
                hu[t] = g.hal ? ux[pk + roff[t + 1] + g.hcol] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < R; t++) {
                double bl, br, ulx, ur;
                x_edges<double, PB_M>(g, bq[t], hb[t], bl, br);
                x_edges<double, PB_M>(g, vx[t], hu[t], ulx, ur);
                (void)ulx;
                // x fluxes: left face of cell 0, between the cells, right face of cell 1
                const double F[3] = {0.5 * (bl + bq[t].v[0]) * vx[t].v[0],
                                     0.5 * (bq[t].v[0] + bq[t].v[1]) * vx[t].v[1], 0.5 * (bq[t].v[1] + br) * ur};
                const S2& below = t == 0 ? blo : bq[t > 0 ? t - 1 : 0];
                const S2& above = t == R - 1 ? bhi : bq[t < R - 1 ? t + 1 : 0];
                S2 out;
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const double b0 = bq[t].v[c];
                    const double fyl = 0.5 * (below.v[c] + b0) * vy[t].v[c];
                    const double fyh = 0.5 * (b0 + above.v[c]) * vy[t + 1].v[c];
                    const double fzh = hzp ? 0.5 * (b0 + bn[t].v[c]) * vz[t].v[c] : 0.0;
                    const double div = ((F[c + 1] - F[c]) + (fyh - fyl) + (fzh - fzl[t][c])) * inv_h;
                    const double v = b0 * src_of(d, sv[t].v[c], sbar, smode, g.xi + c, g.j0 + t, k) - div;
                    if (shift) {
                        const double e2 = v - sh0;
                        acc = fma(e2, e2, acc);
                    } else {
                        acc += v;
                        acc2 = fma(v, v, acc2);
                    }
                    out.v[c] = v;
                    fzl[t][c] = fzh;
                }
                if (!shift) st_strip<double, PB_M>(b, pk + roff[t + 1] + g.xi, out);
            }
#pragma unroll
            for (int t = 0; t < R; t++) bq[t] = bn[t];
        }
    }
    const long long bid = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[bid] = s;
    if (part2) {
        const double s2 = block_sum(acc2, sh);
        if (threadIdx.x == 0) part2[bid] = s2;
    }
}

// U <- U - (c / beta0_f) G phi on the low faces of every cell (the cell owns
// them), c the harmonic mean of the cell values beta0/rho; a Neumann z wall
// keeps its value.
__global__ __launch_bounds__(BK_T) void k_vc_blk(Dims d, int lz, double inv_h, const double* __restrict__ cc,
                                                 const double* __restrict__ beta0, const double* __restrict__ phi,
                                                 double* __restrict__ ux, double* __restrict__ uy,
                                                 double* __restrict__ uz)
{
    constexpr int R = PB_R;
    const BlkGeo g = blk_geo<PB_M, R>(d, lz);
    if (!g.live) return;
    const long long sz = (long long)d.nx * d.ny;
    long long roff[R + 1];  // rows j0-1 .. j0+R-1 (wrapped)
#pragma unroll
    for (int t = 0; t < R + 1; t++) roff[t] = (long long)wrap_row(d, g.j0 - 1 + t) * d.nx;
    // the previous plane (z low neighbours) of rows j0 .. j0+R-1
    S2 cm[R], bm[R], pm[R];
    const bool hzm0 = g.z0 > 0 || d.pz;
#pragma unroll
    for (int t = 0; t < R; t++) {
        const long long q = (long long)wrap_plane(d, g.z0 - 1) * sz + roff[t + 1] + g.xi;
        cm[t] = ld_strip<double, PB_M>(cc, q);
        bm[t] = ld_strip<double, PB_M>(beta0, q);
        pm[t] = ld_strip<double, PB_M>(phi, q);
    }
    (void)hzm0;
    for (int k = g.z0; k < g.z1; k++) {
        const long long pk = (long long)k * sz;
        const bool hzm = k > 0 || d.pz;
        S2 c[R + 1], bb[R + 1], p[R + 1];
#pragma unroll
        for (int t = 0; t <= R; t++) {
            const long long q = pk + roff[t] + g.xi;
            c[t] = ld_strip<double, PB_M>(cc, q);
            bb[t] = ld_strip<double, PB_M>(beta0, q);
            p[t] = ld_strip<double, PB_M>(phi, q);
        }
        double hc[R], hb[R], hp[R];
        S2 vx[R], vy[R], vz[R];
#pragma unroll
        for (int t = 0; t < R; t++) {
            const long long q = pk + roff[t + 1] + g.xi;
            hc[t] = g.hal ? cc[pk + roff[t + 1] + g.hcol] : 0.0;
            hb[t] = g.hal ? beta0[pk + roff[t + 1] + g.hcol] : 0.0;
            hp[t] = g.hal ? phi[pk + roff[t + 1] + g.hcol] : 0.0;
            vx[t] = ld_strip<double, PB_M>(ux, q);
            vy[t] = ld_strip<double, PB_M>(uy, q);
            vz[t] = ld_strip<double, PB_M>(uz, q);
        }
#pragma unroll
        for (int t = 0; t < R; t++) {
            const S2& co = c[t + 1];
            const S2& bo = bb[t + 1];
            const S2& po = p[t + 1];
            double cl, cr_, bl, br_, pl, pr_;
            x_edges<double, PB_M>(g, co, hc[t], cl, cr_);
            x_edges<double, PB_M>(g, bo, hb[t], bl, br_);
            x_edges<double, PB_M>(g, po, hp[t], pl, pr_);
            (void)cr_;
            (void)br_;
            (void)pr_;
            S2 nx_, ny_, nz_;
#pragma unroll
            for (int q = 0; q < 2; q++) {
                // x low face: the neighbour on the left is the previous cell of
                // the strip, or the previous lane's last cell
                const double ccl = q == 0 ? cl : co.v[0];
                const double bbl = q == 0 ? bl : bo.v[0];
                const double ppl = q == 0 ? pl : po.v[0];
                nx_.v[q] = vx[t].v[q] - harm(ccl, co.v[q]) / (0.5 * (bbl + bo.v[q])) * ((po.v[q] - ppl) * inv_h);
                ny_.v[q] = vy[t].v[q] -
                           harm(c[t].v[q], co.v[q]) / (0.5 * (bb[t].v[q] + bo.v[q])) * ((po.v[q] - p[t].v[q]) * inv_h);
                nz_.v[q] = vz[t].v[q] -
                           harm(cm[t].v[q], co.v[q]) / (0.5 * (bm[t].v[q] + bo.v[q])) * ((po.v[q] - pm[t].v[q]) * inv_h);
            }
            const long long q = pk + roff[t + 1] + g.xi;
            st_strip<double, PB_M>(ux, q, nx_);
            st_strip<double, PB_M>(uy, q, ny_);
            if (hzm) st_strip<double, PB_M>(uz, q, nz_);
            cm[t] = co;
            bm[t] = bo;
            pm[t] = po;
        }
    }
}

void launch_rhs_blk(const Dims& d, double inv_h, const double* beta0, const double* ux, const double* uy,
                    const double* uz, const double* S, const double* sbar, int smode, double* b, const double* shift,
                    double* partials, int* nb_out, hipStream_t s, double* partials2)
{
    int lz = 0;
    const dim3 grid = blk_grid(d, PB_M, PB_R, kBlkMinBlocks, kMaxRedBlocks, lz);
    *nb_out = (int)(grid.x * grid.y * grid.z);
    hipLaunchKernelGGL(k_rhs_blk, grid, dim3(BK_T), 0, s, d, lz, inv_h, beta0, ux, uy, uz, S, sbar, smode, b,
                       partials, shift, shift ? nullptr : partials2);
}

void launch_vc_blk(const Dims& d, double inv_h, const double* cc, const double* beta0, const double* phi, double* ux,
                   double* uy, double* uz, hipStream_t s)
{
    int lz = 0;
    const dim3 grid = blk_grid(d, PB_M, PB_R, kBlkMinBlocks, 1LL << 30, lz);
    hipLaunchKernelGGL(k_vc_blk, grid, dim3(BK_T), 0, s, d, lz, inv_h, cc, beta0, phi, ux, uy, uz);
}

int proj_blk_reduce_blocks(const Dims& d)
{
    int lz = 0;
    const dim3 grid = blk_grid(d, PB_M, PB_R, kBlkMinBlocks, kMaxRedBlocks, lz);
    return (int)(grid.x * grid.y * grid.z);
}

}  // namespace mp
