// k_coarse.hip -- the coarse end of a V-cycle in one workgroup.
//
// On the smallest levels (a few hundred cells) a kernel finishes in well under
// the cost of a launch, so a V-cycle would spend its coarse-grid time in launch
// gaps.
// This kernel runs every level of the coarse set (pre-smoothing, residual
// restriction, bottom solve, prolongation, post-smoothing) in a single
// 1024-thread workgroup, separated by workgroup barriers, with every array of
// the set held in LDS (up to kCoarseLdsBytes; 160 KB per CU on gfx950).  The per-cell
// arithmetic is the shared code of the one-launch-per-operation kernels, so
// the smoother and the transfers agree with them bit for bit.
//
// The bottom solve is conjugate gradients in FP64 run by the first wavefront
// alone: each lane holds up to NS cells in registers, neighbour values come
// from cross-lane shuffles and dot products from wavefront reductions
// broadcast from lane 0, so no barrier is needed inside the iteration.
#include "mp_device.h"
#include "mp_kernels.h"

namespace mp {

// Value of cell nq of a register-distributed vector (cell q lives in lane
// q % 64, slot q / 64).  Every lane must call this (it shuffles).
template <int NS>
__device__ __forceinline__ double wave_get(const double (&v)[NS], int nq)
{
    const int src = nq & (kWave - 1), slot = nq >> 6;
    double r = 0.0;
#pragma unroll
    for (int t = 0; t < NS; t++) {
        const double u = __shfl(v[t], src, kWave);
        if (t == slot) r = u;
    }
    return r;
}

// Wavefront minimum broadcast from lane 0.
__device__ __forceinline__ double wave_min_bcast(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return __shfl(v, 0, kWave);
}

template <typename T, int NS>
__device__ void wave_cg(const Dims& d, const T* __restrict__ bin, T* __restrict__ xout,
                              const T* __restrict__ cx, const T* __restrict__ cy, const T* __restrict__ cz, double h2,
                              double rtol, int maxit, double* __restrict__ iters)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int n = (int)d.n();
    const double inv_h2 = 1.0 / h2;
    // per-slot cell data: coefficients and neighbour indices
    double c[NS][6];
    int nbi[NS][6];
    bool live[NS];
    double b[NS], x[NS], r[NS], p[NS], v[NS];
#pragma unroll
    for (int u = 0; u < NS; u++) {
        const int q = lane + kWave * u;
        live[u] = q < n;
        const int qq = live[u] ? q : 0;
        int i, j, k;
        cell_ijk(d, qq, i, j, k);
        const Nbr nb = neighbours(d, qq, i, j, k);
        c[u][0] = cx[qq];
        c[u][1] = (double)ld_or0(cx, nb.cxp);
        c[u][2] = cy[qq];
        c[u][3] = (double)ld_or0(cy, nb.cyp);
        c[u][4] = cz[qq];
        c[u][5] = (double)ld_or0(cz, nb.czp);
        nbi[u][0] = (int)nb.xm;
        nbi[u][1] = (int)nb.xp;
        nbi[u][2] = (int)nb.ym;
        nbi[u][3] = (int)nb.yp;
        nbi[u][4] = (int)nb.zm;
        nbi[u][5] = (int)nb.zp;
        b[u] = live[u] ? (double)bin[qq] : 0.0;
    }
    // Connected parts of the grid: each cell's label becomes the smallest
    // cell index joined to it through nonzero faces (minimum-label
    // propagation, settled within a part's diameter).  The constants on each
    // part span the null space of the operator, so the right-hand side, the
    // residual and the result are made mean-zero part by part: a right-hand
    // side left with a component on a part's constant (rounding, where the
    // cells are not all coupled) would otherwise drive the iterates along
    // that constant without bound.  With every cell coupled this is the plain
    // mean removal, in the same operations.
    double lab[NS];
#pragma unroll
    for (int u = 0; u < NS; u++) lab[u] = live[u] ? (double)(lane + kWave * u) : (double)n;
    for (;;) {
        double nl[NS];
        int changed = 0;
#pragma unroll
        for (int u = 0; u < NS; u++) {
            double m = lab[u];
#pragma unroll
            for (int f = 0; f < 6; f++) {
                const double w = wave_get<NS>(lab, nbi[u][f]);
                if (live[u] && c[u][f] != 0.0 && w < m) m = w;
            }
            nl[u] = m;
            changed |= m != lab[u];
        }
#pragma unroll
        for (int u = 0; u < NS; u++) lab[u] = nl[u];
        if (wave_sum_bcast((double)changed) == 0.0) break;
    }
    auto demean = [&](double (&y)[NS]) {
        double lo = (double)n;
#pragma unroll
        for (int u = 0; u < NS; u++)
            if (live[u]) lo = fmin(lo, lab[u]);
        double cur = wave_min_bcast(lo);
        while (cur < (double)n) {
            double s = 0.0, cnt = 0.0, nxt = (double)n;
#pragma unroll
            for (int u = 0; u < NS; u++) {
                if (live[u] && lab[u] == cur) {
                    s += y[u];
                    cnt += 1.0;
                }
                if (live[u] && lab[u] > cur) nxt = fmin(nxt, lab[u]);
            }
            const double m = wave_sum_bcast(s) / wave_sum_bcast(cnt);
#pragma unroll
            for (int u = 0; u < NS; u++)
                if (live[u] && lab[u] == cur) y[u] -= m;
            cur = wave_min_bcast(nxt);
        }
    };
    demean(b);
#pragma unroll
    for (int u = 0; u < NS; u++) {
        x[u] = 0.0;
        r[u] = b[u];
        p[u] = b[u];
    }
    auto apply = [&](const double (&y)[NS], double (&out)[NS]) {
#pragma unroll
        for (int u = 0; u < NS; u++) {
            double nv[6];
#pragma unroll
            for (int f = 0; f < 6; f++) nv[f] = wave_get<NS>(y, nbi[u][f]);
            const double csum = ((((c[u][0] + c[u][1]) + c[u][2]) + c[u][3]) + c[u][4]) + c[u][5];
            double sv = c[u][0] * nv[0];
#pragma unroll
            for (int f = 1; f < 6; f++) sv = fma(c[u][f], nv[f], sv);
            out[u] = live[u] ? (csum * y[u] - sv) * inv_h2 : 0.0;
        }
    };
    auto dot = [&](const double (&a)[NS], const double (&bb)[NS]) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < NS; u++) acc = fma(a[u], bb[u], acc);
        return wave_sum_bcast(acc);
    };
    // conjugate gradients: A is symmetric and positive on vectors mean-zero
    // on every part; the residual is kept so against rounding.  An
    // unconverged solve returns the iterate of the smallest residual; a
    // converged one returns its last iterate.
    double rr = dot(r, r);
    const double tol2 = rtol * rtol * rr;
    double rr_best = rr;
    double xb[NS];
#pragma unroll
    for (int u = 0; u < NS; u++) xb[u] = x[u];
    int it = 0;
    for (; it < maxit && rr > tol2 && rr > 0.0; it++) {
        apply(p, v);
        const double pv = dot(p, v);
        if (!(pv > 0.0)) break;
        const double alpha = rr / pv;
#pragma unroll
        for (int u = 0; u < NS; u++) {
            x[u] = fma(alpha, p[u], x[u]);
            r[u] = live[u] ? fma(-alpha, v[u], r[u]) : 0.0;
        }
        demean(r);
        const double rr1 = dot(r, r);
        const double beta = rr1 / rr;
        rr = rr1;
        if (rr1 < rr_best) {
            rr_best = rr1;
#pragma unroll
            for (int u = 0; u < NS; u++) xb[u] = x[u];
        }
#pragma unroll
        for (int u = 0; u < NS; u++) p[u] = fma(beta, p[u], r[u]);
    }
    if (rr <= tol2) {
#pragma unroll
        for (int u = 0; u < NS; u++) xb[u] = x[u];
    }
    // iterations of this solve added to the caller's running count (one
    // lane; the solves of a stream run one after another)
    if (iters && lane == 0) iters[0] += (double)it;
    demean(xb);
#pragma unroll
    for (int u = 0; u < NS; u++)
        if (live[u]) xout[lane + kWave * u] = (T)xb[u];
}

// ---- direct bottom solve ----------------------------------------------------
// A workgroup of 1024 threads applies G: thread t holds G[t % 64][4 (t / 64)
// .. 4 (t / 64) + 3], forms its four products, and the first wavefront sums
// the sixteen partials of each row in a fixed order.
constexpr int kGRow = kDirectBottomCells;
static_assert(kGRow == 64, "one row of G per lane of a wavefront");

__device__ __forceinline__ void load_ginv(const double* __restrict__ G, double (&g)[4])
{
    const int t = (int)threadIdx.x, r = t & (kGRow - 1), cb = t / kGRow;
    const double2* p = reinterpret_cast<const double2*>(G + r * kGRow + 4 * cb);
    const double2 u = p[0], v = p[1];
    g[0] = u.x;
    g[1] = u.y;
    g[2] = v.x;
    g[3] = v.y;
}

// x = h2 (G b - mean(G b)) on n <= 64 cells; part: 1024 doubles of LDS.
// Ends with the first wavefront's stores (the caller synchronises).
template <typename T>
__device__ void direct_bottom(int n, const double (&g)[4], const T* b, T* x, double h2, double* part)
{
    const int t = (int)threadIdx.x, r = t & (kGRow - 1), cb = t / kGRow;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int col = 4 * cb + u;
        s = fma(g[u], col < n ? (double)b[col] : 0.0, s);
    }
    part[cb * kGRow + r] = s;
    __syncthreads();
    if (t < kWave) {
        double y = 0.0;
#pragma unroll
        for (int k = 0; k < 16; k++) y += part[k * kGRow + t];
        if (t >= n) y = 0.0;
        const double m = wave_sum_bcast(y) / n;
        if (t < n) x[t] = (T)(h2 * (y - m));
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_bottom_direct(int n, const double* __restrict__ G,
                                                        const double* __restrict__ valid, const T* __restrict__ b,
                                                        T* __restrict__ x, double h2)
{
    __shared__ double part[1024];
    if (valid[0] != 1.0) return;
    double g[4];
    load_ginv(G, g);
    direct_bottom<T>(n, g, b, x, h2, part);
}

template <typename T>
void launch_bottom_direct(const Dims& d, const double* G, const double* valid, const T* b, T* x, double h2,
                          hipStream_t s)
{
    hipLaunchKernelGGL((k_bottom_direct<T>), dim3(1), dim3(1024), 0, s, (int)d.n(), G, valid, b, x, h2);
}

// G = (L + alpha 1 1^T)^-1 by Gauss-Jordan elimination on [B | I] (B in
// columns 0..63, I in columns 64..127), held in registers: thread t owns
// column t % 128 of rows 8 (t / 128) .. +7.  Per pivot the owners of the
// next pivot's column and row publish them to LDS (double-buffered), so one
// barrier separates consecutive pivots.
template <typename T>
__global__ __launch_bounds__(1024) void k_bottom_inverse(Dims d, const T* __restrict__ cx, const T* __restrict__ cy,
                                                         const T* __restrict__ cz, double* __restrict__ G,
                                                         double* __restrict__ valid)
{
    __shared__ double Ls[kGRow][kGRow];
    __shared__ double fb[2][kGRow], pb[2][2 * kGRow], ip[2];
    __shared__ double sc[2];
    const int n = (int)d.n(), t = (int)threadIdx.x;
    for (int e = t; e < kGRow * kGRow; e += (int)blockDim.x) Ls[e / kGRow][e % kGRow] = 0.0;
    __syncthreads();
    // row q of L (one thread per row: no two threads write one entry)
    if (t < n) {
        int i, j, k;
        cell_ijk(d, t, i, j, k);
        const Nb32 nb = nb32(d, t, i, j, k);
        const double c[6] = {(double)cx[t], nb.hx ? (double)cx[nb.xp] : 0.0, (double)cy[t],
                             nb.hy ? (double)cy[nb.yp] : 0.0, (double)cz[t], nb.hz ? (double)cz[nb.zp] : 0.0};
        const int nq[6] = {nb.xm, nb.xp, nb.ym, nb.yp, nb.zm, nb.zp};
        Ls[t][t] += ((((c[0] + c[1]) + c[2]) + c[3]) + c[4]) + c[5];
#pragma unroll
        for (int f = 0; f < 6; f++) Ls[t][nq[f]] -= c[f];
    }
    __syncthreads();
    if (t == 0) {
        double tr = 0.0, mx = 0.0;
        for (int q = 0; q < n; q++) {
            tr += Ls[q][q];
            mx = fmax(mx, Ls[q][q]);
        }
        sc[0] = tr / ((double)n * n);
        sc[1] = 1e-12 * (mx + sc[0]);
    }
    __syncthreads();
    const double alpha = sc[0], thr = sc[1];
    const int col = t % (2 * kGRow), rg = t / (2 * kGRow);
    double m[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const int r = rg * 8 + u;
        if (col < kGRow)
            m[u] = (r < n && col < n) ? Ls[r][col] + alpha : 0.0;
        else
            m[u] = (r < n && col - kGRow == r) ? 1.0 : 0.0;
    }
    // pivot 0's column and row
    if (col == 0) {
#pragma unroll
        for (int u = 0; u < 8; u++) fb[0][rg * 8 + u] = m[u];
    }
    if (rg == 0) pb[0][col] = m[0];
    if (t == 0) ip[0] = 1.0 / m[0];
    __syncthreads();
    bool good = alpha > 0.0;
    for (int p = 0; p < n && good; p++) {
        const int cur = p & 1, nxt = cur ^ 1;
        good = fb[cur][p] > thr;  // the same value in every thread
        if (!good) break;
        // the pivot's reciprocal comes from the thread that published the
        // pivot row (one division per pivot)
        const double v = pb[cur][col] * ip[cur];
        // the column's eight factors read before the updates, so the reads
        // issue together; only the pivot row's group (whole wavefronts)
        // selects the scaled row for row p
        double f[8];
#pragma unroll
        for (int u = 0; u < 8; u++) f[u] = fb[cur][rg * 8 + u];
        if (rg == p / 8) {
#pragma unroll
            for (int u = 0; u < 8; u++) m[u] = rg * 8 + u == p ? v : fma(-f[u], v, m[u]);
        } else {
#pragma unroll
            for (int u = 0; u < 8; u++) m[u] = fma(-f[u], v, m[u]);
        }
        if (p + 1 < n) {
            if (col == p + 1) {
#pragma unroll
                for (int u = 0; u < 8; u++) fb[nxt][rg * 8 + u] = m[u];
            }
            if (rg == (p + 1) / 8) {
                double w = 0.0;
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (u == (p + 1) % 8) w = m[u];
                pb[nxt][col] = w;
                if (col == p + 1) ip[nxt] = 1.0 / w;
            }
        }
        __syncthreads();
    }
    if (col >= kGRow) {
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int r = rg * 8 + u, c = col - kGRow;
            G[r * kGRow + c] = (good && r < n && c < n) ? m[u] : 0.0;
        }
    }
    if (t == 0) valid[0] = good ? 1.0 : 0.0;
}

template <typename T>
void launch_bottom_inverse(const Dims& d, const T* cx, const T* cy, const T* cz, double* G, double* valid,
                           hipStream_t s)
{
    hipLaunchKernelGGL((k_bottom_inverse<T>), dim3(1), dim3(1024), 0, s, d, cx, cy, cz, G, valid);
}

// The six low/high face coefficients of cell q (the values of coef6 in face
// mode: a high face on a wall is 0).
template <typename T>
__device__ __forceinline__ void cc_coef(const CoarseLevel<T>& L, int q, const Nb32& b, T (&c)[6])
{
    const T xh = L.cx[b.xp], yh = L.cy[b.yp], zh = L.cz[b.zp];
    c[0] = L.cx[q];
    c[1] = b.hx ? xh : T(0);
    c[2] = L.cy[q];
    c[3] = b.hy ? yh : T(0);
    c[4] = L.cz[q];
    c[5] = b.hz ? zh : T(0);
}

// One red-black sweep of a level in LDS: the cell arithmetic of rbgs_cell
// (gs_value on the same operands), with 32-bit indexing.
template <typename T>
__device__ void cg_smooth(const CoarseLevel<T>& L, const Dims& d, int zero_init)
{
    const int nxh = (d.nx + 1) / 2;
    const int cnt = nxh * d.ny * d.nz;
    const FastDiv fa((unsigned)nxh), fb((unsigned)d.ny);
    for (int colour = 0; colour < 2; colour++) {
        const bool zi = zero_init && colour == 0;
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
            int p, j, k;
            split3((unsigned)e, fa, fb, p, j, k);
            const int par = (j + k + colour) & 1;
            const int i = 2 * p + par;
            const int rbase = (k * d.ny + j) * d.nx;
            if (zi) {
                // x is zero on entry: clear the other cell of the pair
                const int io = 2 * p + (1 - par);
                if (io < d.nx) L.x[rbase + io] = T(0);
            }
            if (i >= d.nx) continue;
            const int q = rbase + i;
            const Nb32 nb = nb32(d, q, i, j, k);
            T c[6];
            cc_coef<T>(L, q, nb, c);
            if (zi)
                L.x[q] = gs_value<T>(c[0], c[1], c[2], c[3], c[4], c[5], T(0), T(0), T(0), T(0), T(0), T(0), L.b[q],
                                     L.h2, T(0));
            else
                L.x[q] = gs_value<T>(c[0], c[1], c[2], c[3], c[4], c[5], L.x[nb.xm], L.x[nb.xp], L.x[nb.ym],
                                     L.x[nb.yp], L.x[nb.zm], L.x[nb.zp], L.b[q], L.h2, L.x[q]);
        }
        __syncthreads();
    }
}

// ---- thread-owned cells ------------------------------------------------------
// A level's cells taken in pairs (2p, 2p + 1) of a row, one of each colour.
// Thread t owns pairs t + 1024 u (u < U) and holds, for a whole visit of the
// level, each cell's index, neighbour indices, six coefficients, their sum
// and its right-hand side in registers: a colour pass is then six LDS reads,
// the stencil sums and one write per cell instead of index arithmetic and
// thirteen reads.  gs_value and resid_value arithmetic in the same order
// (the same bits as cg_smooth and cc_resid).
// pairs per thread at most (FP32: levels of <= 2048 pairs; FP64: 1024, whose
// registers would not hold two)
template <typename T>
constexpr int own_max() { return sizeof(T) == 4 ? 2 : 1; }

template <typename T, int U>
struct Owned {
    int q[U][2];  // cell of colour s of pair u, -1 when the row has no such cell
    int nb[U][2][6];
    T c[U][2][6];
    T cs[U][2];
    T b[U][2];
};

template <typename T, int U>
__device__ __forceinline__ void own_load(Owned<T, U>& o, const CoarseLevel<T>& L, const Dims& d)
{
    const int nxh = (d.nx + 1) / 2, np = nxh * d.ny * d.nz;
    const FastDiv fa((unsigned)nxh), fb((unsigned)d.ny);
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int e = (int)threadIdx.x + 1024 * u;
        int p = 0, j = 0, k = 0;
        if (e < np) split3((unsigned)e, fa, fb, p, j, k);
#pragma unroll
        for (int s = 0; s < 2; s++) {
            int i = 2 * p + ((j + k + s) & 1);
            const bool live = e < np && i < d.nx;
            if (!live) i = 0;
            const int q = (k * d.ny + j) * d.nx + i;
            const Nb32 nb = nb32(d, q, i, j, k);
            T c[6];
            cc_coef<T>(L, q, nb, c);
            o.q[u][s] = live ? q : -1;
            o.nb[u][s][0] = nb.xm;
            o.nb[u][s][1] = nb.xp;
            o.nb[u][s][2] = nb.ym;
            o.nb[u][s][3] = nb.yp;
            o.nb[u][s][4] = nb.zm;
            o.nb[u][s][5] = nb.zp;
#pragma unroll
            for (int f = 0; f < 6; f++) o.c[u][s][f] = c[f];
            o.cs[u][s] = coef_sum<T>(c[0], c[1], c[2], c[3], c[4], c[5]);
            o.b[u][s] = L.b[q];
        }
    }
}

// One red-black sweep over the owned cells (zero_init: x is zero on entry).
template <typename T, int U>
__device__ void own_smooth(const Owned<T, U>& o, const CoarseLevel<T>& L, bool zero_init)
{
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const bool zi = zero_init && s == 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int q = o.q[u][s];
            const T(&c)[6] = o.c[u][s];
            if (zi) {
                // the pair's other cell is cleared; the neighbours count as 0
                if (o.q[u][1] >= 0) L.x[o.q[u][1]] = T(0);
                if (q >= 0)
                    L.x[q] = gs_value_cs<T>(o.cs[u][s], c[0], c[1], c[2], c[3], c[4], c[5], T(0), T(0), T(0), T(0),
                                            T(0), T(0), o.b[u][s], L.h2, T(0));
            } else if (q >= 0 && o.cs[u][s] > T(0)) {
                const int(&n)[6] = o.nb[u][s];
                const T xm = L.x[n[0]], xp = L.x[n[1]], ym = L.x[n[2]], yp = L.x[n[3]], zm = L.x[n[4]],
                        zp = L.x[n[5]];
                L.x[q] = gs_value_cs<T>(o.cs[u][s], c[0], c[1], c[2], c[3], c[4], c[5], xm, xp, ym, yp, zm, zp,
                                        o.b[u][s], L.h2, L.x[q]);
            }
        }
        __syncthreads();
    }
}

// Residuals of the owned cells into rs (indexed by cell).
template <typename T, int U>
__device__ __forceinline__ void own_resid(const Owned<T, U>& o, const CoarseLevel<T>& L, T* rs)
{
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const int q = o.q[u][s];
            if (q < 0) continue;
            const T(&c)[6] = o.c[u][s];
            const int(&n)[6] = o.nb[u][s];
            rs[q] = resid_value_cs<T>(o.cs[u][s], c[0], c[1], c[2], c[3], c[4], c[5], L.x[n[0]], L.x[n[1]],
                                      L.x[n[2]], L.x[n[3]], L.x[n[4]], L.x[n[5]], L.x[q], o.b[u][s], L.inv_h2);
        }
}

// Residual of cell q = (i, j, k): the arithmetic of resid_cell.
template <typename T>
__device__ __forceinline__ T cc_resid(const CoarseLevel<T>& L, const Dims& d, int q, int i, int j, int k)
{
    const Nb32 nb = nb32(d, q, i, j, k);
    T c[6];
    cc_coef<T>(L, q, nb, c);
    return resid_value<T>(c[0], c[1], c[2], c[3], c[4], c[5], L.x[nb.xm], L.x[nb.xp], L.x[nb.ym], L.x[nb.yp],
                          L.x[nb.zm], L.x[nb.zp], L.x[q], L.b[q], L.inv_h2);
}

// Extents of coarse level l (from the kernel arguments: an array of them in
// the kernel would live in scratch memory, indexed at run time).
template <typename T>
__device__ __forceinline__ Dims cdims(const CoarseArgs<T>& a, int l)
{
    return Dims{a.lv[l].nx, a.lv[l].ny, a.lv[l].nz, a.px, a.py, a.pz};
}

// The arrays of every coarse level (x, b and the three low-face
// coefficients) staged in LDS for the whole cycle: level l starts at
// 5 * (cells of the levels above it), in the order x, b, cx, cy, cz.
template <typename T>
__device__ __forceinline__ CoarseLevel<T> lds_level(const CoarseArgs<T>& a, int l, T* lds)
{
    long long off = 0;
    for (int q = 0; q < l; q++) off += 5LL * a.lv[q].nx * a.lv[q].ny * a.lv[q].nz;
    const long long n = (long long)a.lv[l].nx * a.lv[l].ny * a.lv[l].nz;
    CoarseLevel<T> L = a.lv[l];
    L.x = lds + off;
    L.b = lds + off + n;
    L.cx = lds + off + 2 * n;
    L.cy = lds + off + 3 * n;
    L.cz = lds + off + 4 * n;
    return L;
}

// 16-byte vector of T.
template <typename T>
struct V16;
template <>
struct V16<float> {
    using type = float4;
    static constexpr int k = 4;
};
template <>
struct V16<double> {
    using type = double2;
    static constexpr int k = 2;
};

template <typename T, int NS>
__global__ __launch_bounds__(1024) void k_coarse_cycle(CoarseArgs<T> a)
{
    __shared__ T lds[kCoarseLdsBytes / sizeof(T)];
    __shared__ double part[1024];  // the direct bottom's partial sums
    const int nl = a.nlev;
    // residual scratch for the restrictions, after the last level
    T* rs = lds_level(a, nl - 1, lds).x + 5 * cdims(a, nl - 1).n();
    // this thread's entries of G (direct bottom), loaded while the levels stage
    const bool direct = a.bottom_inv && a.bottom_ok[0] == 1.0;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    if (direct) load_ginv(a.bottom_inv, g);
    // stage the coefficients of every level and the right-hand side (and,
    // unless it starts from zero, the iterate) of the top level, 16 bytes
    // per access where the level allows it
    for (int l = 0; l < nl; l++) {
        const CoarseLevel<T> S = lds_level(a, l, lds);
        const int n = (int)cdims(a, l).n();
        const bool top = l == 0, xin = l == 0 && !a.zero_init;
        if (n % (int)V16<T>::k == 0) {
            using V = typename V16<T>::type;
            const int nv = n / (int)V16<T>::k;
            for (int e = threadIdx.x; e < nv; e += blockDim.x) {
                const V vx = ((const V*)a.lv[l].cx)[e], vy = ((const V*)a.lv[l].cy)[e], vz = ((const V*)a.lv[l].cz)[e];
                V vb, vi;
                if (top) vb = ((const V*)a.lv[0].b)[e];
                if (xin) vi = ((const V*)a.lv[0].x)[e];
                ((V*)S.cx)[e] = vx;
                ((V*)S.cy)[e] = vy;
                ((V*)S.cz)[e] = vz;
                if (top) ((V*)S.b)[e] = vb;
                if (xin) ((V*)S.x)[e] = vi;
            }
        } else {
            for (int e = threadIdx.x; e < n; e += blockDim.x) {
                const_cast<T*>(S.cx)[e] = a.lv[l].cx[e];
                const_cast<T*>(S.cy)[e] = a.lv[l].cy[e];
                const_cast<T*>(S.cz)[e] = a.lv[l].cz[e];
                if (top) S.b[e] = a.lv[0].b[e];
                if (xin) S.x[e] = a.lv[0].x[e];
            }
        }
    }
    __syncthreads();
    // down
    for (int l = 0; l < nl - 1; l++) {
        const CoarseLevel<T> L = lds_level(a, l, lds);
        const int zi = (l > 0) || a.zero_init;
        if (zi && a.nu1 == 0) {
            const int cnt0 = a.lv[l].nx * a.lv[l].ny * a.lv[l].nz;
            for (int e = threadIdx.x; e < cnt0; e += blockDim.x) L.x[e] = T(0);
            __syncthreads();
        }
        const Dims f = cdims(a, l);
        const int nxc = f.nx / 2, nyc = f.ny / 2, nzc = f.nz / 2;
        const int cnt = nxc * nyc * nzc;
        T* bc = lds_level(a, l + 1, lds).b;
        // residual restriction in two parallel phases: every fine residual
        // into the scratch, then the 8 children of each coarse cell summed in
        // the order of restrict_cell (the same bits)
        const int nf = (int)f.n();
        const FastDiv fx((unsigned)f.nx), fy((unsigned)f.ny), fxc((unsigned)nxc), fyc((unsigned)nyc);
        const int npair = (f.nx + 1) / 2 * f.ny * f.nz;
        if (npair <= 1024) {
            Owned<T, 1> o;
            own_load<T, 1>(o, L, f);
            for (int s = 0; s < a.nu1; s++) own_smooth<T, 1>(o, L, zi && s == 0);
            own_resid<T, 1>(o, L, rs);
        } else if (own_max<T>() > 1 && npair <= 1024 * own_max<T>()) {
            Owned<T, own_max<T>()> o;
            own_load<T, own_max<T>()>(o, L, f);
            for (int s = 0; s < a.nu1; s++) own_smooth<T, own_max<T>()>(o, L, zi && s == 0);
            own_resid<T, own_max<T>()>(o, L, rs);
        } else {
            for (int s = 0; s < a.nu1; s++) cg_smooth<T>(L, f, zi && s == 0);
            for (int e = threadIdx.x; e < nf; e += blockDim.x) {
                int i, j, k;
                split3((unsigned)e, fx, fy, i, j, k);
                rs[e] = cc_resid<T>(L, f, e, i, j, k);
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
            int I, J, K;
            split3((unsigned)e, fxc, fyc, I, J, K);
            T acc = T(0);
#pragma unroll
            for (int c = 0; c < 2; c++)
#pragma unroll
                for (int bb = 0; bb < 2; bb++)
#pragma unroll
                    for (int aa = 0; aa < 2; aa++)
                        acc += rs[((2 * K + c) * f.ny + 2 * J + bb) * f.nx + 2 * I + aa];
            bc[e] = T(0.125) * acc;
        }
        __syncthreads();
    }
    // bottom: directly from G, or conjugate gradients in the first wavefront
    // (the others wait at the barrier below)
    if (direct) {
        const CoarseLevel<T> B = lds_level(a, nl - 1, lds);
        direct_bottom<T>((int)cdims(a, nl - 1).n(), g, B.b, B.x, B.h2d, part);
    } else if (threadIdx.x < kWave) {
        const CoarseLevel<T> B = lds_level(a, nl - 1, lds);
        wave_cg<T, NS>(cdims(a, nl - 1), B.b, B.x, B.cx, B.cy, B.cz, B.h2d, a.bottom_rtol, a.bottom_maxit,
                       a.bottom_iters);
    }
    __syncthreads();
    // up
    for (int l = nl - 2; l >= 0; l--) {
        const CoarseLevel<T> L = lds_level(a, l, lds);
        const Dims f = cdims(a, l);
        const int nxc = f.nx / 2, nyc = f.ny / 2;
        const int cnt = f.nx * f.ny * f.nz;
        const T* ec = lds_level(a, l + 1, lds).x;
        const FastDiv fx((unsigned)f.nx), fy((unsigned)f.ny);
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
            int i, j, k;
            split3((unsigned)e, fx, fy, i, j, k);
            L.x[e] += ec[((k >> 1) * nyc + (j >> 1)) * nxc + (i >> 1)];
        }
        __syncthreads();
        const int npair = (f.nx + 1) / 2 * f.ny * f.nz;
        if (npair <= 1024) {
            Owned<T, 1> o;
            own_load<T, 1>(o, L, f);
            for (int s = 0; s < a.nu2; s++) own_smooth<T, 1>(o, L, false);
        } else if (own_max<T>() > 1 && npair <= 1024 * own_max<T>()) {
            Owned<T, own_max<T>()> o;
            own_load<T, own_max<T>()>(o, L, f);
            for (int s = 0; s < a.nu2; s++) own_smooth<T, own_max<T>()>(o, L, false);
        } else {
            for (int s = 0; s < a.nu2; s++) cg_smooth<T>(L, f, 0);
        }
    }
    // the top level's iterate goes back to the finer level's prolongation
    {
        const CoarseLevel<T> L = lds_level(a, 0, lds);
        const int n = (int)cdims(a, 0).n();
        for (int e = threadIdx.x; e < n; e += blockDim.x) a.lv[0].x[e] = L.x[e];
    }
}

template <typename T>
void launch_coarse_cycle(const CoarseArgs<T>& a, hipStream_t s)
{
    const int nb = a.lv[a.nlev - 1].nx * a.lv[a.nlev - 1].ny * a.lv[a.nlev - 1].nz;
    if (nb <= 64)
        hipLaunchKernelGGL((k_coarse_cycle<T, 1>), dim3(1), dim3(1024), 0, s, a);
    else if (nb <= 128)
        hipLaunchKernelGGL((k_coarse_cycle<T, 2>), dim3(1), dim3(1024), 0, s, a);
    else
        hipLaunchKernelGGL((k_coarse_cycle<T, 4>), dim3(1), dim3(1024), 0, s, a);
}

template void launch_coarse_cycle<float>(const CoarseArgs<float>&, hipStream_t);
template void launch_coarse_cycle<double>(const CoarseArgs<double>&, hipStream_t);
template void launch_bottom_inverse<float>(const Dims&, const float*, const float*, const float*, double*, double*,
                                           hipStream_t);
template void launch_bottom_inverse<double>(const Dims&, const double*, const double*, const double*, double*, double*,
                                            hipStream_t);
template void launch_bottom_direct<float>(const Dims&, const double*, const double*, const float*, float*, double,
                                          hipStream_t);
template void launch_bottom_direct<double>(const Dims&, const double*, const double*, const double*, double*, double,
                                           hipStream_t);

}  // namespace mp
