// k_coarse.hip -- the coarse end of a V-cycle in one workgroup.
//
// On the smallest levels (a few hundred cells) a kernel finishes in well under
// the cost of a launch, so a V-cycle would spend its coarse-grid time in launch
// gaps.
// This kernel runs every level of the coarse set (pre-smoothing, residual
// restriction, bottom solve, prolongation, post-smoothing) in a single
// 1024-thread workgroup, separated by workgroup barriers.  The per-cell
// arithmetic is the shared code of the one-launch-per-operation kernels, so
// the smoother and the transfers agree with them bit for bit.
//
// The bottom solve is BiCGStab in FP64 run by the first wavefront alone: each
// lane holds up to NS cells in registers, neighbour values come from
// cross-lane shuffles and dot products from wavefront reductions broadcast
// from lane 0, so no barrier is needed inside the iteration.
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

template <typename T, int NS>
__device__ void wave_bicgstab(const Dims& d, const T* __restrict__ bin, T* __restrict__ xout,
                              const T* __restrict__ cx, const T* __restrict__ cy, const T* __restrict__ cz, double h2,
                              double rtol, int maxit)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int n = (int)d.n();
    const double inv_h2 = 1.0 / h2;
    // per-slot cell data: coefficients and neighbour indices
    double c[NS][6];
    int nbi[NS][6];
    bool live[NS];
    double b[NS], x[NS], r[NS], rh[NS], p[NS], v[NS], s[NS], t[NS];
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
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < NS; u++) part += b[u];
    const double mean = wave_sum_bcast(part) / n;
#pragma unroll
    for (int u = 0; u < NS; u++) {
        b[u] = live[u] ? b[u] - mean : 0.0;
        x[u] = 0.0;
        r[u] = b[u];
        rh[u] = b[u];
        p[u] = 0.0;
        v[u] = 0.0;
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
    const double bnorm2 = dot(b, b);
    const double tol2 = rtol * rtol * bnorm2;
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    if (bnorm2 > 0.0) {
        for (int it = 0; it < maxit; it++) {
            const double rho1 = dot(rh, r);
            if (rho1 == 0.0) break;
            const double beta = (rho1 / rho) * (alpha / omega);
#pragma unroll
            for (int u = 0; u < NS; u++) p[u] = r[u] + beta * (p[u] - omega * v[u]);
            apply(p, v);
            const double rhv = dot(rh, v);
            if (rhv == 0.0) break;
            alpha = rho1 / rhv;
#pragma unroll
            for (int u = 0; u < NS; u++) s[u] = r[u] - alpha * v[u];
            const double ss = dot(s, s);
            if (ss <= tol2) {
#pragma unroll
                for (int u = 0; u < NS; u++) x[u] += alpha * p[u];
                break;
            }
            apply(s, t);
            const double ts = dot(t, s);
            const double tt = dot(t, t);
            if (tt == 0.0) {
#pragma unroll
                for (int u = 0; u < NS; u++) x[u] += alpha * p[u];
                break;
            }
            omega = ts / tt;
#pragma unroll
            for (int u = 0; u < NS; u++) {
                x[u] += alpha * p[u] + omega * s[u];
                r[u] = s[u] - omega * t[u];
            }
            const double rr = dot(r, r);
            rho = rho1;
            if (rr <= tol2 || omega == 0.0) break;
        }
    }
    part = 0.0;
#pragma unroll
    for (int u = 0; u < NS; u++) part += live[u] ? x[u] : 0.0;
    const double xm = wave_sum_bcast(part) / n;
#pragma unroll
    for (int u = 0; u < NS; u++)
        if (live[u]) xout[lane + kWave * u] = (T)(x[u] - xm);
}

template <typename T>
__device__ void cg_smooth(const CoarseLevel<T>& L, const Dims& d, int zero_init)
{
    const int nxh = (d.nx + 1) / 2;
    const int cnt = nxh * d.ny * d.nz;
    for (int colour = 0; colour < 2; colour++) {
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
            const int p = e % nxh, t = e / nxh, j = t % d.ny, k = t / d.ny;
            rbgs_cell<T, false>(d, L.x, L.b, Coef<T>{L.cx, L.cy, L.cz, nullptr}, L.h2, colour,
                                zero_init && colour == 0, p, j, k);
        }
        __syncthreads();
    }
}

template <typename T, int NS>
__global__ __launch_bounds__(1024) void k_coarse_cycle(CoarseArgs<T> a)
{
    const int nl = a.nlev;
    Dims dims[kMaxCoarse];
    for (int l = 0; l < nl; l++) dims[l] = Dims{a.lv[l].nx, a.lv[l].ny, a.lv[l].nz, a.px, a.py, a.pz};
    // down
    for (int l = 0; l < nl - 1; l++) {
        const CoarseLevel<T>& L = a.lv[l];
        const int zi = (l > 0) || a.zero_init;
        if (zi && a.nu1 == 0) {
            const int cnt0 = dims[l].nx * dims[l].ny * dims[l].nz;
            for (int e = threadIdx.x; e < cnt0; e += blockDim.x) L.x[e] = T(0);
            __syncthreads();
        }
        for (int s = 0; s < a.nu1; s++) cg_smooth<T>(L, dims[l], zi && s == 0);
        const Dims& f = dims[l];
        const int nxc = f.nx / 2, nyc = f.ny / 2, nzc = f.nz / 2;
        const int cnt = nxc * nyc * nzc;
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
            const int I = e % nxc, t = e / nxc, J = t % nyc, K = t / nyc;
            a.lv[l + 1].b[e] = restrict_cell<T, false>(f, L.x, L.b, Coef<T>{L.cx, L.cy, L.cz, nullptr}, L.inv_h2, I, J,
                                                       K);
        }
        __syncthreads();
    }
    // bottom: first wavefront only; the others wait at the barrier below
    if (threadIdx.x < kWave) {
        const CoarseLevel<T>& B = a.lv[nl - 1];
        wave_bicgstab<T, NS>(dims[nl - 1], B.b, B.x, B.cx, B.cy, B.cz, B.h2d, a.bottom_rtol, a.bottom_maxit);
    }
    __syncthreads();
    // up
    for (int l = nl - 2; l >= 0; l--) {
        const CoarseLevel<T>& L = a.lv[l];
        const Dims& f = dims[l];
        const int nxc = f.nx / 2, nyc = f.ny / 2;
        const int cnt = f.nx * f.ny * f.nz;
        const T* ec = a.lv[l + 1].x;
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
            const int i = e % f.nx, t = e / f.nx, j = t % f.ny, k = t / f.ny;
            L.x[e] += ec[((k >> 1) * nyc + (j >> 1)) * nxc + (i >> 1)];
        }
        __syncthreads();
        for (int s = 0; s < a.nu2; s++) cg_smooth<T>(L, f, 0);
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

}  // namespace mp
