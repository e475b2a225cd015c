// k_base.hip -- lateral Average over the irregular radial base state.
//
// Sec. 3.1: with the star centre on a grid node, every cell centre lies at a
// radius h sqrt(0.75 + 2m) for an integer m, and the lateral average of a
// cell field at radius m is the sum over those cells divided by their count
// (the Average module of Sec. 3.2; its global sum is the paper's scaling
// bottleneck).  On one GPU the sum is a segmented reduction: the cells are
// listed once per grid, grouped by m in memory order (a counting sort done
// on the host when the context first needs it), and one wavefront reduces
// one radius in a fixed order, so the result is deterministic.
#include "mp_device.h"
#include "mp_kernels.h"

namespace mp {

// One wavefront per radius: lanes take every 64th listed cell, then a fixed
// butterfly sum.  avg[m] = sum / count (0 for radii no cell reaches).
__global__ __launch_bounds__(kBlock) void k_average(long long nm, const long long* __restrict__ offs,
                                                    const unsigned* __restrict__ cells,
                                                    const double* __restrict__ phi, double* __restrict__ avg,
                                                    double* __restrict__ count)
{
    const long long m = (long long)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (m >= nm) return;  // whole wavefronts leave together
    const int lane = threadIdx.x & (kWave - 1);
    const long long a = offs[m], e = offs[m + 1];
    double s = 0.0;
    for (long long p = a + lane; p < e; p += kWave) s += phi[cells[p]];
    s = wave_sum_bcast(s);
    if (lane == 0) {
        const long long n = e - a;
        avg[m] = n > 0 ? s / (double)n : 0.0;
        if (count) count[m] = (double)n;
    }
}

void launch_average(long long nm, const long long* offs, const unsigned* cells, const double* phi, double* avg,
                    double* count, hipStream_t s)
{
    const long long per = kBlock / kWave;
    const long long nb = (nm + per - 1) / per;
    hipLaunchKernelGGL(k_average, dim3((unsigned)nb), dim3(kBlock), 0, s, nm, offs, cells, phi, avg, count);
}

}  // namespace mp

// ------------------------------------------------------- 1D base state

namespace mp {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;  // consecutive elements per thread and tile

// Inclusive prefix sums of value(j), j = 0 .. n-1, by one workgroup of
// kScanThreads threads, in a fixed association (tiles of kScanThreads *
// kScanPer elements: sequential within a thread, then a wavefront scan, then
// the wavefront totals, then the running total of the previous tiles).
// out(j, prefix) receives each sum.  Every thread must call it.
template <typename V, typename O>
__device__ void block_scan(long long n, V value, O out, double* sh)
{
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const int nw = kScanThreads / kWave;
    double carry = 0.0;
    for (long long base = 0; base < n; base += (long long)kScanThreads * kScanPer) {
        const long long j0 = base + (long long)t * kScanPer;
        double loc[kScanPer];
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < kScanPer; u++) {
            const long long j = j0 + u;
            s += j < n ? value(j) : 0.0;
            loc[u] = s;
        }
        // inclusive scan of the thread totals within the wavefront
        double incl = s;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const double y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
        }
        __syncthreads();
        if (lane == kWave - 1) sh[w] = incl;
        __syncthreads();
        double wbase = 0.0, tile = 0.0;
        for (int q = 0; q < nw; q++) {
            if (q < w) wbase += sh[q];
            tile += sh[q];
        }
        const double before = carry + wbase + (incl - s);
#pragma unroll
        for (int u = 0; u < kScanPer; u++) {
            const long long j = j0 + u;
            if (j < n) out(j, before + loc[u]);
        }
        carry += tile;
    }
}

}  // namespace

// Centres h sqrt(0.75 + 2m) and edges h sqrt(2m - 1/4) (edge 0 at the centre)
// of the irregular base state.
__global__ __launch_bounds__(kBlock) void k_irregular_radii(long long nm, double h, double* __restrict__ rc,
                                                            double* __restrict__ re)
{
    for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m <= nm;
         m += (long long)gridDim.x * blockDim.x) {
        if (m < nm) rc[m] = h * sqrt(0.75 + 2.0 * (double)m);
        re[m] = m == 0 ? 0.0 : h * sqrt(2.0 * (double)m - 0.25);
    }
}

void launch_irregular_radii(long long nm, double h, double* rc, double* re, hipStream_t s)
{
    long long nb = (nm + kBlock) / kBlock;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_irregular_radii, dim3((unsigned)nb), dim3(kBlock), 0, s, nm, h, rc, re);
}

// Enforce HSE: p0[j] = p0_base - sum_{i=1..j, i <= jc} (rc[i] - rc[i-1]) g_edge[i]
// (rho0[i-1] + rho0[i]) / 2, jc the first centre with rho0 <= rho_cutoff.
// jc_out[0] = jc (as a double).
__global__ __launch_bounds__(kScanThreads) void k_enforce_hse(long long n, const double* __restrict__ rc,
                                                              const double* __restrict__ rho0,
                                                              const double* __restrict__ g_edge, double p0_base,
                                                              double rho_cutoff, double* __restrict__ p0,
                                                              double* jc_out)
{
    __shared__ double sh[kScanThreads / kWave];
    __shared__ long long shm[kScanThreads / kWave];
    long long jm = n;
    for (long long j = threadIdx.x; j < n; j += blockDim.x)
        if (rho0[j] <= rho_cutoff && j < jm) jm = j;
    // block minimum
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const long long y = __shfl_xor(jm, o, kWave);
        jm = y < jm ? y : jm;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) shm[threadIdx.x / kWave] = jm;
    __syncthreads();
    long long jc = n;
    for (int q = 0; q < kScanThreads / kWave; q++) jc = shm[q] < jc ? shm[q] : jc;
    if (threadIdx.x == 0) jc_out[0] = (double)jc;
    auto inc = [&](long long j) -> double {
        if (j == 0) return p0_base;
        if (j > jc) return 0.0;
        return -((rc[j] - rc[j - 1]) * g_edge[j] * (0.5 * (rho0[j - 1] + rho0[j])));
    };
    auto put = [&](long long j, double v) {
        if (j <= jc) p0[j] = v;
    };
    block_scan(n, inc, put, sh);
    // beyond the cutoff p0 is the value at the cutoff itself, bit for bit
    __syncthreads();
    if (jc < n) {
        const double pc = p0[jc];
        for (long long j = jc + 1 + threadIdx.x; j < n; j += blockDim.x) p0[j] = pc;
    }
}

void launch_enforce_hse(long long n, const double* rc, const double* rho0, const double* g_edge, double p0_base,
                        double rho_cutoff, double* p0, double* jc_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_enforce_hse, dim3(1), dim3(kScanThreads), 0, s, n, rc, rho0, g_edge, p0_base, rho_cutoff,
                       p0, jc_out);
}

// beta0[j] = rho0_centre exp(sum_{i=1..j} ln(p0[i] / p0[i-1]) / ((Gamma1[i-1] + Gamma1[i]) / 2));
// bad[0] = number of non-positive or non-finite p0 / Gamma1 entries.
__global__ __launch_bounds__(kScanThreads) void k_beta0_from_p0(long long n, double rho0_centre,
                                                                const double* __restrict__ p0,
                                                                const double* __restrict__ gamma1,
                                                                double* __restrict__ beta0, double* bad)
{
    __shared__ double sh[kScanThreads / kWave];
    double nbad = 0.0;
    for (long long j = threadIdx.x; j < n; j += blockDim.x)
        nbad += (p0[j] > 0.0 && isfinite(p0[j]) && gamma1[j] > 0.0 && isfinite(gamma1[j])) ? 0.0 : 1.0;
    nbad = block_sum(nbad, sh);
    if (threadIdx.x == 0) bad[0] = nbad;
    auto inc = [&](long long j) -> double {
        if (j == 0) return 0.0;
        return log(p0[j] / p0[j - 1]) / (0.5 * (gamma1[j - 1] + gamma1[j]));
    };
    auto put = [&](long long j, double v) { beta0[j] = rho0_centre * exp(v); };
    block_scan(n, inc, put, sh);
}

void launch_beta0_from_p0(long long n, double rho0_centre, const double* p0, const double* gamma1, double* beta0,
                          double* bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_beta0_from_p0, dim3(1), dim3(kScanThreads), 0, s, n, rho0_centre, p0, gamma1, beta0, bad);
}

// w0 on the n + 1 edges: F[e] = sum_{j<e} beta0[j] (sbar[j] - psi[j]) V[j]
// (V = re[j+1] - re[j] planar, (re[j+1]^3 - re[j]^3)/3 spherical), w0[0] = 0,
// w0[e] = F[e] / (area(e) beta0_edge(e)), beta0 on an edge linear in r
// between the neighbouring centres (extrapolated at the outer edge).
__global__ __launch_bounds__(kScanThreads) void k_w0(int spherical, long long n, const double* __restrict__ rc,
                                                     const double* __restrict__ re,
                                                     const double* __restrict__ beta0,
                                                     const double* __restrict__ sbar,
                                                     const double* __restrict__ psi, double* __restrict__ w0)
{
    __shared__ double sh[kScanThreads / kWave];
    if (threadIdx.x == 0) w0[0] = 0.0;
    auto inc = [&](long long j) -> double {
        const double a = re[j], b = re[j + 1];
        const double V = spherical ? (b * b * b - a * a * a) / 3.0 : b - a;
        return beta0[j] * (sbar[j] - (psi ? psi[j] : 0.0)) * V;
    };
    auto put = [&](long long j, double F) {
        const long long e = j + 1;
        double be;
        if (n == 1) {
            be = beta0[0];
        } else {
            const long long a = e < n ? e - 1 : n - 2, b = a + 1;
            const double t = (re[e] - rc[a]) / (rc[b] - rc[a]);
            be = beta0[a] + t * (beta0[b] - beta0[a]);
        }
        const double area = spherical ? re[e] * re[e] : 1.0;
        w0[e] = F / (area * be);
    };
    block_scan(n, inc, put, sh);
}

void launch_w0(int spherical, long long n, const double* rc, const double* re, const double* beta0, const double* sbar,
               const double* psi, double* w0, hipStream_t s)
{
    hipLaunchKernelGGL(k_w0, dim3(1), dim3(kScanThreads), 0, s, spherical, n, rc, re, beta0, sbar, psi, w0);
}

}  // namespace mp
