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
#include "mp_base.h"
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

}  // namespace mp
