// k_scan1d.hip -- the one-dimensional base state by multi-block scans:
// Enforce HSE, beta0 from its definition, and w0 of the velocity split (the
// base-state modules of Sec. 3.2 and Appendix A), plus the allocation-free
// form of Enforce HSE for callers that cannot allocate device memory.
//
// Each quantity is a prefix sum over the base-state cells.  The values are cut
// into tiles of kScanTile = 4096 (one 1024-thread workgroup per tile, four
// consecutive values per thread):
//   1. every tile's total (and, for Enforce HSE, the first centre at or below
//      the cutoff density within the tile; for beta0, the count of invalid
//      inputs);
//   2. one workgroup: the exclusive prefix of the tile totals (and the
//      smallest cutoff index, or the total invalid count);
//   3. every tile again, its prefix added, each value written.
// Within a tile a thread sums its four values in order, a wavefront scans its
// threads' totals, and the wavefront totals are added in order; step 2 uses
// the same pattern over the tile totals.  The association is fixed, so the
// results are reproducible bit for bit.
#include "../../include/mproj.h"
#include "mp_base.h"
#include "mp_device.h"

#include <stdio.h>

#include <cmath>
#include <mutex>

namespace mp {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
static_assert(kScanThreads * kScanPer == kScanTile, "a tile is one workgroup's four values per thread");

// Scratch of one scan: tile totals, tile prefixes, a per-tile extra value and
// a few scalars (scal[0]: the reduced extra).
struct ScanWork {
    double* tot;
    double* off;
    double* ext;
    double* scal;
};
inline ScanWork scan_work(double* w, long long tiles) { return ScanWork{w, w + tiles, w + 2 * tiles, w + 3 * tiles}; }

enum { EXT_NONE = 0, EXT_MIN = 1, EXT_SUM = 2 };

// Prefix sums of value(j) within tile t: loc[u] holds the thread's running sum
// through its value u, `before` the tile's sum ahead of the thread's first
// value; returns the tile total (every thread).  All threads must call.
template <typename V>
__device__ double tile_scan(long long n, long long t, V value, double (&loc)[kScanPer], double& before, double* sh)
{
    const int th = threadIdx.x, lane = th & (kWave - 1), w = th / kWave;
    constexpr int nw = kScanThreads / kWave;
    const long long j0 = t * kScanTile + (long long)th * kScanPer;
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
    before = wbase + (incl - s);
    return tile;
}

// Smallest of v over the workgroup (every thread receives it).
__device__ double block_min(double v, double* sh)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double y = __shfl_xor(v, o, kWave);
        v = y < v ? y : v;
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double m = sh[0];
    for (int q = 1; q < (int)(blockDim.x / kWave); q++) m = sh[q] < m ? sh[q] : m;
    return m;
}

// Step 1: the total of each tile, and its extra value.
template <typename Op>
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(long long n, Op op, ScanWork w)
{
    __shared__ double sh[kScanThreads / kWave];
    const long long t = blockIdx.x;
    double loc[kScanPer], before;
    const double tot = tile_scan(n, t, [&](long long j) { return op.inc(j); }, loc, before, sh);
    if constexpr (Op::kExt != EXT_NONE) {
        double e = Op::kExt == EXT_MIN ? (double)n : 0.0;
        const long long j0 = t * kScanTile + (long long)threadIdx.x * kScanPer;
#pragma unroll
        for (int u = 0; u < kScanPer; u++) {
            const long long j = j0 + u;
            if (j < n) {
                const double x = op.ext(j);
                if constexpr (Op::kExt == EXT_MIN) e = x < e ? x : e;
                else e += x;
            }
        }
        e = Op::kExt == EXT_MIN ? block_min(e, sh) : block_sum(e, sh);
        if (threadIdx.x == 0) w.ext[t] = e;
    }
    if (threadIdx.x == 0) w.tot[t] = tot;
}

// Step 2 (one workgroup): off[t] = tot[0] + ... + tot[t-1]; scal[0] = the
// smallest (EXT_MIN) or the sum (EXT_SUM) of the tile extras, copied to
// ext_out when given.
__global__ __launch_bounds__(kScanThreads) void k_scan_offsets(long long tiles, ScanWork w, int ext_mode,
                                                               double* ext_out)
{
    __shared__ double sh[kScanThreads / kWave];
    for (long long t0 = 0; t0 < tiles; t0 += kScanTile) {
        double loc[kScanPer], before;
        (void)tile_scan(tiles, t0 / kScanTile, [&](long long t) { return t > 0 ? w.tot[t - 1] : 0.0; }, loc, before,
                        sh);
        // the values before this chunk: the inclusive prefix through t0 - 1
        const double carry = t0 > 0 ? w.off[t0 - 1] : 0.0;
        const long long j0 = t0 + (long long)threadIdx.x * kScanPer;
#pragma unroll
        for (int u = 0; u < kScanPer; u++)
            if (j0 + u < tiles) w.off[j0 + u] = carry + before + loc[u];
        __syncthreads();
    }
    if (ext_mode == EXT_NONE) return;
    double e = ext_mode == EXT_MIN ? 1e300 : 0.0;
    if (ext_mode == EXT_MIN) {
        for (long long t = threadIdx.x; t < tiles; t += blockDim.x) e = w.ext[t] < e ? w.ext[t] : e;
        e = block_min(e, sh);
    } else {
        for (long long t = threadIdx.x; t < tiles; t += blockDim.x) e += w.ext[t];
        e = block_sum(e, sh);
    }
    if (threadIdx.x == 0) {
        w.scal[0] = e;
        if (ext_out) ext_out[0] = e;
    }
}

// Step 3: every tile again from its prefix; values up to op.last(...) written.
template <typename Op>
__global__ __launch_bounds__(kScanThreads) void k_scan_put(long long n, Op op, ScanWork w)
{
    __shared__ double sh[kScanThreads / kWave];
    const long long t = blockIdx.x;
    const long long last = op.last(w.scal, n);
    if (t * kScanTile > last) return;  // the whole workgroup: nothing of this tile is written
    double loc[kScanPer], before;
    (void)tile_scan(n, t, [&](long long j) { return j > last ? 0.0 : op.inc(j); }, loc, before, sh);
    const double off = w.off[t];
    const long long j0 = t * kScanTile + (long long)threadIdx.x * kScanPer;
#pragma unroll
    for (int u = 0; u < kScanPer; u++) {
        const long long j = j0 + u;
        if (j < n && j <= last) op.put(j, off + before + loc[u]);
    }
    if (t == 0 && threadIdx.x == 0) op.first();
}

// Enforce HSE: p0[j] = p0_base - sum_{i=1..j, i <= jc} (rc[i] - rc[i-1]) g_edge[i]
// (rho0[i-1] + rho0[i]) / 2, jc the first centre with rho0 <= rho_cutoff.
struct HseOp {
    static constexpr int kExt = EXT_MIN;
    const double* rc;
    const double* rho0;
    const double* g;
    double p0_base, rho_cut;
    double* p0;
    __device__ double inc(long long j) const
    {
        if (j == 0) return p0_base;
        return -((rc[j] - rc[j - 1]) * g[j] * (0.5 * (rho0[j - 1] + rho0[j])));
    }
    __device__ double ext(long long j) const { return rho0[j] <= rho_cut ? (double)j : 1e300; }
    __device__ long long last(const double* scal, long long n) const
    {
        const double jc = scal[0];
        return jc < (double)n ? (long long)jc : n - 1;
    }
    __device__ void put(long long j, double v) const { p0[j] = v; }
    __device__ void first() const {}
};

// Beyond the cutoff p0 keeps its value at the cutoff, bit for bit; the index
// goes to the outputs.
__global__ __launch_bounds__(kBlock) void k_hse_hold(long long n, const double* scal, double* __restrict__ p0,
                                                     double* jc_d, long long* jc_ll)
{
    const double e = scal[0];
    const long long jc = e < (double)n ? (long long)e : n;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (jc_d) jc_d[0] = (double)jc;
        if (jc_ll) jc_ll[0] = jc;
    }
    if (jc >= n) return;
    const double pc = p0[jc];
    for (long long j = jc + 1 + blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n;
         j += (long long)gridDim.x * blockDim.x)
        p0[j] = pc;
}

// beta0[j] = rho0_centre exp(sum_{i=1..j} ln(p0[i] / p0[i-1]) / ((Gamma1[i-1] + Gamma1[i]) / 2));
// the extra counts non-positive or non-finite p0 / Gamma1 entries.
struct Beta0Op {
    static constexpr int kExt = EXT_SUM;
    const double* p0;
    const double* g1;
    double rho0c;
    double* beta0;
    __device__ double inc(long long j) const
    {
        if (j == 0) return 0.0;
        return log(p0[j] / p0[j - 1]) / (0.5 * (g1[j - 1] + g1[j]));
    }
    __device__ double ext(long long j) const
    {
        return (p0[j] > 0.0 && isfinite(p0[j]) && g1[j] > 0.0 && isfinite(g1[j])) ? 0.0 : 1.0;
    }
    __device__ long long last(const double*, long long n) const { return n - 1; }
    __device__ void put(long long j, double v) const { beta0[j] = rho0c * exp(v); }
    __device__ void first() const {}
};

// w0 on the n + 1 edges: F[e] = sum_{j<e} beta0[j] (sbar[j] - psi[j]) V[j]
// (V = re[j+1] - re[j] planar, (re[j+1]^3 - re[j]^3)/3 spherical), w0[0] = 0,
// w0[e] = F[e] / (area(e) beta0_edge(e)), beta0 on an edge linear in r
// between the neighbouring centres (extrapolated at the outer edge).
struct W0Op {
    static constexpr int kExt = EXT_NONE;
    int spherical;
    long long n;
    const double* rc;
    const double* re;
    const double* beta0;
    const double* sbar;
    const double* psi;
    double* w0;
    __device__ double inc(long long j) const
    {
        const double a = re[j], b = re[j + 1];
        const double V = spherical ? (b * b * b - a * a * a) / 3.0 : b - a;
        return beta0[j] * (sbar[j] - (psi ? psi[j] : 0.0)) * V;
    }
    __device__ double ext(long long) const { return 0.0; }
    __device__ long long last(const double*, long long nn) const { return nn - 1; }
    __device__ void put(long long j, double F) const
    {
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
    }
    __device__ void first() const { w0[0] = 0.0; }
};

// Offsets of buckets from their counts: offs[j + 1] = the inclusive sum.
struct OffsetsOp {
    static constexpr int kExt = EXT_NONE;
    const double* cnt;
    long long* offs;
    __device__ double inc(long long j) const { return cnt[j]; }
    __device__ double ext(long long) const { return 0.0; }
    __device__ long long last(const double*, long long n) const { return n - 1; }
    __device__ void put(long long j, double v) const { offs[j + 1] = (long long)v; }
    __device__ void first() const { offs[0] = 0; }
};

template <typename Op>
void run_scan(long long n, const Op& op, double* work, double* ext_out, hipStream_t s)
{
    const long long tiles = scan_tiles(n);
    const ScanWork w = scan_work(work, tiles);
    hipLaunchKernelGGL((k_scan_tiles<Op>), dim3((unsigned)tiles), dim3(kScanThreads), 0, s, n, op, w);
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(kScanThreads), 0, s, tiles, w, (int)Op::kExt, ext_out);
    hipLaunchKernelGGL((k_scan_put<Op>), dim3((unsigned)tiles), dim3(kScanThreads), 0, s, n, op, w);
}

}  // namespace

void launch_enforce_hse(long long n, const double* rc, const double* rho0, const double* g_edge, double p0_base,
                        double rho_cutoff, double* p0, double* work, double* jc_d, long long* jc_ll, hipStream_t s)
{
    const HseOp op{rc, rho0, g_edge, p0_base, rho_cutoff, p0};
    run_scan(n, op, work, nullptr, s);
    const ScanWork w = scan_work(work, scan_tiles(n));
    long long nb = (n + kBlock - 1) / kBlock;
    nb = nb < 1 ? 1 : nb > 1024 ? 1024 : nb;
    hipLaunchKernelGGL(k_hse_hold, dim3((unsigned)nb), dim3(kBlock), 0, s, n, (const double*)w.scal, p0, jc_d, jc_ll);
}

void launch_beta0_from_p0(long long n, double rho0_centre, const double* p0, const double* gamma1, double* beta0,
                          double* work, double* bad, hipStream_t s)
{
    const Beta0Op op{p0, gamma1, rho0_centre, beta0};
    run_scan(n, op, work, bad, s);
}

void launch_w0(int spherical, long long n, const double* rc, const double* re, const double* beta0, const double* sbar,
               const double* psi, double* w0, double* work, hipStream_t s)
{
    const W0Op op{spherical, n, rc, re, beta0, sbar, psi, w0};
    run_scan(n, op, work, nullptr, s);
}

void launch_offsets_of_counts(long long nm, const double* cnt, long long* offs, double* work, hipStream_t s)
{
    const OffsetsOp op{cnt, offs};
    run_scan(nm, op, work, nullptr, s);
}

// ---------------------------------------------------------------------------
// Allocation-free Enforce HSE.  The scan's scratch lives in `scratch`, one
// copy per device for the life of the process, sized for kNoAllocMaxRadii
// centres.  Host code never uses the array's name as a device address: the
// address comes from hipGetSymbolAddress, once per device, with that device
// current.

constexpr long long kNoAllocMaxRadii = 1LL << 24;  // 4096 tiles
constexpr long long kScratchDoubles = 3 * ((kNoAllocMaxRadii + kScanTile - 1) / kScanTile) + 8;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
hipError_t scratch_for(int dev, double** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

thread_local char g_noalloc_err[256] = "";

int na_fail(int code, const char* msg)
{
    snprintf(g_noalloc_err, sizeof g_noalloc_err, "%s", msg);
    return code;
}

}  // namespace

const char* noalloc_last_error() { return g_noalloc_err; }

}  // namespace mp

extern "C" int mp_enforce_hse_noalloc(void* stream, long long n, const double* rc, const double* rho0,
                                      const double* g_edge, double p0_base, double rho_cutoff, double* p0,
                                      long long* cutoff_index)
{
    using namespace mp;
    if (n < 1 || !rc || !rho0 || !g_edge || !p0)
        return na_fail(MP_ERR_ARG, "mp_enforce_hse_noalloc: n >= 1, rc, rho0, g_edge and p0 are required");
    if (n > kNoAllocMaxRadii)
        return na_fail(MP_ERR_ARG, "mp_enforce_hse_noalloc: n exceeds the static scratch (at most 16777216 centres)");
    if (!std::isfinite(p0_base) || std::isnan(rho_cutoff))
        return na_fail(MP_ERR_ARG, "mp_enforce_hse_noalloc: p0_base must be finite");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return na_fail(MP_ERR_DEVICE, "mp_enforce_hse_noalloc: no current HIP device");
    double* work = nullptr;
    if (scratch_for(dev, &work) != hipSuccess) {
        (void)hipGetLastError();
        return na_fail(MP_ERR_DEVICE, "mp_enforce_hse_noalloc: hipGetSymbolAddress of the scratch array failed");
    }
    launch_enforce_hse(n, rc, rho0, g_edge, p0_base, rho_cutoff, p0, work, nullptr, cutoff_index,
                       (hipStream_t)stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return na_fail(MP_ERR_DEVICE, hipGetErrorString(e));
    g_noalloc_err[0] = '\0';
    return MP_OK;
}
