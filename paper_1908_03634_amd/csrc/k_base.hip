// k_base.hip -- lateral Average over the radial base state, and w0 on faces.
//
// Sec. 3.1: with the star centre on the grid node in the middle of the box,
// the centre of cell (i,j,k) lies at h sqrt(0.75 + 2m) with
//     m = (a^2 + b^2 + c^2 - 3) / 8,  a = 2i + 1 - nx, b = 2j + 1 - ny, c = 2k + 1 - nz,
// and the lateral average of a cell field at radius m is the sum over those
// cells divided by their count (the Average module of Sec. 3.2).  The offsets
// a, b, c are odd, so every cell has seven mirror images (a, b, c with
// independent signs) at the same radius, one in each octant of the box:
//   - fold: the eight mirror cells of each cell of the high octant summed in a
//     fixed order (one streaming pass over the field);
//   - list: the octant cells grouped by radius, in memory order within a
//     radius (built on the device once per context, below);
//   - average: one wavefront per radius sums the folded values of its octant
//     cells in a fixed order and divides by eight times their number.
// The onto-a-uniform-grid form (the base state of spacing dr used before the
// irregular one) interpolates the radius averages quadratically.
//
// The list is a stable counting sort by radius.  Within an octant plane
// (fixed c) a row (fixed b) holds each radius at most once (m grows with a),
// so walking the rows of a plane in order, one workgroup per plane, gives
// every cell its rank among the cells of its radius in that plane without
// conflicts; a radius's planes are then prefixed in plane order, the radius
// counts scanned, and every cell written to offs[m] + (its plane's prefix) +
// (its rank in the plane).
#include "mp_base.h"
#include "mp_device.h"
#include "mp_kernels.h"

namespace mp {

namespace {

// Octant geometry: octant cell (a', b', c') (a' < nx/2 ...) is the cell with
// offsets a = 2a' + 1, b = 2b' + 1, c = 2c' + 1, i.e. i = nx/2 + a'.
struct Oct {
    int hx, hy, hz;  // half extents
    __host__ __device__ long long n() const { return (long long)hx * hy * hz; }
};

__device__ __forceinline__ long long oct_m(long long a, long long b, long long c)
{
    return ((2 * a + 1) * (2 * a + 1) + (2 * b + 1) * (2 * b + 1) + (2 * c + 1) * (2 * c + 1) - 3) / 8;
}

// Smallest radius index of octant plane c' (its cell a' = b' = 0), and the
// width of every plane's window of radius indices.
__device__ __forceinline__ long long plane_mlo(long long c) { return oct_m(0, 0, c); }

}  // namespace

// Width of every octant plane's window of radius indices (the radii of its
// cells a' = b' = 0 through a' = nx/2 - 1, b' = ny/2 - 1; the difference does
// not depend on the plane).
long long oct_window(int nx, int ny)
{
    const long long a = nx - 1, b = ny - 1;
    return (a * a - 1 + b * b - 1) / 8 + 1;
}

// Rank of every octant cell among the cells of its radius in its plane, and
// the plane's count per radius (cnt: hz x win ints, zero on entry).  One
// workgroup per plane walks its rows in order.
__global__ __launch_bounds__(kBlock) void k_oct_rank(Oct o, long long win, unsigned* __restrict__ cnt,
                                                     unsigned* __restrict__ rank)
{
    const long long c = blockIdx.x;
    const long long mlo = plane_mlo(c);
    unsigned* pc = cnt + c * win;
    for (int b = 0; b < o.hy; b++) {
        for (int a = threadIdx.x; a < o.hx; a += blockDim.x) {
            const long long w = oct_m(a, b, c) - mlo;
            // one cell per counter within a row: the old value is the rank
            rank[(c * o.hy + b) * o.hx + a] = atomicAdd(pc + w, 1u);
        }
        __syncthreads();  // the next row may hold the radii of this one
    }
}

// For each radius: the planes' counts replaced by their exclusive prefix in
// plane order; cntm[m] = the number of octant cells at radius m.
__global__ __launch_bounds__(kBlock) void k_oct_radius_prefix(Oct o, long long win, long long nm,
                                                              unsigned* __restrict__ cnt, double* __restrict__ cntm)
{
    const long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (m >= nm) return;
    unsigned off = 0;
    for (long long c = 0; c < o.hz; c++) {
        const long long w = m - plane_mlo(c);
        if (w < 0) break;  // the windows move outward with c
        if (w >= win) continue;
        unsigned* p = cnt + c * win + w;
        const unsigned v = *p;
        *p = off;
        off += v;
    }
    cntm[m] = (double)off;
}

// list[offs[m] + plane prefix + rank] = octant cell index.
__global__ __launch_bounds__(kBlock) void k_oct_scatter(Oct o, long long win, const unsigned* __restrict__ cnt,
                                                        const unsigned* __restrict__ rank,
                                                        const long long* __restrict__ offs,
                                                        unsigned* __restrict__ list)
{
    const long long n = o.n();
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const long long a = q % o.hx, t = q / o.hx, b = t % o.hy, c = t / o.hy;
        const long long m = oct_m(a, b, c);
        list[offs[m] + cnt[c * win + (m - plane_mlo(c))] + rank[q]] = (unsigned)q;
    }
}

// fold[q] = the eight mirror cells of octant cell q, summed in a fixed order
// (low x before high x, then y, then z).
__global__ __launch_bounds__(kBlock) void k_oct_fold(Dims d, Oct o, const double* __restrict__ phi,
                                                     double* __restrict__ fold)
{
    const long long n = o.n();
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(q % o.hx);
        const long long t = q / o.hx;
        const int b = (int)(t % o.hy), c = (int)(t / o.hy);
        const long long il = o.hx - 1 - a, ih = o.hx + a;
        const long long jl = o.hy - 1 - b, jh = o.hy + b;
        const long long kl = o.hz - 1 - c, kh = o.hz + c;
        const long long sy = d.nx, sz = (long long)d.nx * d.ny;
        double s = 0.0;
        s += phi[kl * sz + jl * sy + il];
        s += phi[kl * sz + jl * sy + ih];
        s += phi[kl * sz + jh * sy + il];
        s += phi[kl * sz + jh * sy + ih];
        s += phi[kh * sz + jl * sy + il];
        s += phi[kh * sz + jl * sy + ih];
        s += phi[kh * sz + jh * sy + il];
        s += phi[kh * sz + jh * sy + ih];
        fold[q] = s;
    }
}

// One wavefront per radius: lanes take every 64th listed octant cell, then a
// fixed butterfly sum.  avg[m] = sum / (8 count) (0 for radii no cell
// reaches); count[m] = 8 x the octant cells.
__global__ __launch_bounds__(kBlock) void k_average(long long nm, const long long* __restrict__ offs,
                                                    const unsigned* __restrict__ list,
                                                    const double* __restrict__ fold, double* __restrict__ avg,
                                                    double* __restrict__ count)
{
    const long long m = (long long)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (m >= nm) return;  // whole wavefronts leave together
    const int lane = threadIdx.x & (kWave - 1);
    const long long a = offs[m], e = offs[m + 1];
    double s = 0.0;
    for (long long p = a + lane; p < e; p += kWave) s += fold[list[p]];
    s = wave_sum_bcast(s);
    if (lane == 0) {
        const double n = 8.0 * (double)(e - a);
        avg[m] = n > 0 ? s / n : 0.0;
        if (count) count[m] = n;
    }
}

// ------------------------------------------------- onto a uniform base state

namespace {

__device__ __forceinline__ double rhat(double h, long long m) { return h * sqrt(0.75 + 2.0 * (double)m); }

// Lagrange polynomial through (x[q], y[q]), q < np, at r (the oracle's order
// of operations is not required; this is the plain product form).
__device__ __forceinline__ double lagrange3(const double (&x)[3], const double (&y)[3], int np, double r)
{
    double v = 0.0;
    for (int q = 0; q < np; q++) {
        double w = 1.0;
        for (int s = 0; s < np; s++)
            if (s != q) w *= (r - x[s]) / (x[q] - x[s]);
        v += w * y[q];
    }
    return v;
}

}  // namespace

// avg_u[j], r_j = (j + 1/2) dr: the parabola through the reached radius
// nearest r_j and the reached radii on either side of it (shifted inward at
// the first and last reached radius, which are m = 0 and m = nm - 1: the
// cells next to the centre and the corner cells), the end averages held
// outside them.  A radius is reached when its count is positive.
__global__ __launch_bounds__(kBlock) void k_average_uniform(long long nm, double h, const double* __restrict__ avg,
                                                            const long long* __restrict__ offs, int n1d, double dr,
                                                            double* __restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n1d) return;
    const double r = (j + 0.5) * dr;
    auto reached = [&](long long m) { return offs[m + 1] > offs[m]; };
    if (r <= rhat(h, 0)) {
        out[j] = avg[0];
        return;
    }
    if (r >= rhat(h, nm - 1)) {
        out[j] = avg[nm - 1];
        return;
    }
    // the radius interval [rhat(m0), rhat(m0 + 1)) holding r
    const double s = r / h;
    long long m0 = (long long)floor((s * s - 0.75) * 0.5);
    m0 = m0 < 0 ? 0 : m0 > nm - 2 ? nm - 2 : m0;
    while (m0 + 1 < nm - 1 && rhat(h, m0 + 1) <= r) m0++;
    while (m0 > 0 && rhat(h, m0) > r) m0--;
    long long lo = m0, hi = m0 + 1;
    while (!reached(lo)) lo--;
    while (!reached(hi)) hi++;
    const long long q = (r - rhat(h, lo) <= rhat(h, hi) - r) ? lo : hi;
    // nm < 3: every radius is reached and there are nm of them
    const int np = nm < 3 ? (int)nm : 3;
    long long pts[3];
    if (np == 3) {
        long long pm = q - 1, pp = q + 1;
        if (q == 0) {
            pm = q;
            while (!reached(pp)) pp++;
            long long p2 = pp + 1;
            while (!reached(p2)) p2++;
            pts[0] = pm, pts[1] = pp, pts[2] = p2;
        } else if (q == nm - 1) {
            while (!reached(pm)) pm--;
            long long p2 = pm - 1;
            while (!reached(p2)) p2--;
            pts[0] = p2, pts[1] = pm, pts[2] = q;
        } else {
            while (!reached(pm)) pm--;
            while (!reached(pp)) pp++;
            pts[0] = pm, pts[1] = q, pts[2] = pp;
        }
    } else {
        for (int t = 0; t < np; t++) pts[t] = t;
    }
    double x[3] = {0.0, 0.0, 0.0}, y[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < np; t++) {
        x[t] = rhat(h, pts[t]);
        y[t] = avg[pts[t]];
    }
    out[j] = lagrange3(x, y, np, r);
}

// ------------------------------------------------------------ w0 on faces

namespace {

// w0 at radius r, linear between the edges re[0..ne) (sorted), the end
// values held outside them.
__device__ __forceinline__ double w0_at(const double* __restrict__ w0, const double* __restrict__ re, long long ne,
                                        double r)
{
    if (r >= re[ne - 1]) return w0[ne - 1];
    if (r <= re[0]) return w0[0];
    long long lo = 0, hi = ne - 1;  // re[lo] <= r < re[hi]
    while (hi - lo > 1) {
        const long long mid = (lo + hi) / 2;
        if (re[mid] <= r) lo = mid;
        else hi = mid;
    }
    const double t = (r - re[lo]) / (re[hi] - re[lo]);
    return w0[lo] + t * (w0[hi] - w0[lo]);
}

}  // namespace

// Planar: z face k (1 <= k < nz, the low face of cell k) gains w0[k].
__global__ __launch_bounds__(kBlock) void k_w0_planar(Dims d, const double* __restrict__ w0, double* __restrict__ uz)
{
    const long long per = (long long)d.nx * d.ny;
    const long long n = (long long)(d.nz - 1) * per;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const long long k = q / per + 1;
        uz[k * per + q % per] += w0[k];
    }
}

// Spherical: each non-wall face of the axis `axis` (0 x, 1 y, 2 z; face
// layout of the external arrays: b = 1 extra face on a Neumann axis) gains
// w0(r_f) (x_f - centre)_axis / r_f.
__global__ __launch_bounds__(kBlock) void k_w0_sphere(Dims d, int axis, double h, double c0, double c1, double c2,
                                                      const double* __restrict__ w0, const double* __restrict__ re,
                                                      long long ne, double* __restrict__ u)
{
    const int bx = axis == 0 && !d.px, by = axis == 1 && !d.py, bz = axis == 2 && !d.pz;
    const long long fx = d.nx + bx, fy = d.ny + by, fz = d.nz + bz;
    const long long n = fx * fy * fz;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const long long i = q % fx, t = q / fx, j = t % fy, k = t / fy;
        if ((bx && (i == 0 || i == d.nx)) || (by && (j == 0 || j == d.ny)) || (bz && (k == 0 || k == d.nz)))
            continue;  // walls keep their values
        const double x = (axis == 0 ? (double)i : i + 0.5) * h - c0;
        const double y = (axis == 1 ? (double)j : j + 0.5) * h - c1;
        const double z = (axis == 2 ? (double)k : k + 0.5) * h - c2;
        const double r = sqrt(x * x + y * y + z * z);
        if (r > 0.0) {
            const double comp = axis == 0 ? x : axis == 1 ? y : z;
            u[q] += w0_at(w0, re, ne, r) * (comp / r);
        }
    }
}

// ------------------------------------------------------------- launchers

namespace {

unsigned grid_for(long long n)
{
    long long nb = (n + kBlock - 1) / kBlock;
    return (unsigned)(nb < 1 ? 1 : nb > 8192 ? 8192 : nb);
}

}  // namespace

long long oct_count_bytes(int nx, int ny, int nz) { return (long long)(nz / 2) * oct_window(nx, ny) * 4; }

void launch_radius_list(int nx, int ny, int nz, long long nm, unsigned* cnt, unsigned* rank, double* cntm,
                        long long* offs, unsigned* list, double* scan_work, hipStream_t s)
{
    const Oct o{nx / 2, ny / 2, nz / 2};
    const long long win = oct_window(nx, ny);
    (void)hipMemsetAsync(cnt, 0, (size_t)oct_count_bytes(nx, ny, nz), s);
    hipLaunchKernelGGL(k_oct_rank, dim3((unsigned)o.hz), dim3(kBlock), 0, s, o, win, cnt, rank);
    hipLaunchKernelGGL(k_oct_radius_prefix, dim3((unsigned)((nm + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, o, win,
                       nm, cnt, cntm);
    launch_offsets_of_counts(nm, cntm, offs, scan_work, s);
    hipLaunchKernelGGL(k_oct_scatter, dim3(grid_for(o.n())), dim3(kBlock), 0, s, o, win, (const unsigned*)cnt,
                       (const unsigned*)rank, (const long long*)offs, list);
}

void launch_average(const Dims& d, long long nm, const long long* offs, const unsigned* list, const double* phi,
                    double* fold, double* avg, double* count, hipStream_t s)
{
    const Oct o{d.nx / 2, d.ny / 2, d.nz / 2};
    hipLaunchKernelGGL(k_oct_fold, dim3(grid_for(o.n())), dim3(kBlock), 0, s, d, o, phi, fold);
    const long long per = kBlock / kWave;
    const long long nb = (nm + per - 1) / per;
    hipLaunchKernelGGL(k_average, dim3((unsigned)nb), dim3(kBlock), 0, s, nm, offs, list, (const double*)fold, avg,
                       count);
}

void launch_average_uniform(long long nm, double h, const double* avg, const long long* offs, int n1d, double dr,
                            double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_average_uniform, dim3((unsigned)((n1d + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, nm, h,
                       avg, offs, n1d, dr, out);
}

void launch_w0_faces(const Dims& d, int planar, double h, const double* center, const double* w0, const double* re,
                     long long ne, double* ux, double* uy, double* uz, hipStream_t s)
{
    if (planar) {
        const long long n = (long long)(d.nz - 1) * d.nx * d.ny;
        if (n > 0) hipLaunchKernelGGL(k_w0_planar, dim3(grid_for(n)), dim3(kBlock), 0, s, d, w0, uz);
        return;
    }
    double* us[3] = {ux, uy, uz};
    for (int a = 0; a < 3; a++) {
        const long long n = (long long)(d.nx + (a == 0 && !d.px)) * (d.ny + (a == 1 && !d.py)) * (d.nz + (a == 2 && !d.pz));
        hipLaunchKernelGGL(k_w0_sphere, dim3(grid_for(n)), dim3(kBlock), 0, s, d, a, h, center[0], center[1],
                           center[2], w0, re, ne, us[a]);
    }
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
