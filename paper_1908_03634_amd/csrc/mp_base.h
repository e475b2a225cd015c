// mp_base.h -- launchers of the base-state kernels (Sec. 3.1 and the base
// state modules of Sec. 3.2): the lateral Average, the irregular radii and
// the one-dimensional scans (Enforce HSE, beta0, w0).  Host side.
#pragma once
#include <hip/hip_runtime.h>

namespace mp {

struct Dims;

// ---- lateral Average over the radii h sqrt(0.75 + 2m) (even extents) -----
// The octant list: the cells of the high octant (nx/2 x ny/2 x nz/2, octant
// index a' + nx/2 (b' + ny/2 c')) grouped by radius, memory order within a
// radius: list[offs[m] .. offs[m+1]).  Built on the device by a stable
// counting sort; cnt (oct_count_bytes), rank (one unsigned per octant cell),
// cntm (nm doubles) and scan_work (scan_work_doubles(nm)) are scratch.
long long oct_window(int nx, int ny);
long long oct_count_bytes(int nx, int ny, int nz);
void launch_radius_list(int nx, int ny, int nz, long long nm, unsigned* cnt, unsigned* rank, double* cntm,
                        long long* offs, unsigned* list, double* scan_work, hipStream_t s);
// avg[m] = (sum of phi over the cells of radius m) / their count, count[m] =
// that count (count may be nullptr); fold: one double per octant cell.
void launch_average(const Dims& d, long long nm, const long long* offs, const unsigned* list, const double* phi,
                    double* fold, double* avg, double* count, hipStream_t s);
// The radius averages avg (nm) interpolated onto r_j = (j + 1/2) dr, j < n1d.
void launch_average_uniform(long long nm, double h, const double* avg, const long long* offs, int n1d, double dr,
                            double* out, hipStream_t s);
// U += w0 e_r on the faces (planar: interior z faces from w0[k]; spherical:
// w0(r_f) e_r . n_f, w0 linear between the edges re[0..ne)); walls unchanged.
void launch_w0_faces(const Dims& d, int planar, double h, const double* center, const double* w0, const double* re,
                     long long ne, double* ux, double* uy, double* uz, hipStream_t s);

// Centres rc (nm) and edges re (nm + 1) of the irregular base state.
void launch_irregular_radii(long long nm, double h, double* rc, double* re, hipStream_t s);

// ---- multi-block scans of the one-dimensional base state ----------------
// Each scan runs over tiles of kScanTile values, one workgroup per tile: the
// tile totals, then (one workgroup) their exclusive prefix, then every tile
// again from its prefix; the association of the sums is fixed, so results are
// reproducible.  work: scan_work_doubles(n) doubles of device memory that
// every value of the call's scratch comes from (nothing is assumed zero).
constexpr long long kScanTile = 4096;
inline long long scan_tiles(long long n) { return (n + kScanTile - 1) / kScanTile; }
inline long long scan_work_doubles(long long n) { return 3 * scan_tiles(n) + 8; }

// Enforce HSE (trapezoidal across centres, cutoff density).  The first
// centre at or below rho_cutoff (n if none) goes to jc_d (as a double) and
// to jc_ll (as a long long); either may be nullptr.
void launch_enforce_hse(long long n, const double* rc, const double* rho0, const double* g_edge, double p0_base,
                        double rho_cutoff, double* p0, double* work, double* jc_d, long long* jc_ll,
                        hipStream_t s);
// beta0 from p0 and Gamma1 (definition of beta0); bad[0] counts invalid inputs.
void launch_beta0_from_p0(long long n, double rho0_centre, const double* p0, const double* gamma1, double* beta0,
                          double* work, double* bad, hipStream_t s);
// w0 on the n + 1 edges from div(beta0 w0 e_r) = beta0 (sbar - psi) (psi may be nullptr).
void launch_w0(int spherical, long long n, const double* rc, const double* re, const double* beta0, const double* sbar,
               const double* psi, double* w0, double* work, hipStream_t s);

// out = S - Sbar(cell) with Sbar filled from the table tab (n1d entries at
// r_j = (j + 1/2) dr about center) linearly (geometry 1) or quadratically (3).
void launch_split_fill(const Dims& d, double h, int geometry, const double* tab, int n1d, double dr,
                       const double* center, const double* S, double* out, hipStream_t s);

// offs[0] = 0, offs[m + 1] = cnt[0] + ... + cnt[m] (integer-valued doubles).
void launch_offsets_of_counts(long long nm, const double* cnt, long long* offs, double* work, hipStream_t s);

// Text of the last failure of mp_enforce_hse_noalloc on the calling thread.
const char* noalloc_last_error();

}  // namespace mp
