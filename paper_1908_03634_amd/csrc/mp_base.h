// mp_base.h -- launchers of the base-state kernels (Sec. 3.1 and the base
// state modules of Sec. 3.2): the lateral Average, the irregular radii and
// the one-dimensional scans (Enforce HSE, beta0, w0).  Host side.
#pragma once
#include <hip/hip_runtime.h>

namespace mp {

// Lateral Average over the irregular radii: avg[m] = sum of phi over the
// cells listed for radius m (cells[offs[m] .. offs[m+1])) / their count.
void launch_average(long long nm, const long long* offs, const unsigned* cells, const double* phi, double* avg,
                    double* count, hipStream_t s);

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

// Text of the last failure of mp_enforce_hse_noalloc on the calling thread.
const char* noalloc_last_error();

}  // namespace mp
