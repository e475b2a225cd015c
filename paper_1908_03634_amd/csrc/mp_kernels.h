// mp_kernels.h -- host-side launchers of the gfx950 kernels (no HIP types
// beyond hipStream_t).  Every launcher enqueues on `s` and does not synchronise.
#pragma once
#include <hip/hip_runtime.h>

namespace mp {

struct Dims;

// Coefficients of one level.  Face mode: three low-face arrays (x, y, z).
// Cell mode (cell != nullptr): one array of cell values beta0/rho; the face
// value between cells L and R is their harmonic mean, formed when needed.
// The mapping defines the faces exactly that way, so on the finest level cell
// mode reads one word per cell instead of three.
template <typename T>
struct Coef {
    const T* x;
    const T* y;
    const T* z;
    const T* cell;
};

constexpr int kBlock = 256;
// Reductions write one partial per block; z-marching launches are shaped to
// stay near this many blocks (see mp_launch.h).
constexpr long long kZBlocks = 8192;
// Partial sums of 1D grid-stride reductions use at most this many blocks.
constexpr int kMaxRedBlocks = 2048;

int red_blocks(long long n);
// Number of partials written by the z-marching reductions on these dims.
int zred_blocks(const Dims& d);

// ---- reductions ---------------------------------------------------------
// out[0] = scale * sum(partials[0..nb)); when rms_out != nullptr also
// rms_out[0] = sqrt(sum / count), rms_out[1] = 1 / rms_out[0] (1 if the sum is 0).
// zero_out (or nullptr): a device scalar set to 0 by the same launch.
void launch_final_sum(const double* partials, int nb, double* out, double scale, double* rms_out, double count,
                      hipStream_t s, double* zero_out = nullptr);
// partials[b] = per-block sum of x (grid-stride, fixed order).
void launch_sum(const double* x, long long n, double* partials, int nb, hipStream_t s);
// x[q] -= mean[0]; partials = per-block sum of x^2 after the update; when
// x32 != nullptr also x32[q] = float(x[q] * pair[1]).  keep: x is left as it
// was (the sums and x32 as if updated).
void launch_sub_mean_sumsq(double* x, long long n, const double* mean, double* partials, int nb, hipStream_t s,
                           float* x32 = nullptr, const double* pair = nullptr, bool keep = false);
// From per-block sums s1 (partials) and s2 (partials2) of b and b^2 over n
// values: mean_out[0] = s1 / n and a scale for b - mean, the rms
// r = sqrt(s2 / n - mean^2) (sqrt(s2 / n) where cancellation leaves under
// 1e-6 of it; 1 for a zero b), written as the pairs (r, 1 / r) at pair0 and
// pair1.
void launch_final_moments(const double* partials, const double* partials2, int nb, long long n, double* mean_out,
                          double* pair0, double* pair1, hipStream_t s);
// x[q] -= mean[0].
void launch_sub_mean(double* x, long long n, const double* mean, hipStream_t s);
// y[q] = a y[q] + b x[q] (y not read when a == 0).
void launch_axpby(long long n, double a, double b, const double* x, double* y, hipStream_t s);
// b[q] = -rhs[q]; partials = per-block sum of b.
void launch_neg_copy_sum(const double* rhs, double* b, long long n, double* partials, int nb, hipStream_t s);

// ---- mapping and coefficients ---------------------------------------------
// beta0 on cells (planar injection or spherical linear interpolation) and
// ccell = beta0 / rho (and its FP32 copy when ccell32 != nullptr); partials
// (zred_blocks) = per-block count of invalid cells.
void launch_fill(const Dims& d, double h, int geometry, const double* tab, int n1d, double dr, double cx0, double cy0,
                 double cz0, const double* rho, double* beta0, double* ccell, float* ccell32, double* partials,
                 hipStream_t s);
// Face coefficients from cell values (harmonic mean): internal low-face FP64
// (c64*, may be nullptr) and FP32 (c32*, may be nullptr) arrays and external
// FP64 face arrays (e*, may be nullptr).
void launch_faces_from_cells(const Dims& d, const double* ccell, double* c64x, double* c64y, double* c64z,
                             float* c32x, float* c32y, float* c32z, double* ex, double* ey, double* ez,
                             hipStream_t s);
// Internal low-face coefficients from external face arrays; partials
// (zred_blocks) counts invalid (negative or non-finite) entries.
void launch_import_faces(const Dims& d, const double* ex, const double* ey, const double* ez, double* c64x,
                         double* c64y, double* c64z, float* c32x, float* c32y, float* c32z, double* partials,
                         hipStream_t s);
// Coarse low-face coefficients: mean of the 4 fine faces covering each face.
template <typename Tin, typename Tout>
void launch_coef_restrict(const Dims& fine, const Tin* fx, const Tin* fy, const Tin* fz, Tout* cx, Tout* cy,
                          Tout* cz, hipStream_t s);
// The same from fine cell values (fine faces = harmonic means, in FP64).
template <typename Tout>
void launch_coef_restrict_cells(const Dims& fine, const double* cc, Tout* cx, Tout* cy, Tout* cz, hipStream_t s);
// The same in FP32 from the half reciprocals h = 0.5 / c of the fine cell
// values (fine face = 1 / (h_a + h_b), the FP32 smoother's harmonic mean).
void launch_coef_restrict_cells32(const Dims& fine, const float* hc, float* cx, float* cy, float* cz, hipStream_t s);

// ---- projection ------------------------------------------------------------
// b = beta0 S' - D(beta0 U) (= minus the MAC right-hand side); partials
// (zred_blocks) = sum b, and partials2 = sum b^2 when given.  S' = S (smode
// 0), or S - Sbar with Sbar per plane (smode 1) or per irregular radius
// (smode 2): the velocity-split source.
void launch_mac_rhs(const Dims& d, double inv_h, const double* beta0, const double* ux, const double* uy,
                    const double* uz, const double* S, const double* sbar, int smode, double* b, double* partials,
                    hipStream_t s, double* partials2 = nullptr);
// partials (zred_blocks) = per-block sum of (beta0 S' - D(beta0 U) - shift[0])^2
// (no write): the divergence defect of a projected velocity.
void launch_rhs_defect(const Dims& d, double inv_h, const double* beta0, const double* ux, const double* uy,
                       const double* uz, const double* S, const double* sbar, int smode, const double* shift,
                       double* partials, hipStream_t s);
// avg[k] = mean of plane k (lateral average of a planar atmosphere).
void launch_plane_average(const Dims& d, const double* phi, double* avg, hipStream_t s);
// U <- U - (c/beta0_f) G phi on every non-wall face (in place).
void launch_vel_correct(const Dims& d, double inv_h, const Coef<double>& c64, const double* beta0, const double* phi,
                        double* ux, double* uy, double* uz, hipStream_t s);
// g = (G lam)(G phi) on every non-wall face, external layout; walls 0.
void launch_coef_grad(const Dims& d, double inv_h2, const double* lam, const double* phi, double* gx, double* gy,
                      double* gz, hipStream_t s);

// ---- multigrid -----------------------------------------------------------
// One colour of red-black Gauss-Seidel, in place (reference / fallback).
template <typename T>
void launch_rbgs(const Dims& d, T* phi, const T* rhs, const Coef<T>& c, T h2, int colour, int zero_init,
                 hipStream_t s);
// The two colour passes after a prolongation with the prolongation folded in
// (ec: the coarse correction): first = 1 for the first colour (every value
// read as x + e of its parent cell), 0 for the second (own value x + e).
// Equal bit for bit to launch_prolong and two launch_rbgs passes; even extents.
template <typename T>
void launch_rbgs_e(const Dims& d, T* phi, const T* rhs, const Coef<T>& c, T h2, int colour, int first, const T* ec,
                   hipStream_t s);
// Both colours in one launch, out of place (xo -> xn).  zero_init: xo is
// taken as zero.  ec: coarse correction added to xo while reading
// (prolongation fused into the sweep), or nullptr.
template <typename T>
void launch_sweep(const Dims& d, const T* xo, T* xn, const T* b, const T* cx, const T* cy, const T* cz, T h2,
                  int zero_init, const T* ec, hipStream_t s);
bool sweep_supported(const Dims& d);
template <typename T>
void launch_resid_restrict(const Dims& fine, const T* phi, const T* rhs, const Coef<T>& c, T inv_h2, T* coarse_rhs,
                           hipStream_t s);
template <typename T>
void launch_prolong(const Dims& fine, T* phi, const T* coarse_phi, hipStream_t s);
// BiCGStab in FP64 on the coarsest grid (one workgroup), made mean-zero on
// each connected part of the grid; work = 9 * n doubles.
// use_x0: start from phi (tolerance relative to the initial residual).
// iters: device counter the iterations are added to, or nullptr.
// skip_if_direct: a device flag (1: the direct bottom solve applies and this
// kernel returns at once), or nullptr.
template <typename T>
void launch_bottom(const Dims& d, const T* rhs, T* phi, const T* cx, const T* cy, const T* cz, double h2, double rtol,
                   int maxit, int use_x0, double* work, double* iters, const double* skip_if_direct, hipStream_t s);

// Direct bottom solve on grids of at most kDirectBottomCells cells.  With L
// the grid's Laplacian (diagonal: sum of the cell's six face coefficients,
// off-diagonal: minus the face coefficient; symmetric, positive semidefinite,
// null space the constants when every cell is coupled), A = L / h^2 and
// G = (L + alpha 1 1^T)^-1, alpha = trace(L) / n^2, the mean-zero solution of
// A x = b - mean(b) is
//   x = h^2 (G b - mean(G b))
// (G 1 = 1 / (alpha n), so G maps the mean of b onto a constant that the
// last mean removes).  G is built once per coefficient set by Gauss-Jordan
// elimination without pivoting (B = L + alpha 1 1^T is symmetric positive
// definite); a pivot at or below 1e-12 of the largest diagonal entry (a grid
// whose cells are not all coupled) marks G unusable: *valid = 0, else 1.
// G: kDirectBottomCells^2 doubles, row-major, zero outside n x n.
constexpr int kDirectBottomCells = 64;
template <typename T>
void launch_bottom_inverse(const Dims& d, const T* cx, const T* cy, const T* cz, double* G, double* valid,
                           hipStream_t s);
// x = the direct solution above for right-hand side b on the bottom grid d
// when *valid == 1 (else the kernel returns at once).
template <typename T>
void launch_bottom_direct(const Dims& d, const double* G, const double* valid, const T* b, T* x, double h2,
                          hipStream_t s);

// The coarse end of a V-cycle in one workgroup (levels lv[0..nlev), the last
// one solved directly from G when bottom_inv is set, else by one-wavefront
// conjugate gradients; it must hold <= 256 cells).
// The five arrays of every level and a residual scratch of the first level's
// size ((5 * all cells + cells of lv[0]) * sizeof(T) bytes) must fit in
// kCoarseLdsBytes of LDS.
constexpr int kMaxCoarse = 8;
constexpr int kCoarseLdsBytes = 128 * 1024;
template <typename T>
struct CoarseLevel {
    int nx, ny, nz;
    T h2, inv_h2;  // smoother / residual scalars in the level's precision
    double h2d;    // h^2 for the FP64 bottom solve
    T* x;
    T* b;
    const T* cx;
    const T* cy;
    const T* cz;
};
template <typename T>
struct CoarseArgs {
    int nlev;
    int px, py, pz;
    int nu1, nu2;
    int zero_init;  // x of lv[0] is zero on entry
    double bottom_rtol;
    int bottom_maxit;
    double* bottom_iters;  // device counter the bottom solve adds its iterations to, or nullptr
    const double* bottom_inv;  // G of the last level, or nullptr (conjugate gradients)
    const double* bottom_ok;   // device flag: 1 when G is usable (direct bottom)
    CoarseLevel<T> lv[kMaxCoarse];
};
template <typename T>
void launch_coarse_cycle(const CoarseArgs<T>& a, hipStream_t s);

// ---- register-blocked finest-level kernels (cell-value coefficients) -----
// Each lane owns a strip of 2-8 x-adjacent cells in 2-4 rows and marches
// along z; valid when blk_supported(d) and every array is 16-byte aligned.
// Results equal the one-cell kernels' bit for bit.
bool blk_supported(const Dims& d);
// Partials written by launch_resid64_blk on these dims (<= kMaxRedBlocks
// unless nx * ny alone needs more blocks).
int blk_reduce_blocks(const Dims& d);
// Smoother pass modes.
//   GS_PLAIN:  x as stored.
//   GS_ZERO:   x is zero on entry (not read; the other colour is written 0).
//   GS_E_ALL:  first colour after prolongation: every x value read is taken
//              as x + e of its parent coarse cell (ec = coarse correction).
//   GS_E_OWN:  second colour after prolongation: the updated cell's own value
//              is x + e.  GS_E_ALL then GS_E_OWN equals launch_prolong
//              followed by two GS_PLAIN passes.
enum { GS_PLAIN = 0, GS_ZERO = 1, GS_E_ALL = 2, GS_E_OWN = 3 };
// phi != nullptr (FP32 only): also phi += irs[0] * x on every cell (the
// refinement update fused into the last pass of a V-cycle).  ev0 != nullptr:
// the launch records its own start and end in ev0 / ev1.
template <typename T>
void launch_gs_blk(const Dims& d, T* x, const T* b, const T* cc, T h2, int colour, int mode, const T* ec,
                   double* phi, const double* irs, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s);
// Both colours of one red-black sweep in one pass, out of place (xo -> xn),
// in FP32 when fsw_supported(d) (blocked layout, nx = 128, 256, 384 or 512;
// whole rows per workgroup, rows exchanged through LDS).  Modes:
//   FS_PLAIN:   xo as stored;
//   FS_ZERO:    xo is zero (not read);
//   FS_PROLONG: xo + e of each cell's parent coarse cell (ec), i.e. the
//               prolongation applied on the fly.
// phi != nullptr (FP32): also phi += irs[0] * xn, or phi = irs[0] * xn when
// bit 0 of irf is set (phi zero on entry, not read).  Equal bit for bit to
// two launch_gs_blk colour passes.
enum { FS_PLAIN = 0, FS_ZERO = 1, FS_PROLONG = 2 };
// Both colours of one red-black sweep in one launch, out of place (xo -> xn),
// on a level with stored faces and even extents (rb_pair_supported), in the
// modes above: a thread updates one red and one black cell, evaluating the
// black cell's other red neighbours again from old values.  Equal bit for bit
// to two launch_rbgs / launch_rbgs_e colour passes.
bool rb_pair_supported(const Dims& d);
template <typename T>
void launch_rb_pair(const Dims& d, const T* xo, T* xn, const T* b, const Coef<T>& c, T h2, int mode, const T* ec,
                    hipStream_t s);
bool fsw_supported(const Dims& d);
// Rows of 192 cells with walls in x: the stored-face sweep below on 256-cell
// strips, the lanes past the row's end idle.
bool fsw_narrow_supported(const Dims& d);
template <typename T>
void launch_fsw_blk(const Dims& d, const T* xo, T* xn, const T* b, const T* cc, T h2, int mode, const T* ec,
                    double* phi, const double* irs, int irf, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s);
// The same sweep on a level with stored low-face coefficients c (FP32; equal
// bit for bit to two launch_gs_blkf colour passes).
template <typename T>
void launch_fsw_blkf(const Dims& d, const T* xo, T* xn, const T* b, const Coef<T>& c, T h2, int mode, const T* ec,
                     hipStream_t s);
// The same two kernels on a level with stored low-face coefficients c.
template <typename T>
void launch_gs_blkf(const Dims& d, T* x, const T* b, const Coef<T>& c, T h2, int colour, int mode, const T* ec,
                    hipStream_t s);
template <typename T>
void launch_rr_blkf(const Dims& d, const T* x, const T* b, const Coef<T>& c, T inv_h2, T* bc, hipStream_t s);
// Coarse rhs = mean of the 8 fine residuals b - A x (as launch_resid_restrict).
template <typename T>
void launch_rr_blk(const Dims& d, const T* x, const T* b, const T* cc, T inv_h2, T* bc, hipStream_t s);
// As launch_resid64 with cell-value coefficients cc; shift != nullptr: b is
// taken as b - shift[0] (the same bits as b stored with the mean removed).
void launch_resid64_blk(const Dims& d, const double* x, const double* b, const double* cc, double inv_h2, float* r32,
                        const double* inv_s, double* partials, int* nb_out, hipStream_t s,
                        const double* shift = nullptr);

// ---- register-blocked projection kernels (finest level, periodic x and y) --
// Same results, bit for bit, as launch_mac_rhs / launch_rhs_defect /
// launch_vel_correct (cell-value coefficients) when proj_blk_supported(d)
// and every array is 16-byte aligned.
bool proj_blk_supported(const Dims& d);
// shift == nullptr: b written, partials = per-block sums of b (and, when
// partials2 != nullptr, partials2 = per-block sums of b^2); otherwise no
// write and partials = per-block sums of (b - shift[0])^2.  *nb_out partials.
void launch_rhs_blk(const Dims& d, double inv_h, const double* beta0, const double* ux, const double* uy,
                    const double* uz, const double* S, const double* sbar, int smode, double* b, const double* shift,
                    double* partials, int* nb_out, hipStream_t s, double* partials2 = nullptr);
void launch_vc_blk(const Dims& d, double inv_h, const double* cc, const double* beta0, const double* phi, double* ux,
                   double* uy, double* uz, hipStream_t s);
int proj_blk_reduce_blocks(const Dims& d);

// ---- FP64 level-0 operations --------------------------------------------
// y = M x = -(A x).
void launch_apply64(const Dims& d, const double* x, const Coef<double>& c, double inv_h2, double* y, hipStream_t s);
// r = b - A phi; partials (*nb_out of them) = per-block sum r^2; when
// r32 != nullptr, r32 = float(r * inv_s[0]).
void launch_resid64(const Dims& d, const double* phi, const double* b, const Coef<double>& c, double inv_h2,
                    float* r32, const double* inv_s, double* partials, int* nb_out, hipStream_t s);
// phi += s[0] * e.
void launch_ir_update(long long n, double* phi, const float* e, const double* s, hipStream_t st);
// First refinement step from a zero iterate (residual = b): r32 =
// float(b * pair_in[1]) when r32 != nullptr; pair_out = pair_in.
void launch_scale32(long long n, const double* b, float* r32, const double* pair_in, double* pair_out, hipStream_t st);

// ---- nodal projection (node-based phi, cell-centred U and sigma) --------
// Cells nx x ny x nz with per-axis periodicity; nodes mx = nx + (1 - px) etc.
// Node arrays [mz][my][mx], cell arrays [nz][ny][nx].  A is the trilinear
// finite-element operator h^-3 sum_e sigma_e int grad . grad (symmetric
// positive semi-definite); the solver works on A x = b with b = -R.
struct NDims {
    int nx, ny, nz;
    int px, py, pz;
    int mx, my, mz;
};
// One colour (0..3, by i and j parity) of Gauss-Seidel on A x = b; h12 = 12 h^2.
template <typename T>
void launch_nd_gs(const NDims& d, T* x, const T* b, const T* sg, T h12, int colour, hipStream_t s);
// The two colours of the rows of parity rowpar (x parity lead first), out of
// place: own rows read from xo, rows of the other parity from xnb, own rows
// written to xn (FP32, nd_pair_supported: periodic x and y, 128 or 256 nodes
// per row).  Equal bit for bit to the two launch_nd_gs colours.
bool nd_pair_supported(const NDims& d);
template <typename T>
void launch_nd_pair(const NDims& d, const T* xo, const T* xnb, T* xn, const T* b, const T* sg, T h12, int rowpar,
                    int lead, hipStream_t s);
// r = b - A x; inv_h12 = 1 / (12 h^2).
template <typename T>
void launch_nd_resid(const NDims& d, const T* x, const T* b, const T* sg, T inv_h12, T* r, hipStream_t s);
// bc = (1/8) P^T rf (P trilinear interpolation from the grid coarsened by 2).
template <typename T>
void launch_nd_restrict(const NDims& f, const NDims& c, const T* rf, T* bc, hipStream_t s);
// xf += P ec; col != 0: a column of fine nodes per thread, each coarse
// plane's sum formed once (the same bits as one thread per node).
template <typename T>
void launch_nd_prolong(const NDims& f, const NDims& c, T* xf, const T* ec, int col, hipStream_t s);
// The smoother colour and the residuals above by threads that walk node
// columns along z (registers carry the neighbour planes); bitwise equal to
// the one-node kernels.  Valid when nd_col_supported(d).
bool nd_col_supported(const NDims& d);
// Partials written by launch_nd_resid64_col on these dims.
int nd_col_reduce_blocks(const NDims& d);
// As launch_nd_rhs by node columns (bitwise equal); *nb_out partials
// (<= nd_col_reduce_blocks(d)).
void launch_nd_rhs_col(const NDims& d, double inv4h, const double* beta0, const double* ux, const double* uy,
                       const double* uz, const double* S, const double* mean, double* out, int squares,
                       double* partials, int* nb_out, hipStream_t s);
template <typename T>
void launch_nd_gs_col(const NDims& d, T* x, const T* b, const T* sg, T h12, int colour, hipStream_t s);
template <typename T>
void launch_nd_resid_col(const NDims& d, const T* x, const T* b, const T* sg, T inv_h12, T* r, hipStream_t s);
// As launch_nd_resid64; *nb_out partials (<= kMaxRedBlocks).
void launch_nd_resid64_col(const NDims& d, const double* x, const double* b, const double* sg, double inv_h12,
                           float* r32, const double* inv_s, double* partials, int* nb_out, hipStream_t s);
// Cell sigma of the grid coarsened by 2 (mean of 8 children), or, with
// coarsen = 0, a precision conversion of the same grid.
template <typename Tin, typename Tout>
void launch_nd_sigma(int nx, int ny, int nz, const Tin* sf, Tout* sc, int coarsen, hipStream_t s);
// FP64 conjugate gradients on the coarsest nodes (one workgroup); x from 0
// (or from x when use_x0), returned mean-zero; work = 4 * nodes doubles;
// iters: device counter the iterations are added to, or nullptr.
template <typename T>
void launch_nd_bottom(const NDims& d, const T* b, T* x, const T* sg, double inv_h12, double rtol, int maxit,
                      int use_x0, double* work, double* iters, hipStream_t s);
// The coarse end of a nodal V-cycle in one workgroup, every array in LDS
// (levels lv[0..nlev), all starting from zero; lv[0].b in, lv[0].x out).
template <typename T>
struct NdCoarseLevel {
    NDims d;
    T h12, inv_h12;  // 12 h^2 and its inverse
    T* x;            // global iterate of lv[0] (written at the end)
    const T* b;      // global right-hand side of lv[0]
    const T* sig;    // global cell sigma
};
template <typename T>
struct NdCoarseArgs {
    int nlev, nu1, nu2;
    double bottom_rtol;
    int bottom_maxit;
    double bottom_inv_h12;
    double* bottom_iters;  // device counter the bottom solve adds its iterations to, or nullptr
    NdCoarseLevel<T> lv[kMaxCoarse];
};
// LDS bytes the coarse set lv[0..nlev) needs (must be <= kCoarseLdsBytes).
template <typename T>
long long nd_coarse_lds_bytes(const NDims* lv, int nlev);
template <typename T>
void launch_nd_coarse(const NdCoarseArgs<T>& a, hipStream_t s);
// partials (nb blocks) = per-block sum of beta0 * S over the cells.
void launch_nd_src_sum(long long n, const double* beta0, const double* S, double* partials, int nb, hipStream_t s);
// b = L(beta0 S - mean[0]) - D(beta0 U) on the nodes (out may be nullptr);
// partials (nb blocks) = per-block sum of b^2 (squares) or of b.
// inv4h = 1 / (4h).
void launch_nd_rhs(const NDims& d, double inv4h, const double* beta0, const double* ux, const double* uy,
                   const double* uz, const double* S, const double* mean, double* out, int squares,
                   double* partials, int nb, hipStream_t s);
// r = b - A x in FP64 (sigma FP64); r32 = float(r * inv_s[0]) when r32 !=
// nullptr; partials (nb blocks) = per-block sum of r^2.
void launch_nd_resid64(const NDims& d, const double* x, const double* b, const double* sg, double inv_h12,
                       float* r32, const double* inv_s, double* partials, int nb, hipStream_t s);
// y = -(A x) in FP64.
void launch_nd_apply64(const NDims& d, const double* x, const double* sg, double inv_h12, double* y, hipStream_t s);
// U -= (sigma / beta0) G phi on every cell (cell-average gradient of phi_h).
void launch_nd_correct(const NDims& d, double inv4h, const double* sg, const double* beta0, const double* phi,
                       double* ux, double* uy, double* uz, hipStream_t s);

// Plain device copy (bandwidth calibration of the traffic counters).
void launch_copy(const double* src, double* dst, long long n, hipStream_t s);

}  // namespace mp
