/*
 * mproj.h -- C ABI of the MI355X (gfx950) MAC-projection library libmproj.so.
 *
 * The operation is the MAC projection of the low Mach number method of Fan,
 * Nonaka, Almgren, Harpole and Zingale ("MAESTROeX: A Massively Parallel Low
 * Mach Number Astrophysical Solver"): Sec. 3.2, Steps 3 and 7, enforce the
 * velocity constraint of Sec. 2,
 *        div(beta0 U) = beta0 (S - (1/(Gamma1 p0)) dp0/dt),
 * on face-centred velocities by a variable-coefficient Poisson solve (Appendix
 * A).  With the dp0/dt term folded into S by the caller, the library solves
 *        div((beta0/rho) grad phi) = div(beta0 U) - beta0 S       (mean removed)
 * and sets U <- U - (beta0/rho)/beta0 grad phi, so that div(beta0 U) = beta0 S
 * up to the solve residual and the mean.  beta0 comes from a 1D base state
 * mapped onto the cells by the fill module of Sec. 3.1.
 *
 * Discretisation: uniform cell-centred grid of spacing h; for a face f between
 * cells L and R, (G phi)_f = (phi_R - phi_L)/h; (D F)_i = sum over the three
 * axes of (F_high - F_low)/h; the operator is M = D C G with C the face
 * coefficients (harmonic mean of beta0/rho of the two cells); beta0 on a face
 * is the arithmetic mean of the two cells.  Periodic axes wrap; Neumann axes
 * end in walls (c = 0 and U = 0 on the two boundary faces).  M is symmetric
 * negative semi-definite with the constants as null space: right-hand sides
 * are made mean-zero and solutions are returned mean-zero.
 *
 * Layouts: every array is C order with x fastest.
 *   cells    [nz][ny][nx]
 *   x faces  [nz][ny][nx + bx]      b = 0 (periodic): n faces per row, face i
 *   y faces  [nz][ny + by][nx]      is the low face of cell i; b = 1 (Neumann):
 *   z faces  [nz + bz][ny][nx]      n + 1 faces, faces 0 and n are walls.
 * Entries of U on wall faces are ignored on input and left unchanged; wall
 * coefficients are ignored on input and written as 0 on output.
 *
 * Pointers: every array argument is a DEVICE pointer (HIP global memory on the
 * context's device), owned by the caller, float64, contiguous, and must not
 * alias another argument of the same call unless stated.  Scalars and the
 * small structs below live in host memory.  Calls enqueue work on the
 * context's stream and return after the last device->host read that the call
 * needs, so outputs are ready in stream order when the call returns.
 *
 * Errors: every call returns an mp_status; no call aborts or throws.  Argument
 * checks that need no device run before any HIP call.  mp_last_error() gives a
 * text for the last failure on a context.  A context is not thread-safe; use
 * one per host thread and stream.
 */
#ifndef MPROJ_H
#define MPROJ_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MP_OK = 0,
    MP_ERR_ARG = 1,            /* bad argument (null pointer, size, enum, table) */
    MP_ERR_DEVICE = 2,         /* no usable HIP device, or a HIP call failed */
    MP_ERR_NOMEM = 3,          /* device allocation failed */
    MP_ERR_NOT_CONVERGED = 4,  /* max_outer reached; outputs hold the best iterate */
    MP_ERR_NONFINITE = 5,      /* NaN/Inf found in an input or a norm */
    MP_ERR_SINGULAR_RHS = 6,   /* demean == 0 and the right-hand side has a mean */
    MP_ERR_STATE = 7           /* call order: coefficients or base state missing */
} mp_status;

enum { MP_BC_PERIODIC = 0, MP_BC_NEUMANN = 1 };
enum { MP_PLANAR = 0, MP_SPHERICAL = 1, MP_SPHERICAL_IRREGULAR = 2, MP_SPHERICAL_QUADRATIC = 3 };
enum { MP_FP64 = 0, MP_MIXED = 1 };
enum { MP_SMOOTH_AUTO = 0, MP_SMOOTH_PER_COLOUR = 1, MP_SMOOTH_FUSED = 2 };

/* Solver configuration, fixed for the life of a context. */
typedef struct mp_config {
    int nx, ny, nz;          /* cells per axis, each >= 1 */
    double h;                /* cell size, > 0 */
    int bc[3];               /* MP_BC_PERIODIC or MP_BC_NEUMANN for x, y, z */
    int precision;           /* MP_FP64: FP64 V-cycles; MP_MIXED: FP32 V-cycles
                                inside FP64 iterative refinement */
    double rtol;             /* stop when ||rhs - M phi||_2 <= rtol ||rhs||_2 (FP64) */
    int max_outer;           /* max residual checks: refinement steps (MIXED)
                                or groups of V-cycles (FP64) */
    int nu1, nu2;            /* red-black Gauss-Seidel sweeps (over-relaxed,
                                omega = 1.08) before / after */
    int cycles_per_outer;    /* V-cycles between residual checks (FP32
                                V-cycles per refinement step in MIXED);
                                0: predicted from the last step's
                                contraction (1 to 4; a last cycle the
                                prediction would use for <= 0.45 of it is
                                replaced by one more finest-level
                                post-smoothing sweep) */
    double bottom_rtol;      /* bottom-solver tolerance on the coarsest grid
                                where it is not solved directly (<= 64 cells,
                                all coupled): conjugate gradients in one
                                wavefront up to 256 cells, BiCGStab in one
                                workgroup above, mean-zero on each connected
                                part of the grid */
    int bottom_max_iter;     /* bottom-solver iteration cap */
    int demean;              /* 1: remove the mean of the rhs; 0: require mean ~ 0 */
    int kernel_timing;       /* 1: time the finest-level smoother launches with
                                HIP events (mp_info.smooth_*) */
    int smoother;            /* MP_SMOOTH_AUTO: both colours of a sweep in one
                                launch wherever it pays: register-blocked
                                levels in MIXED whose rows are 128, 256, 384
                                or 512 cells, face-coefficient levels of >= 4M cells
                                (tiled), and the other FP32 levels below the
                                finest of <= 64^3 cells with even extents (one
                                red and one black cell per thread); one launch
                                per colour elsewhere.
                                MP_SMOOTH_PER_COLOUR: one launch per colour on
                                every level; MP_SMOOTH_FUSED: both colours in
                                one launch wherever the grid allows.  All
                                three give the same bits. */
    int coarse_cycle;        /* 1: run levels of <= 4096 cells in one workgroup
                                (bottom <= 256 cells by one wavefront); 0: one
                                launch per operation on every level */
    int blocked;             /* 1: on the finest level, register-blocked
                                kernels (a strip of 2-8 x cells in 2-4 rows
                                per lane, marching along z) when its
                                coefficients are cell values (after
                                mp_map_base_state), nx % 128 == 0,
                                ny % 4 == 0, nz is even and >= 4, and the
                                solution array is 16-byte aligned; 0: one
                                cell per thread.  Same bits in FP64. */
    void *stream;            /* hipStream_t for every launch; NULL = null stream */
    int device;              /* HIP device ordinal */
} mp_config;

/* Per-call report, filled by mp_mac_project and mp_solve. */
typedef struct mp_info {
    int outer_iters;         /* residual checks after the first (refinement
                                steps in MIXED) */
    int vcycles;             /* V-cycles run */
    int bottom_iters_total;  /* iterations of every coarsest-grid solve of the
                                call (conjugate gradients or BiCGStab),
                                counted on the device */
    int levels;              /* multigrid levels, finest included */
    double rel_resid;        /* final ||rhs - M phi||_2 / ||rhs||_2 in FP64 */
    double div_defect;       /* ||D(beta0 U_new) - beta0 S - m||_2 / ||rhs||_2 */
    double rhs_norm;         /* ||rhs||_2 after the mean is removed */
    double rhs_mean;         /* mean removed from div(beta0 U) - beta0 S */
    double resid_hist[64];   /* relative residual at each check */
    double ms_setup;         /* duration of the last mp_map_base_state or
                                mp_set_coefs on this context (fill, faces,
                                coefficient hierarchy; HIP events) */
    double ms_rhs, ms_solve, ms_correct;   /* phase times (HIP events) */
    double smooth_ms_total;  /* summed finest-level smoother time (kernel_timing) */
    int smooth_launches;     /* number of launches summed above */
    double smooth_bytes;     /* algorithmic HBM bytes of those launches */
    int smooth_form;         /* finest-level smoother: 0 = one launch per
                                colour, 1 = both colours of a sweep in one
                                launch */
    int flags;               /* bit 0: stagnation detected */
} mp_info;

typedef struct mp_ctx mp_ctx;

/* Fill *cfg with defaults for an nx x ny x nz grid: h = 1/nz, periodic x/y,
 * Neumann z, MIXED, rtol 1e-10, max_outer 100, V(2,2), predicted cycles per
 * step,
 * bottom 1e-8 / 400 iterations, demean 1, automatic smoother, coarse cycle on,
 * blocked kernels on, null stream, device 0. */
void mp_config_default(mp_config *cfg, int nx, int ny, int nz);

/* Create a context: validates cfg, selects the device, allocates the
 * multigrid hierarchy (levels halve every axis while all extents are even and
 * >= 4, so the coarsest grid keeps >= 2 cells per axis; it must hold <= 16384
 * cells).
 * Errors: MP_ERR_ARG (cfg), MP_ERR_DEVICE (no device), MP_ERR_NOMEM. */
int mp_init(const mp_config *cfg, mp_ctx **out);

/* Fill (Sec. 3.1) and face coefficients.
 * geometry MP_PLANAR: beta0_1d has n1d == nz entries, one per z cell (direct
 *   injection); dr and center are ignored (may be NULL).
 * geometry MP_SPHERICAL: beta0_1d[j] is beta0 at radius (j + 1/2) dr about the
 *   point center[3] (host array, physical units); each cell takes the linear
 *   interpolation at the distance of its centre, holding the end values beyond
 *   the table.
 * geometry MP_SPHERICAL_QUADRATIC: the same table, quadratic interpolation
 *   (the parabola through the three table points around the nearest one,
 *   kept inside the table); n1d >= 3.
 * geometry MP_SPHERICAL_IRREGULAR: the irregular base state of Sec. 3.1: the
 *   star centre is the grid node in the middle of the box (all extents even),
 *   every cell centre lies at h sqrt(0.75 + 2m) for an integer m, and
 *   beta0_1d[m] is beta0 at that radius (n1d == mp_radius_count); no
 *   interpolation; dr and center are ignored.
 * rho: cell density (> 0).  cx, cy, cz: output face coefficients beta0/rho
 * (harmonic mean, walls 0), FP64, face layouts above; all three or none may be
 * NULL (the solver keeps its own copy either way).
 * Rebuilds the coefficient hierarchy.  Errors: MP_ERR_ARG (sizes, dr, n1d),
 * MP_ERR_NONFINITE (rho <= 0 or non-finite values). */
int mp_map_base_state(mp_ctx *ctx, int geometry, const double *beta0_1d, int n1d, double dr, const double *center,
                      const double *rho, double *cx, double *cy, double *cz);

/* Use caller face coefficients (>= 0, finite; walls ignored) instead of the
 * mapped ones; keeps any mapped beta0.  Rebuilds the coefficient hierarchy. */
int mp_set_coefs(mp_ctx *ctx, const double *cx, const double *cy, const double *cz);

/* MAC projection (Sec. 3.2 Steps 3/7, Appendix A).  In: ux, uy, uz (U before
 * projection), S (cells), phi (initial guess when use_initial_guess != 0).
 * Out: ux, uy, uz projected in place, phi (mean-zero), *info (may be NULL).
 * Needs mp_map_base_state first (MP_ERR_STATE otherwise).  On
 * MP_ERR_NOT_CONVERGED the outputs hold the last iterate and its projection. */
int mp_mac_project(mp_ctx *ctx, double *ux, double *uy, double *uz, const double *S, double *phi,
                   int use_initial_guess, mp_info *info);

/* Velocity-split MAC projection (Appendix A): as mp_mac_project with the
 * source S replaced by S - Sbar, Sbar being the lateral average of S
 * (Sec. 3.1): the plane averages after an MP_PLANAR mapping; the averages
 * over the irregular radii after an MP_SPHERICAL_IRREGULAR mapping; after an
 * MP_SPHERICAL or MP_SPHERICAL_QUADRATIC mapping the radius averages
 * interpolated onto the mapping's table r_j = (j + 1/2) dr (as
 * mp_average_uniform) and filled back onto the cells with the mapping's
 * interpolation.  The projected velocity U~ then satisfies
 * div(beta0 U~) = beta0 (S - Sbar) up to the solve residual; the base-state
 * velocity w0 (mp_w0) is added by mp_add_w0.  sbar: device array receiving
 * Sbar (nz, mp_radius_count or n1d entries), or NULL.  Errors as
 * mp_mac_project; MP_ERR_STATE when a uniform spherical mapping's centre is
 * not the node in the middle of the box (or an extent is odd); the first
 * call after a spherical mapping builds the radius list (MP_ERR_NOMEM). */
int mp_mac_project_split(mp_ctx *ctx, double *ux, double *uy, double *uz, const double *S, double *phi,
                         int use_initial_guess, double *sbar, mp_info *info);

/* ---- nodal projection (Sec. 3.2 Step 11, Appendix A) --------------------
 * The velocity update of Step 11 projects a CELL-CENTRED velocity with a
 * scalar phi on the grid NODES.  The paper defers the discretisation to an
 * earlier paper; here it is trilinear finite elements on the cells:
 *   phi_h = sum_n phi_n N_n (N_n the trilinear hat function of node n),
 *   sigma = beta0/rho constant per cell (from the last mp_map_base_state),
 *   (M phi)_n = -h^-3 sum_e sigma_e int_e grad phi_h . grad N_n,
 *   (D V)_n   = -h^-3 sum_e V_e . int_e grad N_n      (nodal divergence),
 *   (G phi)_e =  h^-3 int_e grad phi_h                 (cell-average gradient),
 *   (L f)_n   =  h^-3 sum_e f_e int_e N_n              (load: 1/8 per corner).
 * Node counts per axis: n (periodic; node n is node 0) or n + 1 (Neumann
 * walls, whose nodes are unknowns taking only the cells inside).  Node arrays
 * are C order [nz+bz][ny+by][nx+bx], x fastest (b = 1 for Neumann axes).  */

/* Node counts (x, y, z) of this context's grid. */
int mp_nodal_shape(const mp_ctx *ctx, int *mx, int *my, int *mz);

/* Nodal projection.  Solves M phi = D(beta0 U) - L(beta0 S - m), m the cell
 * mean of beta0 S, to the configured relative residual (FP64, or FP32
 * V-cycles inside FP64 refinement in MP_MIXED; 4-colour Gauss-Seidel V(nu1,
 * nu2), full-weighting restriction, trilinear prolongation, cell sigma
 * coarsened as the mean of its 8 children, FP64 conjugate gradients on the
 * coarsest grid of at most 16384 nodes), returns phi with zero node mean,
 * then U_e <- U_e - (sigma_e / beta0_e)(G phi)_e on every cell.  D sigma G
 * differs from M, so U meets the constraint only approximately (an
 * approximate projection); info->div_defect reports
 * ||D(beta0 U_new) - L(beta0 S - m)|| / ||right-hand side||.
 * ux, uy, uz: cells, device, in/out; S: cells; phi: nodes (initial guess when
 * use_initial_guess).  info->rhs_mean = m.  Needs a prior mp_map_base_state
 * (MP_ERR_STATE).  The first call allocates the node hierarchy (MP_ERR_NOMEM).
 * MP_ERR_ARG: NULL arrays, or a coarsest grid above 16384 nodes.
 * MP_ERR_NOT_CONVERGED / MP_ERR_NONFINITE as mp_mac_project. */
int mp_nodal_project(mp_ctx *ctx, double *ux, double *uy, double *uz, const double *S, double *phi,
                     int use_initial_guess, mp_info *info);

/* y = M x on the nodes, FP64, with sigma from the last mapping. */
int mp_nodal_apply(mp_ctx *ctx, const double *x, double *y);

/* Perturbational pressure from the nodal projection's scalar (Sec. 3.2 Step
 * 11; Appendix A: the gradient of that scalar updates pi).  The time-step
 * scaling belongs to an earlier paper, so it is the caller's:
 *   pi <- a pi + s phi   on every node (a = 0: pi is written, not read),
 * so that (sigma/beta0) G(pi)/s is the correction the projection applied
 * when a = 0.  phi, pi: device, nodes (mp_nodal_shape), FP64; may not alias.
 * Errors: MP_ERR_ARG (NULL or aliased arrays), MP_ERR_NONFINITE (a or s). */
int mp_nodal_pi(mp_ctx *ctx, const double *phi, double a, double s, double *pi);

/* Solve M x = rhs (rhs mean removed when demean = 1); x mean-zero.  This is
 * also the adjoint solve, M being symmetric. */
int mp_solve(mp_ctx *ctx, const double *rhs, double *x, int use_initial_guess, mp_info *info);

/* Number of radii h sqrt(0.75 + 2m), m = 0 .. *nm - 1, of the irregular base
 * state (Sec. 3.1) on this grid: ((nx-1)^2 + (ny-1)^2 + (nz-1)^2 - 3)/8 + 1,
 * or 0 when an extent is odd (no grid node in the middle of the box). */
int mp_radius_count(const mp_ctx *ctx, long long *nm);

/* Lateral Average over the irregular radii (Sec. 3.1; the Average module of
 * Sec. 3.2): avg[m] = (sum of phi over the cells whose centres lie at radius
 * m) / (number of those cells); count[m] = that number.  Radii that no cell
 * centre reaches get 0 and 0.  phi: cells; avg, count: device arrays of
 * mp_radius_count doubles (count may be NULL).  Each cell's eight mirror
 * images (one per octant about the centre, all at its radius) are summed
 * first, then each radius in a fixed order, so results are reproducible.  The
 * first call builds, on the device, the list of octant cells per radius
 * (12 bytes per eight cells, kept; about as much again of scratch during the
 * build).  Errors: MP_ERR_ARG (odd extents, NULL), MP_ERR_NOMEM. */
int mp_average(mp_ctx *ctx, const double *phi, double *avg, double *count);

/* Lateral Average onto a uniform base state (Sec. 3.1, the constant
 * Delta r = Delta x / 5 spacing of spherical stars before the irregular base
 * state): the radius averages of mp_average, then quadratic interpolation
 * onto r_j = (j + 1/2) dr, j < n1d, about the node in the middle of the box:
 * the parabola through the reached radius (one some cell centre lies at)
 * nearest r_j and the reached radii just below and above it (shifted inward
 * at the first and last reached radius); the first and last averages are held
 * below the smallest and beyond the largest reached radius.  avg: device
 * array of n1d doubles.  Errors: MP_ERR_ARG (odd extents, NULL, n1d < 1,
 * dr <= 0), MP_ERR_NOMEM (first call). */
int mp_average_uniform(mp_ctx *ctx, const double *phi, int n1d, double dr, double *avg);

/* Full velocity of the velocity split (Appendix A): U = U~ + w0 e_r on the
 * MAC faces, in place on (ux, uy, uz) (face layouts above) holding U~ (e.g.
 * after mp_mac_project_split).  After an MP_PLANAR mapping e_r = e_z and the
 * base-state edges are the z faces: z face k (the low face of cell k,
 * 0 < k < nz) gains w0[k]; ne = nz + 1, re unused (may be NULL); z must be a
 * Neumann axis (MP_ERR_STATE otherwise).  After a spherical mapping every
 * face gains w0(r_f) e_r . n_f: r_f the distance of the face centre from the
 * star centre (the mapping's centre; the middle node for the irregular base
 * state), e_r . n_f the component of the unit radius vector along the face's
 * axis (0 at r_f = 0), w0(r) linear between the ne edges re (device array,
 * increasing; mp_base_radii or r_e = e dr), held outside them.  Wall faces are
 * left unchanged.  w0: device array of ne doubles (mp_w0).  Returns without
 * waiting.  Errors: MP_ERR_ARG (NULL, ne), MP_ERR_STATE (no mapping). */
int mp_add_w0(mp_ctx *ctx, const double *w0, const double *re, long long ne, double *ux, double *uy, double *uz);

/* ---- one-dimensional base state (Sec. 3.2 modules, Appendix A) ----------
 * Arrays are device arrays of doubles owned by the caller; each call is a
 * multi-block scan on the context's stream (tiles of 4096 values: tile
 * totals, their prefix, every tile again from it) and returns without
 * waiting unless it reports a scalar.  Sums run in a fixed association
 * (reproducible).  Beyond about 2.8 million values a call may allocate a
 * scratch buffer of 24 bytes per 4096 values the first time (MP_ERR_NOMEM).  */

/* Centres rc (mp_radius_count entries) and edges re (one more) of the
 * irregular base state (Sec. 3.1): rc[m] = h sqrt(0.75 + 2m), re[m] =
 * h sqrt(2m - 1/4) (the radius map at m - 1/2; re[0] = 0).
 * MP_ERR_ARG: NULL, or odd extents. */
int mp_base_radii(mp_ctx *ctx, double *rc, double *re);

/* Enforce HSE (Sec. 3.2): p0 from rho0 on n base-state centres rc by the
 * hydrostatic condition dp0/dr = -rho0 g of Sec. 2 (g >= 0, the magnitude of
 * a gravity pointing to -e_r), trapezoidal across each pair of centres with
 * the non-uniform Delta r_{j+1/2} = rc[j+1] - rc[j]:
 *   p0[0] = p0_base,  p0[j] = p0[j-1] - (rc[j] - rc[j-1]) g_edge[j] (rho0[j-1] + rho0[j]) / 2,
 * g_edge: n + 1 values on the edges (g_edge[j] between centres j-1 and j).
 * From the first centre with rho0 <= rho_cutoff outward p0 keeps its value
 * there.  cutoff_index (host, may be NULL): that centre, or n; when given the
 * call waits for it.  MP_ERR_ARG: NULL arrays, n < 1, non-finite p0_base. */
int mp_enforce_hse(mp_ctx *ctx, long long n, const double *rc, const double *rho0, const double *g_edge,
                   double p0_base, double rho_cutoff, double *p0, long long *cutoff_index);

/* Allocation-free Enforce HSE, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the computation of mp_enforce_hse (same kernels, same bits),
 * without a context.  Its scan scratch is a static device array of the
 * library (about 96 KiB per device, held until the process ends): n is at
 * most 16777216 centres (MP_ERR_ARG beyond, before any device work).  The
 * call allocates nothing: no hipMalloc, hipFree or allocating routine; the
 * first call on a device looks the array's address up with that device
 * current.  Every call on a device shares that device's array, and every
 * scratch value a call reads it writes first; calls that overlap on one
 * device (other streams, other threads) race and must be ordered by the
 * caller.
 * stream: hipStream_t of the launches (NULL = null stream), on the current
 *   device; returns without waiting.
 * rc, rho0 (n), g_edge (n + 1), p0 (n, out): device arrays as in
 *   mp_enforce_hse.  cutoff_index: DEVICE pointer to one long long receiving
 *   the first centre with rho0 <= rho_cutoff (n if none), or NULL.
 * Errors: MP_ERR_ARG (NULL arrays, n < 1 or too large, non-finite p0_base),
 * MP_ERR_DEVICE (no current device, a failed launch); mp_last_error(NULL)
 * gives the text. */
int mp_enforce_hse_noalloc(void *stream, long long n, const double *rc, const double *rho0, const double *g_edge,
                           double p0_base, double rho_cutoff, double *p0, long long *cutoff_index);

/* beta0 from its definition (Sec. 2), beta0 = rho0(0) exp(int dp0 / (Gamma1 p0)),
 * on n centres: beta0[0] = rho0_centre and across each pair of centres the
 * integral is ln(p0[j] / p0[j-1]) / ((gamma1[j-1] + gamma1[j]) / 2) (exact
 * for a constant Gamma1).  Waits for a validity check: MP_ERR_NONFINITE if
 * any p0 or gamma1 is non-positive or non-finite; MP_ERR_ARG: NULL, n < 1,
 * rho0_centre <= 0. */
int mp_beta0_from_p0(mp_ctx *ctx, long long n, double rho0_centre, const double *p0, const double *gamma1,
                     double *beta0);

/* Base-state velocity w0 of the velocity split (Appendix A): integrates
 * div(beta0 w0 e_r) = beta0 (sbar - psi) outward from w0 = 0 at the bottom
 * wall (MP_PLANAR) or the centre of the star (the spherical geometries):
 *   F[0] = 0, F[j+1] = F[j] + beta0[j] (sbar[j] - psi[j]) V[j],
 *   V[j] = re[j+1] - re[j] (planar) or (re[j+1]^3 - re[j]^3) / 3 (spherical),
 *   w0[e] = F[e] / (A[e] beta0_e[e]),  A = 1 (planar) or re[e]^2,
 * beta0_e linear in r between the neighbouring centres rc (extrapolated from
 * the last two at the outer edge).  psi = (dp0/dt) / (Gamma1 p0) per centre,
 * or NULL for 0.  rc, beta0, sbar, psi: n; re, w0: n + 1.
 * MP_ERR_ARG: bad geometry, NULL arrays, n < 1. */
int mp_w0(mp_ctx *ctx, int geometry, long long n, const double *rc, const double *re, const double *beta0,
          const double *sbar, const double *psi, double *w0);

/* Switch the per-launch timing of the finest-level smoother (mp_config
 * kernel_timing) on or off for the following calls; it records a start and
 * end timestamp with each of those launches.  Errors: MP_ERR_ARG, MP_ERR_DEVICE. */
int mp_set_kernel_timing(mp_ctx *ctx, int on);

/* y = M x with the context's FP64 level-0 coefficients. */
int mp_apply(mp_ctx *ctx, const double *x, double *y);

/* Face-coefficient gradient of L = <w, phi>: g_f = (G lam)_f (G phi)_f, where
 * lam = mp_solve(w) and phi = mp_solve(rhs); walls 0.  Face layouts above. */
int mp_coef_grad(mp_ctx *ctx, const double *lam, const double *phi, double *gx, double *gy, double *gz);

/* Release a context and its device memory; NULL is accepted. */
int mp_free(mp_ctx *ctx);

/* Text of the last failure on ctx (never NULL; "" if none).  With ctx NULL:
 * the last failure of a context-free call (mp_enforce_hse_noalloc) on the
 * calling thread. */
const char *mp_last_error(const mp_ctx *ctx);

/* Library version string. */
const char *mp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MPROJ_H */
