/*
 * mproj_oracle.c -- plain FP64 CPU reference for the MAC-projection solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle the GPU library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it; the product path never does.  It shares no source,
 * header, table or helper with the HIP library.
 *
 * What it computes (Fan, Nonaka, Almgren, Harpole, Zingale, "MAESTROeX: A
 * Massively Parallel Low Mach Number Astrophysical Solver"):
 *
 *  - fill (Sec. 3.1): the 1D base state beta0 mapped onto the Cartesian cells,
 *    by direct injection in planar geometry and by interpolation in the radius
 *    r = |x - centre| in spherical geometry (linear or quadratic, on the
 *    uniform radial grid r_j = (j + 1/2) dr), or, for the irregular base state,
 *    by the index m of the radius h sqrt(0.75 + 2m) of each cell centre;
 *  - the lateral Average (Sec. 3.1 and the Average module of Sec. 3.2) over
 *    those irregular radii, onto a uniform radial base state (quadratic
 *    interpolation of the radius averages), or over the planes of a planar
 *    atmosphere; the source S - Sbar of the velocity-split constraint of
 *    Appendix A, and the full velocity U = U~ + w0 e_r on the faces;
 *  - the one-dimensional base state: centres and edges of the irregular radii,
 *    Enforce HSE (p0 from rho0), beta0 from its definition in Sec. 2, and the
 *    base-state velocity w0 of the velocity split (Appendix A);
 *  - the MAC projection of Sec. 3.2 Steps 3 and 7 (the constraints div1/div2,
 *    i.e. the velocity constraint of Sec. 2 with the dp0/dt term folded into
 *    S) and Appendix A: find phi with
 *        div((beta0/rho) grad phi) = div(beta0 U) - beta0 S,
 *    then U <- U - (beta0/rho)/beta0 grad phi, so div(beta0 U) = beta0 S.
 *
 * Discretisation (cell-centred finite volume on a uniform grid of spacing h):
 *    (G phi)_f = (phi_R - phi_L)/h                 cell -> face
 *    (D F)_i   = sum_d (F_{i+1/2 e_d} - F_{i-1/2 e_d})/h   face -> cell
 *    M phi     = D (C (G phi)),   C = diag(face coefficients c_f)
 *  with c_f the harmonic mean of the cell values beta0/rho on the two sides,
 *  beta0 on a face the arithmetic mean of the two cells, periodic faces
 *  wrapping, and Neumann boundary faces being walls (c_f = 0, U_f = 0).
 *  The right-hand side is made mean-zero and the solution is the unique
 *  mean-zero phi.
 *
 * The solver is a geometric multigrid V-cycle iteration (red-black Gauss-Seidel,
 * 8-cell average restriction, 4-face average coefficient restriction,
 * piecewise-constant prolongation, conjugate gradients on the coarsest grid),
 * iterated until ||rhs - M phi||_2 / ||rhs||_2 <= tol.  Only the converged
 * answer matters; it is the definition above, reached iteratively.
 *
 * Layouts (C order, x fastest):  cells [nz][ny][nx];  x faces [nz][ny][nx+bx];
 * y faces [nz][ny+by][nx]; z faces [nz+bz][ny][nx]; b* = 0 periodic (n faces,
 * face i is the low face of cell i) or 1 Neumann (n+1 faces, 0 and n walls).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nx, ny, nz;
    double h;
    int bx, by, bz; /* 0 periodic, 1 Neumann */
} grid_t;

static grid_t mkgrid(int nx, int ny, int nz, double h, int bx, int by, int bz)
{
    grid_t g = {nx, ny, nz, h, bx, by, bz};
    return g;
}

static long ncell(const grid_t *g) { return (long)g->nx * g->ny * g->nz; }
static long cell(const grid_t *g, int i, int j, int k) { return ((long)k * g->ny + j) * g->nx + i; }
static long xface(const grid_t *g, int f, int j, int k) { return ((long)k * g->ny + j) * (g->nx + g->bx) + f; }
static long yface(const grid_t *g, int i, int f, int k) { return ((long)k * (g->ny + g->by) + f) * g->nx + i; }
static long zface(const grid_t *g, int i, int j, int f) { return ((long)f * g->ny + j) * g->nx + i; }
static long nxface(const grid_t *g) { return (long)g->nz * g->ny * (g->nx + g->bx); }
static long nyface(const grid_t *g) { return (long)g->nz * (g->ny + g->by) * g->nx; }
static long nzface(const grid_t *g) { return (long)(g->nz + g->bz) * g->ny * g->nx; }

/* Cells on the two sides of face f along an axis of n cells.  Returns 0 for a
 * Neumann wall (no cell on one side). */
static int face_sides(int f, int n, int b, int *L, int *R)
{
    if (b) {
        if (f == 0 || f == n) return 0;
        *L = f - 1;
        *R = f;
        return 1;
    }
    *L = (f + n - 1) % n;
    *R = f % n;
    return 1;
}

/* Index of the high face of cell i along an axis of n cells. */
static int high_face(int i, int n, int b) { return b ? i + 1 : (i + 1) % n; }

/* ---------------------------------------------------------------------- */
/* fill: base state -> cells (Sec. 3.1)                                    */
/* ---------------------------------------------------------------------- */

/* Distance from the centre of cell (i,j,k) to `center`. */
static double cell_radius(const grid_t *g, const double *center, int i, int j, int k)
{
    double x = (i + 0.5) * g->h - center[0];
    double y = (j + 0.5) * g->h - center[1];
    double z = (k + 0.5) * g->h - center[2];
    return sqrt(x * x + y * y + z * z);
}

/* Linear interpolation of a table given at r_j = (j + 1/2) dr; the end values
 * are held beyond the first and last table points. */
static double radial_lookup(const double *tab, int n1d, double dr, double r)
{
    double t = r / dr - 0.5;
    if (t <= 0.0) return tab[0];
    if (t >= (double)(n1d - 1)) return tab[n1d - 1];
    int j = (int)floor(t);
    double w = t - j;
    return (1.0 - w) * tab[j] + w * tab[j + 1];
}

/* Quadratic interpolation of the same table: the Lagrange parabola through
 * the three table points around the nearest one (the stencil kept inside the
 * table), end values held beyond the first and last table points. */
static double radial_quadratic(const double *tab, int n1d, double dr, double r)
{
    double t = r / dr - 0.5;
    if (t <= 0.0) return tab[0];
    if (t >= (double)(n1d - 1)) return tab[n1d - 1];
    int j = (int)floor(t + 0.5);
    if (j < 1) j = 1;
    if (j > n1d - 2) j = n1d - 2;
    double s = t - j;
    return tab[j - 1] * (0.5 * s * (s - 1.0)) + tab[j] * (1.0 - s * s) + tab[j + 1] * (0.5 * s * (s + 1.0));
}

/* Irregular radial base state (Sec. 3.1): with the star centre on the grid
 * node in the middle of the box (all extents even), the centre of cell
 * (i,j,k) lies at distance h sqrt(0.75 + 2m) for the integer
 *     m = ((2i+1-nx)^2 + (2j+1-ny)^2 + (2k+1-nz)^2 - 3) / 8,
 * since the three offsets from the centre are odd multiples of h/2.  Returns
 * -1 when an extent is odd. */
static long radius_index(const grid_t *g, int i, int j, int k)
{
    long a = 2L * i + 1 - g->nx, b = 2L * j + 1 - g->ny, c = 2L * k + 1 - g->nz;
    return (a * a + b * b + c * c - 3) / 8;
}

/* Number of radii of the irregular base state (m = 0 .. m_max), or 0 when an
 * extent is odd (no grid node at the centre of the box). */
long or_radius_count(int nx, int ny, int nz)
{
    if (nx % 2 || ny % 2 || nz % 2) return 0;
    grid_t g = mkgrid(nx, ny, nz, 1.0, 0, 0, 0);
    return radius_index(&g, 0, 0, 0) + 1;
}

/* m of every cell (layout of a cell array). */
int or_radius_index(int nx, int ny, int nz, long *m)
{
    if (nx % 2 || ny % 2 || nz % 2) return 1;
    grid_t g = mkgrid(nx, ny, nz, 1.0, 0, 0, 0);
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) m[cell(&g, i, j, k)] = radius_index(&g, i, j, k);
    return 0;
}

/* Lateral average over the irregular radii (Sec. 3.1, the Average module of
 * Sec. 3.2): the sum of phi over all cells whose centres lie at radius r_m,
 * divided by the number of those cells.  Radii no cell centre reaches get
 * count 0 and average 0.  Cells are summed in memory order. */
int or_average_irregular(int nx, int ny, int nz, const double *phi, long nm, double *avg, double *count)
{
    if (nx % 2 || ny % 2 || nz % 2 || nm != or_radius_count(nx, ny, nz)) return 1;
    grid_t g = mkgrid(nx, ny, nz, 1.0, 0, 0, 0);
    double *sum = (double *)calloc((size_t)nm, sizeof(double));
    for (long m = 0; m < nm; m++) count[m] = 0.0;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long m = radius_index(&g, i, j, k);
                sum[m] += phi[cell(&g, i, j, k)];
                count[m] += 1.0;
            }
    for (long m = 0; m < nm; m++) avg[m] = count[m] > 0.0 ? sum[m] / count[m] : 0.0;
    free(sum);
    return 0;
}

/* Lateral average in planar geometry (Sec. 3.1): the arithmetic mean of the
 * cells of each horizontal plane k (base-state cells align with the planes). */
void or_plane_average(int nx, int ny, int nz, const double *phi, double *avg)
{
    grid_t g = mkgrid(nx, ny, nz, 1.0, 0, 0, 0);
    for (int k = 0; k < nz; k++) {
        double s = 0.0;
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) s += phi[cell(&g, i, j, k)];
        avg[k] = s / ((double)nx * ny);
    }
}

/* Source of the velocity-split constraint (Appendix A): the perturbational
 * velocity satisfies div(beta0 U~) = beta0 (S - Sbar), with Sbar the lateral
 * average of S filled back onto the cells.  geometry 0: plane averages
 * (sbar has nz entries); 2: averages over the irregular radii (sbar has one
 * entry per radius).  Writes S - Sbar to s_out.  Returns 1 on a bad geometry. */
int or_split_source(int nx, int ny, int nz, int geometry, const double *S, double *s_out, double *sbar)
{
    grid_t g = mkgrid(nx, ny, nz, 1.0, 0, 0, 0);
    if (geometry == 0) {
        or_plane_average(nx, ny, nz, S, sbar);
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) s_out[cell(&g, i, j, k)] = S[cell(&g, i, j, k)] - sbar[k];
        return 0;
    }
    if (geometry == 2) {
        long nm = or_radius_count(nx, ny, nz);
        if (nm == 0) return 1;
        double *cnt = (double *)malloc(sizeof(double) * (size_t)nm);
        or_average_irregular(nx, ny, nz, S, nm, sbar, cnt);
        free(cnt);
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++)
                    s_out[cell(&g, i, j, k)] = S[cell(&g, i, j, k)] - sbar[radius_index(&g, i, j, k)];
        return 0;
    }
    return 1;
}

/* Lagrange polynomial through the points (x[q], y[q]), q < np (np = 1, 2
 * or 3), evaluated at r. */
static double lagrange(const double *x, const double *y, int np, double r)
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

/* Lateral average onto the uniform base state r_j = (j + 1/2) dr, j < n1d
 * (Sec. 3.1; Delta r = Delta x / 5 before the irregular base state): first
 * the arithmetic average over the cells of each radius h sqrt(0.75 + 2m)
 * (or_average_irregular), then quadratic interpolation of those averages onto
 * r_j.  Only radii that cell centres reach carry data.  The parabola runs
 * through the reached radius nearest r_j and the reached radii just below and
 * above it (shifted inward at the first and last reached radius); below the
 * smallest and beyond the largest reached radius the first and last averages
 * are held.  The centre of the star is the node in the middle of the box.
 * Returns 1 when an extent is odd. */
int or_average_uniform(int nx, int ny, int nz, double h, const double *phi, int n1d, double dr, double *avg)
{
    long nm = or_radius_count(nx, ny, nz);
    if (nm == 0 || n1d < 1 || !(dr > 0.0)) return 1;
    double *a = (double *)malloc(sizeof(double) * (size_t)nm);
    double *cnt = (double *)malloc(sizeof(double) * (size_t)nm);
    double *R = (double *)malloc(sizeof(double) * (size_t)nm);
    double *A = (double *)malloc(sizeof(double) * (size_t)nm);
    or_average_irregular(nx, ny, nz, phi, nm, a, cnt);
    long P = 0; /* the reached radii, in increasing order */
    for (long m = 0; m < nm; m++)
        if (cnt[m] > 0.0) {
            R[P] = h * sqrt(0.75 + 2.0 * (double)m);
            A[P] = a[m];
            P++;
        }
    for (int j = 0; j < n1d; j++) {
        double r = (j + 0.5) * dr;
        if (r <= R[0]) {
            avg[j] = A[0];
        } else if (r >= R[P - 1]) {
            avg[j] = A[P - 1];
        } else {
            long lo = 0, hi = P - 1; /* R[lo] <= r < R[hi] */
            while (hi - lo > 1) {
                long mid = (lo + hi) / 2;
                if (R[mid] <= r)
                    lo = mid;
                else
                    hi = mid;
            }
            long q = (r - R[lo] <= R[hi] - r) ? lo : hi;
            int np = P < 3 ? (int)P : 3;
            long first = q - 1;
            if (first > P - np) first = P - np;
            if (first < 0) first = 0;
            avg[j] = lagrange(R + first, A + first, np, r);
        }
    }
    free(a);
    free(cnt);
    free(R);
    free(A);
    return 0;
}

/* Velocity-split source for a uniform spherical base state (Appendix A with
 * the uniform Average of Sec. 3.1): Sbar on the table r_j = (j + 1/2) dr
 * (or_average_uniform of S), filled back onto the cells with the fill of the
 * mapping (geometry 1: linear, 3: quadratic, about the middle node of the
 * box), s_out = S - Sbar(cell).  sbar: n1d entries.  Returns 1 on a bad
 * geometry or odd extents. */
int or_split_source_uniform(int nx, int ny, int nz, double h, int geometry, int n1d, double dr, const double *S,
                            double *s_out, double *sbar)
{
    if (geometry != 1 && geometry != 3) return 1;
    if (or_average_uniform(nx, ny, nz, h, S, n1d, dr, sbar)) return 1;
    grid_t g = mkgrid(nx, ny, nz, h, 0, 0, 0);
    double c[3] = {0.5 * nx * h, 0.5 * ny * h, 0.5 * nz * h};
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double r = cell_radius(&g, c, i, j, k);
                double sb = geometry == 1 ? radial_lookup(sbar, n1d, dr, r) : radial_quadratic(sbar, n1d, dr, r);
                s_out[cell(&g, i, j, k)] = S[cell(&g, i, j, k)] - sb;
            }
    return 0;
}

/* w0 at radius r from its values on the base-state edges re[0..ne) (sorted
 * increasing): linear in r between the two edges around r, the last value
 * held beyond the last edge. */
static double w0_at(const double *w0, const double *re, long ne, double r)
{
    if (r >= re[ne - 1]) return w0[ne - 1];
    if (r <= re[0]) return w0[0];
    long lo = 0, hi = ne - 1; /* re[lo] <= r < re[hi] */
    while (hi - lo > 1) {
        long mid = (lo + hi) / 2;
        if (re[mid] <= r)
            lo = mid;
        else
            hi = mid;
    }
    double t = (r - re[lo]) / (re[hi] - re[lo]);
    return w0[lo] + t * (w0[hi] - w0[lo]);
}

/* Full velocity of the velocity split (Appendix A): U = U~ + w0 e_r on the MAC
 * faces, in place on (ux, uy, uz) holding U~.  geometry 0 (planar, e_r = e_z,
 * base-state edges on the z faces): z face k (the low face of cell k) gains
 * w0[k]; x and y faces are unchanged; ne = nz + 1 and re is not used.
 * Spherical geometries: every face gains w0(r_f) (e_r . n_f), r_f the distance
 * of the face centre from `center`, e_r . n_f the component of (x_f -
 * center) / r_f along the face's axis (0 at r_f = 0), w0(r) linear between
 * the edges re[0..ne).  Wall faces (Neumann axes) are left unchanged.
 * Returns 1 on bad arguments (planar with a periodic z axis or ne != nz + 1). */
int or_add_w0(int nx, int ny, int nz, double h, int bx, int by, int bz, int geometry, const double *w0,
              const double *re, long ne, const double *center, double *ux, double *uy, double *uz)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    if (geometry == 0) {
        if (!bz || ne != nz + 1) return 1;
        for (int f = 1; f < nz; f++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) uz[zface(&g, i, j, f)] += w0[f];
        return 0;
    }
    if (ne < 1) return 1;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int f = 0; f < nx + bx; f++) {
                if (bx && (f == 0 || f == nx)) continue;
                double x = f * h - center[0], y = (j + 0.5) * h - center[1], z = (k + 0.5) * h - center[2];
                double r = sqrt(x * x + y * y + z * z);
                if (r > 0.0) ux[xface(&g, f, j, k)] += w0_at(w0, re, ne, r) * (x / r);
            }
    for (int k = 0; k < nz; k++)
        for (int f = 0; f < ny + by; f++)
            for (int i = 0; i < nx; i++) {
                if (by && (f == 0 || f == ny)) continue;
                double x = (i + 0.5) * h - center[0], y = f * h - center[1], z = (k + 0.5) * h - center[2];
                double r = sqrt(x * x + y * y + z * z);
                if (r > 0.0) uy[yface(&g, i, f, k)] += w0_at(w0, re, ne, r) * (y / r);
            }
    for (int f = 0; f < nz + bz; f++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                if (bz && (f == 0 || f == nz)) continue;
                double x = (i + 0.5) * h - center[0], y = (j + 0.5) * h - center[1], z = f * h - center[2];
                double r = sqrt(x * x + y * y + z * z);
                if (r > 0.0) uz[zface(&g, i, j, f)] += w0_at(w0, re, ne, r) * (z / r);
            }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* One-dimensional base state (Sec. 3.2 modules, Appendix A)               */
/* ---------------------------------------------------------------------- */

/* Centres and edges of the irregular base state (Sec. 3.1): centre m at
 * h sqrt(0.75 + 2m); edge m (the inner edge of radius m) at the same map at
 * m - 1/2, h sqrt(2m - 0.25), i.e. the r^2 midway between the neighbouring
 * centres, with edge 0 at the centre of the star.  rc: nm, re: nm + 1. */
void or_irregular_radii(long nm, double h, double *rc, double *re)
{
    for (long m = 0; m < nm; m++) rc[m] = h * sqrt(0.75 + 2.0 * (double)m);
    re[0] = 0.0;
    for (long m = 1; m <= nm; m++) re[m] = h * sqrt(2.0 * (double)m - 0.25);
}

/* Enforce HSE (Sec. 3.2): p0 from rho0 by integrating dp0/dr = -rho0 g (the
 * hydrostatic condition of Sec. 2, g >= 0 the magnitude of the gravity that
 * points to -e_r) outward from p0[0] = p0_base with the trapezoidal rule
 * across each pair of centres, Delta r_{j+1/2} = rc[j+1] - rc[j] (not
 * constant on the irregular base state):
 *     p0[j+1] = p0[j] - (rc[j+1] - rc[j]) g_edge[j+1] (rho0[j] + rho0[j+1]) / 2,
 * g_edge[j] the gravity at the edge between centres j-1 and j (n + 1
 * entries, edges as in or_irregular_radii).  From the first centre whose
 * density is at or below rho_cutoff outward, p0 stays at its value there.
 * Returns that centre's index (n when no density is that low). */
long or_enforce_hse(long n, const double *rc, const double *rho0, const double *g_edge, double p0_base,
                    double rho_cutoff, double *p0)
{
    long jc = n;
    for (long j = 0; j < n; j++)
        if (rho0[j] <= rho_cutoff) {
            jc = j;
            break;
        }
    p0[0] = p0_base;
    for (long j = 1; j < n; j++) {
        if (j > jc) {
            p0[j] = p0[j - 1];
            continue;
        }
        p0[j] = p0[j - 1] - (rc[j] - rc[j - 1]) * g_edge[j] * 0.5 * (rho0[j - 1] + rho0[j]);
    }
    return jc;
}

/* beta0 by its definition (Sec. 2): beta0(r) = rho0(0) exp(int_0^r dp0/(Gamma1 p0)).
 * Across each pair of centres the integral of dp0/(Gamma1 p0) is taken with
 * Gamma1 at its mean over the pair, which makes it exact for a constant
 * Gamma1: ln(p0[j+1]/p0[j]) / ((Gamma1[j] + Gamma1[j+1]) / 2). */
void or_beta0_from_p0(long n, double rho0_centre, const double *p0, const double *gamma1, double *beta0)
{
    double acc = 0.0;
    beta0[0] = rho0_centre;
    for (long j = 1; j < n; j++) {
        acc += log(p0[j] / p0[j - 1]) / (0.5 * (gamma1[j - 1] + gamma1[j]));
        beta0[j] = rho0_centre * exp(acc);
    }
}

/* Base-state velocity w0 of the velocity split (Appendix A):
 *     div(beta0 w0 e_r) = beta0 (Sbar - psi),  psi = dp0/dt / (Gamma1 p0),
 * integrated outward from w0 = 0 at the bottom wall (planar, geometry 0) or
 * at the centre of the star (spherical, geometry 1) in flux form over the
 * base-state cells [re[j], re[j+1]]:
 *     F[j+1] = F[j] + beta0[j] (sbar[j] - psi[j]) V[j],
 *     planar:    F = beta0_e w0,        V[j] = re[j+1] - re[j],
 *     spherical: F = re^2 beta0_e w0,   V[j] = (re[j+1]^3 - re[j]^3) / 3,
 * with beta0 on an edge interpolated linearly in r between the centres rc on
 * either side, and extrapolated linearly from the last two centres on the
 * outer edge (one centre: its value).  w0 has n + 1 edge values; psi may be
 * NULL (0).  Returns 1 for a bad geometry. */
static double edge_beta0(long n, const double *rc, const double *re, const double *beta0, long e)
{
    if (n == 1) return beta0[0];
    long a = e < n ? e - 1 : n - 2, b = a + 1;
    double t = (re[e] - rc[a]) / (rc[b] - rc[a]);
    return beta0[a] + t * (beta0[b] - beta0[a]);
}

int or_w0(int geometry, long n, const double *rc, const double *re, const double *beta0, const double *sbar,
          const double *psi, double *w0)
{
    if (geometry != 0 && geometry != 1) return 1;
    double F = 0.0;
    w0[0] = 0.0;
    for (long j = 0; j < n; j++) {
        double V = geometry == 0 ? re[j + 1] - re[j]
                                 : (re[j + 1] * re[j + 1] * re[j + 1] - re[j] * re[j] * re[j]) / 3.0;
        F += beta0[j] * (sbar[j] - (psi ? psi[j] : 0.0)) * V;
        long e = j + 1;
        double be = edge_beta0(n, rc, re, beta0, e);
        double area = geometry == 0 ? 1.0 : re[e] * re[e];
        w0[e] = F / (area * be);
    }
    return 0;
}

void or_cell_radius(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *center, double *r)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) r[cell(&g, i, j, k)] = cell_radius(&g, center, i, j, k);
}

/* geometry 0: planar, table indexed by the z cell (n1d == nz, direct injection).
 * geometry 1: spherical, table on r_j = (j + 1/2) dr about `center`, linear.
 * geometry 2: spherical irregular base state, table indexed by the radius
 *             index m of each cell (n1d == number of radii; the centre is the
 *             node in the middle of the box; no interpolation).
 * geometry 3: as 1 with quadratic interpolation (uniform dr). */
int or_fill_beta0(int nx, int ny, int nz, double h, int bx, int by, int bz, int geometry, const double *b1d, int n1d,
                  double dr, const double *center, double *beta0_cc)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    if (geometry == 0 && n1d != nz) return 1;
    if (geometry == 1 && (n1d < 2 || !(dr > 0.0))) return 1;
    if (geometry == 3 && (n1d < 3 || !(dr > 0.0))) return 1;
    if (geometry == 2 && (long)n1d != or_radius_count(nx, ny, nz)) return 1;
    if (geometry < 0 || geometry > 3) return 1;
#pragma omp parallel for
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double v;
                if (geometry == 0)
                    v = b1d[k];
                else if (geometry == 1)
                    v = radial_lookup(b1d, n1d, dr, cell_radius(&g, center, i, j, k));
                else if (geometry == 2)
                    v = b1d[radius_index(&g, i, j, k)];
                else
                    v = radial_quadratic(b1d, n1d, dr, cell_radius(&g, center, i, j, k));
                beta0_cc[cell(&g, i, j, k)] = v;
            }
    return 0;
}

/* Face coefficients: harmonic mean of beta0/rho on the two sides; walls 0. */
void or_face_coefs(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *beta0_cc, const double *rho,
                   double *cx, double *cy, double *cz)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    long n = ncell(&g);
    double *c = (double *)malloc(sizeof(double) * n);
    for (long q = 0; q < n; q++) c[q] = beta0_cc[q] / rho[q];
    int L, R;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int f = 0; f < nx + bx; f++) {
                double v = 0.0;
                if (face_sides(f, nx, bx, &L, &R)) {
                    double a = c[cell(&g, L, j, k)], b = c[cell(&g, R, j, k)];
                    v = 2.0 * a * b / (a + b);
                }
                cx[xface(&g, f, j, k)] = v;
            }
    for (int k = 0; k < nz; k++)
        for (int f = 0; f < ny + by; f++)
            for (int i = 0; i < nx; i++) {
                double v = 0.0;
                if (face_sides(f, ny, by, &L, &R)) {
                    double a = c[cell(&g, i, L, k)], b = c[cell(&g, i, R, k)];
                    v = 2.0 * a * b / (a + b);
                }
                cy[yface(&g, i, f, k)] = v;
            }
    for (int f = 0; f < nz + bz; f++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double v = 0.0;
                if (face_sides(f, nz, bz, &L, &R)) {
                    double a = c[cell(&g, i, j, L)], b = c[cell(&g, i, j, R)];
                    v = 2.0 * a * b / (a + b);
                }
                cz[zface(&g, i, j, f)] = v;
            }
    free(c);
}

/* ---------------------------------------------------------------------- */
/* G, D and M = D C G                                                      */
/* ---------------------------------------------------------------------- */

/* (G phi)_f = (phi_R - phi_L)/h on every face with two sides; 0 on walls. */
void or_gradient(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *phi, double *gx, double *gy,
                 double *gz)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    int L, R;
#pragma omp parallel for private(L, R)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int f = 0; f < nx + bx; f++)
                gx[xface(&g, f, j, k)] =
                    face_sides(f, nx, bx, &L, &R) ? (phi[cell(&g, R, j, k)] - phi[cell(&g, L, j, k)]) / h : 0.0;
#pragma omp parallel for private(L, R)
    for (int k = 0; k < nz; k++)
        for (int f = 0; f < ny + by; f++)
            for (int i = 0; i < nx; i++)
                gy[yface(&g, i, f, k)] =
                    face_sides(f, ny, by, &L, &R) ? (phi[cell(&g, i, R, k)] - phi[cell(&g, i, L, k)]) / h : 0.0;
#pragma omp parallel for private(L, R)
    for (int f = 0; f < nz + bz; f++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++)
                gz[zface(&g, i, j, f)] =
                    face_sides(f, nz, bz, &L, &R) ? (phi[cell(&g, i, j, R)] - phi[cell(&g, i, j, L)]) / h : 0.0;
}

/* (D F)_i = sum_d (F_high - F_low)/h; wall faces carry no flux. */
void or_divergence(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *fx, const double *fy,
                   const double *fz, double *out)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
#pragma omp parallel for
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int ih = high_face(i, nx, bx), jh = high_face(j, ny, by), kh = high_face(k, nz, bz);
                double xl = (bx && i == 0) ? 0.0 : fx[xface(&g, i, j, k)];
                double xh = (bx && ih == nx) ? 0.0 : fx[xface(&g, ih, j, k)];
                double yl = (by && j == 0) ? 0.0 : fy[yface(&g, i, j, k)];
                double yh = (by && jh == ny) ? 0.0 : fy[yface(&g, i, jh, k)];
                double zl = (bz && k == 0) ? 0.0 : fz[zface(&g, i, j, k)];
                double zh = (bz && kh == nz) ? 0.0 : fz[zface(&g, i, j, kh)];
                out[cell(&g, i, j, k)] = ((xh - xl) + (yh - yl) + (zh - zl)) / h;
            }
}

static void face_product(long n, const double *a, const double *b, double *out)
{
    for (long q = 0; q < n; q++) out[q] = a[q] * b[q];
}

/* out = M phi = D (C (G phi)), written as the three steps of its definition. */
void or_apply(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *cx, const double *cy,
              const double *cz, const double *phi, double *out)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    long mx = nxface(&g), my = nyface(&g), mz = nzface(&g);
    double *gx = (double *)malloc(sizeof(double) * mx);
    double *gy = (double *)malloc(sizeof(double) * my);
    double *gz = (double *)malloc(sizeof(double) * mz);
    or_gradient(nx, ny, nz, h, bx, by, bz, phi, gx, gy, gz);
    face_product(mx, cx, gx, gx);
    face_product(my, cy, gy, gy);
    face_product(mz, cz, gz, gz);
    or_divergence(nx, ny, nz, h, bx, by, bz, gx, gy, gz, out);
    free(gx);
    free(gy);
    free(gz);
}

/* beta0 on faces (arithmetic mean of the two cells) times U; walls 0. */
static void beta0_flux(const grid_t *g, const double *beta0_cc, const double *ux, const double *uy, const double *uz,
                       double *fx, double *fy, double *fz)
{
    int L, R;
    for (int k = 0; k < g->nz; k++)
        for (int j = 0; j < g->ny; j++)
            for (int f = 0; f < g->nx + g->bx; f++) {
                long q = xface(g, f, j, k);
                fx[q] = face_sides(f, g->nx, g->bx, &L, &R)
                            ? 0.5 * (beta0_cc[cell(g, L, j, k)] + beta0_cc[cell(g, R, j, k)]) * ux[q]
                            : 0.0;
            }
    for (int k = 0; k < g->nz; k++)
        for (int f = 0; f < g->ny + g->by; f++)
            for (int i = 0; i < g->nx; i++) {
                long q = yface(g, i, f, k);
                fy[q] = face_sides(f, g->ny, g->by, &L, &R)
                            ? 0.5 * (beta0_cc[cell(g, i, L, k)] + beta0_cc[cell(g, i, R, k)]) * uy[q]
                            : 0.0;
            }
    for (int f = 0; f < g->nz + g->bz; f++)
        for (int j = 0; j < g->ny; j++)
            for (int i = 0; i < g->nx; i++) {
                long q = zface(g, i, j, f);
                fz[q] = face_sides(f, g->nz, g->bz, &L, &R)
                            ? 0.5 * (beta0_cc[cell(g, i, j, L)] + beta0_cc[cell(g, i, j, R)]) * uz[q]
                            : 0.0;
            }
}

/* out = D(beta0 U). */
void or_beta0_divergence(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *beta0_cc,
                         const double *ux, const double *uy, const double *uz, double *out)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    long mx = nxface(&g), my = nyface(&g), mz = nzface(&g);
    double *fx = (double *)malloc(sizeof(double) * mx);
    double *fy = (double *)malloc(sizeof(double) * my);
    double *fz = (double *)malloc(sizeof(double) * mz);
    beta0_flux(&g, beta0_cc, ux, uy, uz, fx, fy, fz);
    or_divergence(nx, ny, nz, h, bx, by, bz, fx, fy, fz, out);
    free(fx);
    free(fy);
    free(fz);
}

static double plane_ordered_sum(const grid_t *g, const double *a)
{
    /* sum each z plane, then the planes in order: independent of threads */
    double *ps = (double *)malloc(sizeof(double) * g->nz);
    long plane = (long)g->nx * g->ny;
#pragma omp parallel for
    for (int k = 0; k < g->nz; k++) {
        double s = 0.0;
        for (long q = 0; q < plane; q++) s += a[(long)k * plane + q];
        ps[k] = s;
    }
    double s = 0.0;
    for (int k = 0; k < g->nz; k++) s += ps[k];
    free(ps);
    return s;
}

static double plane_ordered_dot(const grid_t *g, const double *a, const double *b)
{
    double *ps = (double *)malloc(sizeof(double) * g->nz);
    long plane = (long)g->nx * g->ny;
#pragma omp parallel for
    for (int k = 0; k < g->nz; k++) {
        double s = 0.0;
        for (long q = 0; q < plane; q++) s += a[(long)k * plane + q] * b[(long)k * plane + q];
        ps[k] = s;
    }
    double s = 0.0;
    for (int k = 0; k < g->nz; k++) s += ps[k];
    free(ps);
    return s;
}

double or_sum(int nx, int ny, int nz, const double *a)
{
    grid_t g = mkgrid(nx, ny, nz, 1.0, 0, 0, 0);
    return plane_ordered_sum(&g, a);
}

double or_dot(int nx, int ny, int nz, const double *a, const double *b)
{
    grid_t g = mkgrid(nx, ny, nz, 1.0, 0, 0, 0);
    return plane_ordered_dot(&g, a, b);
}

/* MAC right-hand side: rhs = D(beta0 U) - beta0 S, then its mean removed.
 * Returns the removed mean. */
double or_mac_rhs(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *beta0_cc, const double *ux,
                  const double *uy, const double *uz, const double *S, double *rhs)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    long n = ncell(&g);
    or_beta0_divergence(nx, ny, nz, h, bx, by, bz, beta0_cc, ux, uy, uz, rhs);
    for (long q = 0; q < n; q++) rhs[q] -= beta0_cc[q] * S[q];
    double m = plane_ordered_sum(&g, rhs) / (double)n;
    for (long q = 0; q < n; q++) rhs[q] -= m;
    return m;
}

/* U <- U - (c_f / beta0_f) (G phi)_f on every face with two sides. */
void or_velocity_correct(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *cx, const double *cy,
                         const double *cz, const double *beta0_cc, const double *phi, double *ux, double *uy,
                         double *uz)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    int L, R;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int f = 0; f < nx + bx; f++)
                if (face_sides(f, nx, bx, &L, &R)) {
                    long a = cell(&g, L, j, k), b = cell(&g, R, j, k), q = xface(&g, f, j, k);
                    ux[q] -= cx[q] / (0.5 * (beta0_cc[a] + beta0_cc[b])) * (phi[b] - phi[a]) / h;
                }
    for (int k = 0; k < nz; k++)
        for (int f = 0; f < ny + by; f++)
            for (int i = 0; i < nx; i++)
                if (face_sides(f, ny, by, &L, &R)) {
                    long a = cell(&g, i, L, k), b = cell(&g, i, R, k), q = yface(&g, i, f, k);
                    uy[q] -= cy[q] / (0.5 * (beta0_cc[a] + beta0_cc[b])) * (phi[b] - phi[a]) / h;
                }
    for (int f = 0; f < nz + bz; f++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++)
                if (face_sides(f, nz, bz, &L, &R)) {
                    long a = cell(&g, i, j, L), b = cell(&g, i, j, R), q = zface(&g, i, j, f);
                    uz[q] -= cz[q] / (0.5 * (beta0_cc[a] + beta0_cc[b])) * (phi[b] - phi[a]) / h;
                }
}

/* dL/dc_f = (G lam)_f (G phi)_f for L = <w, phi>, where lam solves M lam = w
 * (mean-zero).  Walls get 0. */
void or_coef_grad(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *lam, const double *phi,
                  double *gx, double *gy, double *gz)
{
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    long mx = nxface(&g), my = nyface(&g), mz = nzface(&g);
    double *px = (double *)malloc(sizeof(double) * mx);
    double *py = (double *)malloc(sizeof(double) * my);
    double *pz = (double *)malloc(sizeof(double) * mz);
    or_gradient(nx, ny, nz, h, bx, by, bz, lam, gx, gy, gz);
    or_gradient(nx, ny, nz, h, bx, by, bz, phi, px, py, pz);
    face_product(mx, gx, px, gx);
    face_product(my, gy, py, gy);
    face_product(mz, gz, pz, gz);
    free(px);
    free(py);
    free(pz);
}

/* ---------------------------------------------------------------------- */
/* Multigrid                                                               */
/* ---------------------------------------------------------------------- */

typedef struct {
    grid_t g;
    double *cx, *cy, *cz; /* external face layout */
    double *phi, *rhs, *res;
} level_t;

#define MAX_LEVELS 24

/* One Gauss-Seidel update of cell (i,j,k) for M phi = rhs:
 *   phi_i = (sum_f c_f phi_nb(f) - h^2 rhs_i) / sum_f c_f. */
static void relax_cell(const level_t *lv, int i, int j, int k)
{
    const grid_t *g = &lv->g;
    int nx = g->nx, ny = g->ny, nz = g->nz;
    double num = 0.0, den = 0.0, c;
    int n_;
    /* x low / high */
    if (!(g->bx && i == 0)) {
        c = lv->cx[xface(g, i, j, k)];
        n_ = (i + nx - 1) % nx;
        num += c * lv->phi[cell(g, n_, j, k)];
        den += c;
    }
    if (!(g->bx && i == nx - 1)) {
        c = lv->cx[xface(g, high_face(i, nx, g->bx), j, k)];
        n_ = (i + 1) % nx;
        num += c * lv->phi[cell(g, n_, j, k)];
        den += c;
    }
    if (!(g->by && j == 0)) {
        c = lv->cy[yface(g, i, j, k)];
        n_ = (j + ny - 1) % ny;
        num += c * lv->phi[cell(g, i, n_, k)];
        den += c;
    }
    if (!(g->by && j == ny - 1)) {
        c = lv->cy[yface(g, i, high_face(j, ny, g->by), k)];
        n_ = (j + 1) % ny;
        num += c * lv->phi[cell(g, i, n_, k)];
        den += c;
    }
    if (!(g->bz && k == 0)) {
        c = lv->cz[zface(g, i, j, k)];
        n_ = (k + nz - 1) % nz;
        num += c * lv->phi[cell(g, i, j, n_)];
        den += c;
    }
    if (!(g->bz && k == nz - 1)) {
        c = lv->cz[zface(g, i, j, high_face(k, nz, g->bz))];
        n_ = (k + 1) % nz;
        num += c * lv->phi[cell(g, i, j, n_)];
        den += c;
    }
    long q = cell(g, i, j, k);
    if (den > 0.0) lv->phi[q] = (num - g->h * g->h * lv->rhs[q]) / den;
}

static void rbgs(level_t *lv)
{
    const grid_t *g = &lv->g;
    /* With an odd periodic extent, cells of one colour can touch across the
     * wrap; then the sweep runs serially so the result does not depend on the
     * thread count. */
    int par = !((g->bx == 0 && g->nx % 2) || (g->by == 0 && g->ny % 2) || (g->bz == 0 && g->nz % 2));
    for (int colour = 0; colour < 2; colour++) {
#pragma omp parallel for if (par)
        for (int k = 0; k < g->nz; k++)
            for (int j = 0; j < g->ny; j++)
                for (int i = (j + k + colour) & 1; i < g->nx; i += 2) relax_cell(lv, i, j, k);
    }
}

static void residual(level_t *lv)
{
    const grid_t *g = &lv->g;
    long n = ncell(g);
    or_apply(g->nx, g->ny, g->nz, g->h, g->bx, g->by, g->bz, lv->cx, lv->cy, lv->cz, lv->phi, lv->res);
    for (long q = 0; q < n; q++) lv->res[q] = lv->rhs[q] - lv->res[q];
}

/* coarse face = mean of the 4 fine faces that cover it */
static void restrict_coefs(const level_t *f, level_t *c)
{
    const grid_t *gf = &f->g, *gc = &c->g;
    for (int K = 0; K < gc->nz; K++)
        for (int J = 0; J < gc->ny; J++)
            for (int F = 0; F < gc->nx + gc->bx; F++) {
                double s = 0.0;
                for (int b = 0; b < 2; b++)
                    for (int a = 0; a < 2; a++) s += f->cx[xface(gf, 2 * F, 2 * J + a, 2 * K + b)];
                c->cx[xface(gc, F, J, K)] = 0.25 * s;
            }
    for (int K = 0; K < gc->nz; K++)
        for (int F = 0; F < gc->ny + gc->by; F++)
            for (int I = 0; I < gc->nx; I++) {
                double s = 0.0;
                for (int b = 0; b < 2; b++)
                    for (int a = 0; a < 2; a++) s += f->cy[yface(gf, 2 * I + a, 2 * F, 2 * K + b)];
                c->cy[yface(gc, I, F, K)] = 0.25 * s;
            }
    for (int F = 0; F < gc->nz + gc->bz; F++)
        for (int J = 0; J < gc->ny; J++)
            for (int I = 0; I < gc->nx; I++) {
                double s = 0.0;
                for (int b = 0; b < 2; b++)
                    for (int a = 0; a < 2; a++) s += f->cz[zface(gf, 2 * I + a, 2 * J + b, 2 * F)];
                c->cz[zface(gc, I, J, F)] = 0.25 * s;
            }
}

/* coarse rhs = mean of the 8 fine residuals */
static void restrict_residual(const level_t *f, level_t *c)
{
    const grid_t *gf = &f->g, *gc = &c->g;
#pragma omp parallel for
    for (int K = 0; K < gc->nz; K++)
        for (int J = 0; J < gc->ny; J++)
            for (int I = 0; I < gc->nx; I++) {
                double s = 0.0;
                for (int c_ = 0; c_ < 2; c_++)
                    for (int b = 0; b < 2; b++)
                        for (int a = 0; a < 2; a++) s += f->res[cell(gf, 2 * I + a, 2 * J + b, 2 * K + c_)];
                c->rhs[cell(gc, I, J, K)] = 0.125 * s;
            }
}

/* fine phi += coarse phi of the parent cell */
static void prolong_add(level_t *f, const level_t *c)
{
    const grid_t *gf = &f->g, *gc = &c->g;
#pragma omp parallel for
    for (int k = 0; k < gf->nz; k++)
        for (int j = 0; j < gf->ny; j++)
            for (int i = 0; i < gf->nx; i++) f->phi[cell(gf, i, j, k)] += c->phi[cell(gc, i / 2, j / 2, k / 2)];
}

static void remove_mean(const grid_t *g, double *a)
{
    long n = ncell(g);
    double m = plane_ordered_sum(g, a) / (double)n;
    for (long q = 0; q < n; q++) a[q] -= m;
}

/* Conjugate gradients on A = -M (symmetric, positive on mean-zero vectors)
 * for the coarsest grid; rhs is made mean-zero first. */
static void bottom_cg(level_t *lv)
{
    const grid_t *g = &lv->g;
    long n = ncell(g);
    double *r = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *Ap = (double *)malloc(sizeof(double) * n);
    remove_mean(g, lv->rhs);
    for (long q = 0; q < n; q++) {
        lv->phi[q] = 0.0;
        r[q] = -lv->rhs[q]; /* A x = -rhs */
        p[q] = r[q];
    }
    double rr = plane_ordered_dot(g, r, r), rr0 = rr;
    long maxit = 20 * n + 100;
    for (long it = 0; it < maxit && rr > 1e-30 * rr0 && rr > 0.0; it++) {
        or_apply(g->nx, g->ny, g->nz, g->h, g->bx, g->by, g->bz, lv->cx, lv->cy, lv->cz, p, Ap);
        for (long q = 0; q < n; q++) Ap[q] = -Ap[q];
        double pAp = plane_ordered_dot(g, p, Ap);
        if (!(pAp > 0.0)) break;
        double alpha = rr / pAp;
        for (long q = 0; q < n; q++) {
            lv->phi[q] += alpha * p[q];
            r[q] -= alpha * Ap[q];
        }
        remove_mean(g, r);
        double rr1 = plane_ordered_dot(g, r, r);
        double beta = rr1 / rr;
        rr = rr1;
        for (long q = 0; q < n; q++) p[q] = r[q] + beta * p[q];
    }
    remove_mean(g, lv->phi);
    free(r);
    free(p);
    free(Ap);
}

static void vcycle(level_t *lv, int l, int nlev, int nu1, int nu2)
{
    if (l == nlev - 1) {
        bottom_cg(&lv[l]);
        return;
    }
    for (int s = 0; s < nu1; s++) rbgs(&lv[l]);
    residual(&lv[l]);
    restrict_residual(&lv[l], &lv[l + 1]);
    memset(lv[l + 1].phi, 0, sizeof(double) * ncell(&lv[l + 1].g));
    vcycle(lv, l + 1, nlev, nu1, nu2);
    prolong_add(&lv[l], &lv[l + 1]);
    for (int s = 0; s < nu2; s++) rbgs(&lv[l]);
}

static double norm2(const grid_t *g, const double *a) { return sqrt(plane_ordered_dot(g, a, a)); }

/* Solve M phi = rhs (rhs made mean-zero; phi returned mean-zero).
 * phi is the initial guess on entry.  Returns 0 on convergence, 1 otherwise. */
int or_solve(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *cx, const double *cy,
             const double *cz, const double *rhs, double *phi, double tol, int maxcycles, int nu1, int nu2,
             int *cycles_out, double *relres_out)
{
    level_t lv[MAX_LEVELS];
    int nlev = 0;
    grid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    for (;;) {
        level_t *L = &lv[nlev];
        L->g = g;
        long n = ncell(&g);
        L->phi = (double *)calloc(n, sizeof(double));
        L->rhs = (double *)malloc(sizeof(double) * n);
        L->res = (double *)malloc(sizeof(double) * n);
        if (nlev == 0) {
            L->cx = (double *)cx;
            L->cy = (double *)cy;
            L->cz = (double *)cz;
        } else {
            L->cx = (double *)malloc(sizeof(double) * nxface(&g));
            L->cy = (double *)malloc(sizeof(double) * nyface(&g));
            L->cz = (double *)malloc(sizeof(double) * nzface(&g));
            restrict_coefs(&lv[nlev - 1], L);
        }
        nlev++;
        int can = g.nx % 2 == 0 && g.ny % 2 == 0 && g.nz % 2 == 0 && g.nx >= 8 && g.ny >= 8 && g.nz >= 8;
        if (!can || nlev == MAX_LEVELS) break;
        g = mkgrid(g.nx / 2, g.ny / 2, g.nz / 2, 2.0 * g.h, bx, by, bz);
    }
    long n = ncell(&lv[0].g);
    memcpy(lv[0].rhs, rhs, sizeof(double) * n);
    remove_mean(&lv[0].g, lv[0].rhs);
    memcpy(lv[0].phi, phi, sizeof(double) * n);
    double nb = norm2(&lv[0].g, lv[0].rhs);
    int cyc = 0;
    double rel = 0.0;
    int status = 0;
    if (nb > 0.0) {
        for (;;) {
            residual(&lv[0]);
            rel = norm2(&lv[0].g, lv[0].res) / nb;
            if (rel <= tol) break;
            if (cyc >= maxcycles) {
                status = 1;
                break;
            }
            vcycle(lv, 0, nlev, nu1, nu2);
            cyc++;
        }
    } else {
        memset(lv[0].phi, 0, sizeof(double) * n);
    }
    remove_mean(&lv[0].g, lv[0].phi);
    memcpy(phi, lv[0].phi, sizeof(double) * n);
    for (int l = 0; l < nlev; l++) {
        free(lv[l].phi);
        free(lv[l].rhs);
        free(lv[l].res);
        if (l > 0) {
            free(lv[l].cx);
            free(lv[l].cy);
            free(lv[l].cz);
        }
    }
    if (cycles_out) *cycles_out = cyc;
    if (relres_out) *relres_out = rel;
    return status;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
