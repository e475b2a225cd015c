/*
 * nodal_oracle.c -- plain FP64 CPU reference for the nodal projection.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle the GPU library's nodal
 * projection is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product path never does.  It
 * shares no source, header, table or helper with the HIP library.
 *
 * What it computes (Fan et al., "MAESTROeX", Sec. 3.2 Step 11 and Appendix A):
 * the cell-centred velocity U is projected onto the constraint
 * div(beta0 U) = beta0 S with a scalar phi that lives on the grid NODES:
 *        div((beta0/rho) grad phi) = div(beta0 U) - beta0 S,
 *        U <- U - (1/beta0)(beta0/rho) grad phi.
 * The paper gives only this structure (node-based phi, cell-centred U, its own
 * divergence and gradient, an approximate projection) and defers the
 * discretisation to an earlier paper; the reading taken here is the standard
 * one for a node-based projection, trilinear finite elements on the cells:
 *
 *  - phi_h = sum_n phi_n N_n, N_n the trilinear hat function of node n;
 *  - sigma = beta0/rho is constant on each cell;
 *  - operator:   (M phi)_n = -(1/h^3) sum_e sigma_e  int_e grad phi_h . grad N_n
 *  - divergence: (D V)_n   = -(1/h^3) sum_e V_e . int_e grad N_n   (V cell-constant)
 *  - gradient:   (G phi)_e =  (1/h^3) int_e grad phi_h            (cell average)
 *  - load:       (L f)_n   =  (1/h^3) sum_e f_e int_e N_n          (f cell-constant)
 *  so that D = -G^T and M is symmetric and negative semi-definite with the
 *  constants as null space.  The right-hand side is R = D(beta0 U) - L(beta0 S - m),
 *  m the mean of beta0 S over the cells (the part of the source no velocity on
 *  a closed or periodic domain can carry), the solution the phi of M phi = R
 *  whose arithmetic mean over the nodes is zero, and the corrected velocity
 *  U_e - (sigma_e / beta0_e) (G phi)_e.  Since D sigma G is not M, the
 *  corrected velocity meets the constraint only approximately (an approximate
 *  projection), to second order in h for smooth data.
 *
 * Element integrals on a cell of side h from the 1D linear basis
 * n_0(t) = 1 - t, n_1(t) = t on [0, 1]:
 *     int n_a' n_b' = +-1 / h,   int n_a n_b = h/3 or h/6,
 *     int n_a'      = -+1,       int n_a     = h/2,
 * and the 3D integrals as their tensor products.
 *
 * Nodes: along an axis of n cells there are n nodes when it is periodic (node n
 * is node 0) and n + 1 when it has Neumann walls (nodes 0 and n on the walls;
 * their equations take only the cells inside, the natural boundary condition).
 * Layout C order [nkz][nky][nkx], x fastest.  Cell arrays [nz][ny][nx].
 *
 * The solver is a plain geometric multigrid V-cycle iteration (Gauss-Seidel in
 * 8 colours by node parity, residual restriction by the transpose of trilinear
 * interpolation scaled by 1/8, trilinear prolongation, cell sigma coarsened as
 * the mean of its 8 children, conjugate gradients on the coarsest grid),
 * iterated until ||R - M phi||_2 / ||R||_2 <= tol.  Only the converged answer
 * matters; it is the definition above, reached iteratively.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nx, ny, nz; /* cells */
    double h;
    int bx, by, bz; /* 0 periodic, 1 Neumann */
    int mx, my, mz; /* nodes */
} ngrid_t;

static ngrid_t mkgrid(int nx, int ny, int nz, double h, int bx, int by, int bz)
{
    ngrid_t g = {nx, ny, nz, h, bx, by, bz, nx + bx, ny + by, nz + bz};
    return g;
}

static long nnode(const ngrid_t *g) { return (long)g->mx * g->my * g->mz; }
static long ncell(const ngrid_t *g) { return (long)g->nx * g->ny * g->nz; }
static long node(const ngrid_t *g, int i, int j, int k) { return ((long)k * g->my + j) * g->mx + i; }
static long cell(const ngrid_t *g, int i, int j, int k) { return ((long)k * g->ny + j) * g->nx + i; }

/* Cell index along an axis of n cells for the cell at offset o from a node
 * (o = -1: the cell below the node, o = 0: above); -1 if there is none. */
static int cell_at(int node_i, int o, int n, int b)
{
    int c = node_i + o;
    if (b) return (c < 0 || c >= n) ? -1 : c;
    return (c + n) % n;
}

/* Node index along an axis for corner a (0 low, 1 high) of cell c. */
static int corner_node(int c, int a, int n, int b) { return b ? c + a : (c + a) % n; }

/* ---------------------------------------------------------------------- */
/* Element integrals                                                       */
/* ---------------------------------------------------------------------- */

/* 1D, reference interval, for the linear basis n_0 = 1 - t, n_1 = t. */
static double stiff1(int a, int b) { return a == b ? 1.0 : -1.0; }            /* int n_a' n_b' dt */
static double mass1(int a, int b) { return a == b ? 1.0 / 3.0 : 1.0 / 6.0; } /* int n_a n_b dt */
static double dint1(int a) { return a ? 1.0 : -1.0; }                        /* int n_a' dt */
static double int1(int a) { (void)a; return 0.5; }                           /* int n_a dt */

/* Corner A = (ax, ay, az) bits of a cell. */
static int bit(int A, int d) { return (A >> d) & 1; }

/* int_e grad N_A . grad N_B over a cell of side h. */
static double elem_stiff(int A, int B, double h)
{
    double s = 0.0;
    for (int d = 0; d < 3; d++) {
        double t = stiff1(bit(A, d), bit(B, d)) / h;
        for (int e = 0; e < 3; e++)
            if (e != d) t *= mass1(bit(A, e), bit(B, e)) * h;
        s += t;
    }
    return s;
}

/* int_e dN_A/dx_d over a cell of side h. */
static double elem_grad(int A, int d, double h)
{
    double t = dint1(bit(A, d));
    for (int e = 0; e < 3; e++)
        if (e != d) t *= int1(bit(A, e)) * h;
    return t;
}

/* int_e N_A over a cell of side h. */
static double elem_int(int A, double h)
{
    double t = 1.0;
    for (int e = 0; e < 3; e++) t *= int1(bit(A, e)) * h;
    return t;
}

/* The (up to 8) cells around node (i,j,k): cell index and the node's corner
 * in each.  Returns the count. */
static int cells_of_node(const ngrid_t *g, int i, int j, int k, long *cq, int *corner, int ci[][3])
{
    int cnt = 0;
    for (int oz = -1; oz <= 0; oz++)
        for (int oy = -1; oy <= 0; oy++)
            for (int ox = -1; ox <= 0; ox++) {
                int a = cell_at(i, ox, g->nx, g->bx), b = cell_at(j, oy, g->ny, g->by),
                    c = cell_at(k, oz, g->nz, g->bz);
                if (a < 0 || b < 0 || c < 0) continue;
                cq[cnt] = cell(g, a, b, c);
                corner[cnt] = (ox ? 1 : 0) | (oy ? 2 : 0) | (oz ? 4 : 0);
                ci[cnt][0] = a;
                ci[cnt][1] = b;
                ci[cnt][2] = c;
                cnt++;
            }
    return cnt;
}

static long corner_of_cell(const ngrid_t *g, const int c[3], int B)
{
    return node(g, corner_node(c[0], bit(B, 0), g->nx, g->bx), corner_node(c[1], bit(B, 1), g->ny, g->by),
                corner_node(c[2], bit(B, 2), g->nz, g->bz));
}

/* ---------------------------------------------------------------------- */
/* Operators                                                               */
/* ---------------------------------------------------------------------- */

/* Diagonal and off-diagonal parts of -h^3 (M phi)_n = sum_e sigma_e sum_B K_AB phi_B. */
static void row_parts(const ngrid_t *g, const double *sigma, const double *phi, int i, int j, int k, double *diag,
                      double *off)
{
    long cq[8];
    int corner[8], ci[8][3];
    int cnt = cells_of_node(g, i, j, k, cq, corner, ci);
    double dg = 0.0, of = 0.0;
    for (int e = 0; e < cnt; e++) {
        int A = corner[e];
        for (int B = 0; B < 8; B++) {
            double kab = sigma[cq[e]] * elem_stiff(A, B, g->h);
            if (B == A)
                dg += kab;
            else
                of += kab * phi[corner_of_cell(g, ci[e], B)];
        }
    }
    *diag = dg;
    *off = of;
}

void nd_apply(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *sigma, const double *phi,
              double *out)
{
    ngrid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    double h3 = h * h * h;
#pragma omp parallel for
    for (int k = 0; k < g.mz; k++)
        for (int j = 0; j < g.my; j++)
            for (int i = 0; i < g.mx; i++) {
                double dg, of;
                row_parts(&g, sigma, phi, i, j, k, &dg, &of);
                out[node(&g, i, j, k)] = -(dg * phi[node(&g, i, j, k)] + of) / h3;
            }
}

void nd_divergence(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *vx, const double *vy,
                   const double *vz, double *out)
{
    ngrid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    double h3 = h * h * h;
#pragma omp parallel for
    for (int k = 0; k < g.mz; k++)
        for (int j = 0; j < g.my; j++)
            for (int i = 0; i < g.mx; i++) {
                long cq[8];
                int corner[8], ci[8][3];
                int cnt = cells_of_node(&g, i, j, k, cq, corner, ci);
                double s = 0.0;
                for (int e = 0; e < cnt; e++) {
                    int A = corner[e];
                    s += vx[cq[e]] * elem_grad(A, 0, h) + vy[cq[e]] * elem_grad(A, 1, h) +
                         vz[cq[e]] * elem_grad(A, 2, h);
                }
                out[node(&g, i, j, k)] = -s / h3;
            }
}

void nd_gradient(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *phi, double *gx,
                 double *gy, double *gz)
{
    ngrid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    double h3 = h * h * h;
#pragma omp parallel for
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int c[3] = {i, j, k};
                double s[3] = {0.0, 0.0, 0.0};
                for (int B = 0; B < 8; B++) {
                    double p = phi[corner_of_cell(&g, c, B)];
                    for (int d = 0; d < 3; d++) s[d] += p * elem_grad(B, d, h);
                }
                long q = cell(&g, i, j, k);
                gx[q] = s[0] / h3;
                gy[q] = s[1] / h3;
                gz[q] = s[2] / h3;
            }
}

void nd_load(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *f, double *out)
{
    ngrid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    double h3 = h * h * h;
#pragma omp parallel for
    for (int k = 0; k < g.mz; k++)
        for (int j = 0; j < g.my; j++)
            for (int i = 0; i < g.mx; i++) {
                long cq[8];
                int corner[8], ci[8][3];
                int cnt = cells_of_node(&g, i, j, k, cq, corner, ci);
                double s = 0.0;
                for (int e = 0; e < cnt; e++) s += f[cq[e]] * elem_int(corner[e], h);
                out[node(&g, i, j, k)] = s / h3;
            }
}

/* Sums in a fixed order (each z plane in memory order, then the planes in
 * order) so results do not depend on the thread count. */
static double ordered_sum(long nplane, long per, const double *a, const double *b)
{
    double *ps = (double *)malloc(sizeof(double) * (nplane > 0 ? nplane : 1));
#pragma omp parallel for
    for (long p = 0; p < nplane; p++) {
        double s = 0.0;
        for (long q = p * per; q < (p + 1) * per; q++) s += b ? a[q] * b[q] : a[q];
        ps[p] = s;
    }
    double s = 0.0;
    for (long p = 0; p < nplane; p++) s += ps[p];
    free(ps);
    return s;
}

static double node_dot(const ngrid_t *g, const double *a, const double *b)
{
    return ordered_sum(g->mz, (long)g->mx * g->my, a, b);
}

double nd_node_dot(int nx, int ny, int nz, int bx, int by, int bz, const double *a, const double *b)
{
    ngrid_t g = mkgrid(nx, ny, nz, 1.0, bx, by, bz);
    return node_dot(&g, a, b);
}

/* R = D(beta0 U) - L(beta0 S - m), m = mean of beta0 S over the cells.
 * Returns m. */
double nd_rhs(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *beta0, const double *ux,
              const double *uy, const double *uz, const double *S, double *out)
{
    ngrid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    long n = ncell(&g), nn = nnode(&g);
    double *vx = (double *)malloc(sizeof(double) * n), *vy = (double *)malloc(sizeof(double) * n);
    double *vz = (double *)malloc(sizeof(double) * n), *src = (double *)malloc(sizeof(double) * n);
    double *ld = (double *)malloc(sizeof(double) * nn);
    for (long q = 0; q < n; q++) {
        vx[q] = beta0[q] * ux[q];
        vy[q] = beta0[q] * uy[q];
        vz[q] = beta0[q] * uz[q];
        src[q] = beta0[q] * S[q];
    }
    double m = ordered_sum(nz, (long)nx * ny, src, NULL) / (double)n;
    for (long q = 0; q < n; q++) src[q] -= m;
    nd_divergence(nx, ny, nz, h, bx, by, bz, vx, vy, vz, out);
    nd_load(nx, ny, nz, h, bx, by, bz, src, ld);
    for (long q = 0; q < nn; q++) out[q] -= ld[q];
    free(vx);
    free(vy);
    free(vz);
    free(src);
    free(ld);
    return m;
}

/* U_e <- U_e - (sigma_e / beta0_e) (G phi)_e. */
void nd_correct(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *sigma, const double *beta0,
                const double *phi, double *ux, double *uy, double *uz)
{
    ngrid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    long n = ncell(&g);
    double *gx = (double *)malloc(sizeof(double) * n), *gy = (double *)malloc(sizeof(double) * n);
    double *gz = (double *)malloc(sizeof(double) * n);
    nd_gradient(nx, ny, nz, h, bx, by, bz, phi, gx, gy, gz);
    for (long q = 0; q < n; q++) {
        double w = sigma[q] / beta0[q];
        ux[q] -= w * gx[q];
        uy[q] -= w * gy[q];
        uz[q] -= w * gz[q];
    }
    free(gx);
    free(gy);
    free(gz);
}

/* ---------------------------------------------------------------------- */
/* Grid transfers                                                          */
/* ---------------------------------------------------------------------- */

/* Trilinear interpolation along one axis (fine spacing h, coarse 2h): fine
 * node i takes coarse node i/2 with weight 1 when i is even, and the two
 * coarse nodes (i-1)/2, (i+1)/2 with weight 1/2 each when i is odd.  nf is the
 * number of fine cells on the axis.  Returns the number of coarse nodes. */
static int coarse_nodes_of(int i, int nf, int b, int *I, double *w)
{
    int nc_nodes = nf / 2 + b;
    if (i % 2 == 0) {
        I[0] = i / 2;
        w[0] = 1.0;
        return 1;
    }
    I[0] = (i - 1) / 2;
    I[1] = b ? (i + 1) / 2 : ((i + 1) / 2) % nc_nodes;
    w[0] = w[1] = 0.5;
    return 2;
}

/* The transpose: the fine nodes 2I - 1, 2I, 2I + 1 that take coarse node I,
 * with their weights (wrapped when periodic, dropped beyond a wall). */
static int fine_nodes_of(int I, int nf, int b, int *i, double *w)
{
    int cnt = 0;
    for (int d = -1; d <= 1; d++) {
        int f = 2 * I + d;
        if (b) {
            if (f < 0 || f > nf) continue;
        } else {
            f = (f + nf) % nf;
        }
        i[cnt] = f;
        w[cnt] = d == 0 ? 1.0 : 0.5;
        cnt++;
    }
    return cnt;
}

/* phi_f += P e_c (trilinear interpolation of the coarse nodes). */
void nd_prolong_add(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *ec, double *phi)
{
    ngrid_t f = mkgrid(nx, ny, nz, h, bx, by, bz);
    ngrid_t c = mkgrid(nx / 2, ny / 2, nz / 2, 2 * h, bx, by, bz);
#pragma omp parallel for
    for (int k = 0; k < f.mz; k++)
        for (int j = 0; j < f.my; j++)
            for (int i = 0; i < f.mx; i++) {
                int I[2], J[2], K[2];
                double wi[2], wj[2], wk[2];
                int ni = coarse_nodes_of(i, nx, bx, I, wi), nj = coarse_nodes_of(j, ny, by, J, wj),
                    nk = coarse_nodes_of(k, nz, bz, K, wk);
                double s = 0.0;
                for (int c3 = 0; c3 < nk; c3++)
                    for (int c2 = 0; c2 < nj; c2++)
                        for (int c1 = 0; c1 < ni; c1++)
                            s += wi[c1] * wj[c2] * wk[c3] * ec[node(&c, I[c1], J[c2], K[c3])];
                phi[node(&f, i, j, k)] += s;
            }
}

/* r_c = (1/8) P^T r_f. */
void nd_restrict(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *rf, double *rc)
{
    ngrid_t f = mkgrid(nx, ny, nz, h, bx, by, bz);
    ngrid_t c = mkgrid(nx / 2, ny / 2, nz / 2, 2 * h, bx, by, bz);
#pragma omp parallel for
    for (int K = 0; K < c.mz; K++)
        for (int J = 0; J < c.my; J++)
            for (int I = 0; I < c.mx; I++) {
                int fi[3], fj[3], fk[3];
                double wi[3], wj[3], wk[3];
                int ni = fine_nodes_of(I, nx, bx, fi, wi), nj = fine_nodes_of(J, ny, by, fj, wj),
                    nk = fine_nodes_of(K, nz, bz, fk, wk);
                double s = 0.0;
                for (int c3 = 0; c3 < nk; c3++)
                    for (int c2 = 0; c2 < nj; c2++)
                        for (int c1 = 0; c1 < ni; c1++)
                            s += wi[c1] * wj[c2] * wk[c3] * rf[node(&f, fi[c1], fj[c2], fk[c3])];
                rc[node(&c, I, J, K)] = 0.125 * s;
            }
}

/* Coarse cell sigma = mean of its 8 children. */
void nd_sigma_coarsen(int nx, int ny, int nz, const double *sf, double *sc)
{
    int NX = nx / 2, NY = ny / 2, NZ = nz / 2;
    for (int K = 0; K < NZ; K++)
        for (int J = 0; J < NY; J++)
            for (int I = 0; I < NX; I++) {
                double s = 0.0;
                for (int c = 0; c < 2; c++)
                    for (int b = 0; b < 2; b++)
                        for (int a = 0; a < 2; a++)
                            s += sf[((long)(2 * K + c) * ny + 2 * J + b) * nx + 2 * I + a];
                sc[((long)K * NY + J) * NX + I] = 0.125 * s;
            }
}

/* ---------------------------------------------------------------------- */
/* Multigrid                                                               */
/* ---------------------------------------------------------------------- */

typedef struct {
    ngrid_t g;
    double *sigma, *phi, *rhs, *res;
} nlevel_t;

#define ND_MAX_LEVELS 24

/* Gauss-Seidel on M phi = rhs, nodes in 8 colours by the parity of (i, j, k):
 * two nodes of one colour never share a cell, so a colour updates in any
 * order.  With an odd periodic node count the sweep runs serially. */
static void gs_sweep(nlevel_t *lv)
{
    const ngrid_t *g = &lv->g;
    double h3 = g->h * g->h * g->h;
    int par = !((g->bx == 0 && g->mx % 2) || (g->by == 0 && g->my % 2) || (g->bz == 0 && g->mz % 2));
    for (int col = 0; col < 8; col++) {
        int cx = col & 1, cy = (col >> 1) & 1, cz = (col >> 2) & 1;
#pragma omp parallel for if (par)
        for (int k = cz; k < g->mz; k += 2)
            for (int j = cy; j < g->my; j += 2)
                for (int i = cx; i < g->mx; i += 2) {
                    double dg, of;
                    row_parts(g, lv->sigma, lv->phi, i, j, k, &dg, &of);
                    /* -(dg phi + of) / h^3 = rhs */
                    lv->phi[node(g, i, j, k)] = (-h3 * lv->rhs[node(g, i, j, k)] - of) / dg;
                }
    }
}

static void residual(nlevel_t *lv)
{
    const ngrid_t *g = &lv->g;
    long n = nnode(g);
    nd_apply(g->nx, g->ny, g->nz, g->h, g->bx, g->by, g->bz, lv->sigma, lv->phi, lv->res);
    for (long q = 0; q < n; q++) lv->res[q] = lv->rhs[q] - lv->res[q];
}

static void remove_node_mean(const ngrid_t *g, double *a)
{
    long n = nnode(g);
    double m = ordered_sum(g->mz, (long)g->mx * g->my, a, NULL) / (double)n;
    for (long q = 0; q < n; q++) a[q] -= m;
}

/* Conjugate gradients on -M (symmetric, positive on mean-zero vectors). */
static void bottom_cg(nlevel_t *lv)
{
    const ngrid_t *g = &lv->g;
    long n = nnode(g);
    double *r = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *Ap = (double *)malloc(sizeof(double) * n);
    remove_node_mean(g, lv->rhs);
    for (long q = 0; q < n; q++) {
        lv->phi[q] = 0.0;
        r[q] = -lv->rhs[q];
        p[q] = r[q];
    }
    double rr = node_dot(g, r, r), rr0 = rr;
    long maxit = 20 * n + 100;
    for (long it = 0; it < maxit && rr > 1e-30 * rr0 && rr > 0.0; it++) {
        nd_apply(g->nx, g->ny, g->nz, g->h, g->bx, g->by, g->bz, lv->sigma, p, Ap);
        for (long q = 0; q < n; q++) Ap[q] = -Ap[q];
        double pAp = node_dot(g, p, Ap);
        if (!(pAp > 0.0)) break;
        double alpha = rr / pAp;
        for (long q = 0; q < n; q++) {
            lv->phi[q] += alpha * p[q];
            r[q] -= alpha * Ap[q];
        }
        remove_node_mean(g, r);
        double rr1 = node_dot(g, r, r);
        double beta = rr1 / rr;
        rr = rr1;
        for (long q = 0; q < n; q++) p[q] = r[q] + beta * p[q];
    }
    remove_node_mean(g, lv->phi);
    free(r);
    free(p);
    free(Ap);
}

static void vcycle(nlevel_t *lv, int l, int nlev, int nu1, int nu2)
{
    if (l == nlev - 1) {
        bottom_cg(&lv[l]);
        return;
    }
    const ngrid_t *g = &lv[l].g;
    for (int s = 0; s < nu1; s++) gs_sweep(&lv[l]);
    residual(&lv[l]);
    nd_restrict(g->nx, g->ny, g->nz, g->h, g->bx, g->by, g->bz, lv[l].res, lv[l + 1].rhs);
    memset(lv[l + 1].phi, 0, sizeof(double) * nnode(&lv[l + 1].g));
    vcycle(lv, l + 1, nlev, nu1, nu2);
    nd_prolong_add(g->nx, g->ny, g->nz, g->h, g->bx, g->by, g->bz, lv[l + 1].phi, lv[l].phi);
    for (int s = 0; s < nu2; s++) gs_sweep(&lv[l]);
}

/* Solve M phi = rhs - mean(rhs) (mean over the nodes); phi is the initial
 * guess on entry and is returned with zero node mean.  Returns 0 on
 * convergence, 1 otherwise, 2 for a grid it cannot handle. */
int nd_solve(int nx, int ny, int nz, double h, int bx, int by, int bz, const double *sigma, const double *rhs,
             double *phi, double tol, int maxcycles, int nu1, int nu2, int *cycles_out, double *relres_out)
{
    if (nx < 2 || ny < 2 || nz < 2) return 2;
    nlevel_t lv[ND_MAX_LEVELS];
    int nlev = 0;
    ngrid_t g = mkgrid(nx, ny, nz, h, bx, by, bz);
    for (;;) {
        nlevel_t *L = &lv[nlev];
        L->g = g;
        long n = nnode(&g);
        L->phi = (double *)calloc(n, sizeof(double));
        L->rhs = (double *)malloc(sizeof(double) * n);
        L->res = (double *)malloc(sizeof(double) * n);
        if (nlev == 0) {
            L->sigma = (double *)sigma;
        } else {
            const ngrid_t *f = &lv[nlev - 1].g;
            L->sigma = (double *)malloc(sizeof(double) * ncell(&g));
            nd_sigma_coarsen(f->nx, f->ny, f->nz, lv[nlev - 1].sigma, L->sigma);
        }
        nlev++;
        int can = g.nx % 2 == 0 && g.ny % 2 == 0 && g.nz % 2 == 0 && g.nx >= 8 && g.ny >= 8 && g.nz >= 8;
        if (!can || nlev == ND_MAX_LEVELS) break;
        g = mkgrid(g.nx / 2, g.ny / 2, g.nz / 2, 2.0 * g.h, bx, by, bz);
    }
    long n = nnode(&lv[0].g);
    memcpy(lv[0].rhs, rhs, sizeof(double) * n);
    remove_node_mean(&lv[0].g, lv[0].rhs);
    memcpy(lv[0].phi, phi, sizeof(double) * n);
    double nb = sqrt(node_dot(&lv[0].g, lv[0].rhs, lv[0].rhs));
    int cyc = 0, status = 0;
    double rel = 0.0;
    if (nb > 0.0) {
        for (;;) {
            residual(&lv[0]);
            rel = sqrt(node_dot(&lv[0].g, lv[0].res, lv[0].res)) / nb;
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
    remove_node_mean(&lv[0].g, lv[0].phi);
    memcpy(phi, lv[0].phi, sizeof(double) * n);
    for (int l = 0; l < nlev; l++) {
        free(lv[l].phi);
        free(lv[l].rhs);
        free(lv[l].res);
        if (l > 0) free(lv[l].sigma);
    }
    if (cycles_out) *cycles_out = cyc;
    if (relres_out) *relres_out = rel;
    return status;
}
