/*
 * Driver for the sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host): maps a small stratified planar
 * atmosphere and a small star with each fill, projects a random face
 * velocity, takes the irregular and uniform Averages, the split source, the
 * one-dimensional base state and w0 on the faces, and checks the projection
 * residual.  Any out-of-bounds access or undefined operation aborts the run.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int or_fill_beta0(int, int, int, double, int, int, int, int, const double *, int, double, const double *, double *);
void or_face_coefs(int, int, int, double, int, int, int, const double *, const double *, double *, double *,
                   double *);
double or_mac_rhs(int, int, int, double, int, int, int, const double *, const double *, const double *,
                  const double *, const double *, double *);
int or_solve(int, int, int, double, int, int, int, const double *, const double *, const double *, const double *,
             double *, double, int, int, int, int *, double *);
void or_velocity_correct(int, int, int, double, int, int, int, const double *, const double *, const double *,
                         const double *, const double *, double *, double *, double *);
long or_radius_count(int, int, int);
int or_average_irregular(int, int, int, const double *, long, double *, double *);
int or_average_uniform(int, int, int, double, const double *, int, double, double *);
int or_split_source(int, int, int, int, const double *, double *, double *);
int or_split_source_uniform(int, int, int, double, int, int, double, const double *, double *, double *);
void or_irregular_radii(long, double, double *, double *);
long or_enforce_hse(long, const double *, const double *, const double *, double, double, double *);
void or_beta0_from_p0(long, double, const double *, const double *, double *);
int or_w0(int, long, const double *, const double *, const double *, const double *, const double *, double *);
int or_add_w0(int, int, int, double, int, int, int, int, const double *, const double *, long, const double *,
              double *, double *, double *);

static double urand(unsigned *s)
{
    *s = *s * 1664525u + 1013904223u;
    return (*s >> 8) / 16777216.0 - 0.5;
}

static int project(int n, int geometry, int bx, int by, int bz)
{
    const double h = 1.0 / n;
    const long nc = (long)n * n * n;
    const long nfx = (long)n * n * (n + bx), nfy = (long)n * (n + by) * n, nfz = (long)(n + bz) * n * n;
    int n1d = geometry == 0 ? n : (geometry == 2 ? (int)or_radius_count(n, n, n) : (int)(5 * sqrt(3.0) * n / 2) + 3);
    double dr = h / 5, center[3] = {0.5, 0.5, 0.5};
    double *tab = malloc(sizeof(double) * n1d), *rho = malloc(sizeof(double) * nc), *b0 = malloc(sizeof(double) * nc);
    double *cx = malloc(sizeof(double) * nfx), *cy = malloc(sizeof(double) * nfy), *cz = malloc(sizeof(double) * nfz);
    double *ux = calloc(nfx, sizeof(double)), *uy = calloc(nfy, sizeof(double)), *uz = calloc(nfz, sizeof(double));
    double *S = malloc(sizeof(double) * nc), *rhs = malloc(sizeof(double) * nc), *phi = calloc(nc, sizeof(double));
    unsigned s = 12345u + (unsigned)geometry;
    for (int j = 0; j < n1d; j++) tab[j] = exp(-3.0 * (j + 0.5) / n1d);
    for (long q = 0; q < nc; q++) {
        rho[q] = 1.0 + 0.1 * urand(&s);
        S[q] = 0.01 * urand(&s);
    }
    for (long q = 0; q < nfx; q++) ux[q] = urand(&s);
    for (long q = 0; q < nfy; q++) uy[q] = urand(&s);
    for (long q = 0; q < nfz; q++) uz[q] = urand(&s);
    if (or_fill_beta0(n, n, n, h, bx, by, bz, geometry, tab, n1d, dr, center, b0)) return 1;
    for (long q = 0; q < nc; q++) rho[q] *= b0[q];
    or_face_coefs(n, n, n, h, bx, by, bz, b0, rho, cx, cy, cz);
    double *seff = malloc(sizeof(double) * nc), *sbar = malloc(sizeof(double) * (n1d > n ? n1d : n));
    if (geometry == 0 || geometry == 2) {
        if (or_split_source(n, n, n, geometry, S, seff, sbar)) return 1;
    } else if (or_split_source_uniform(n, n, n, h, geometry, n1d, dr, S, seff, sbar)) {
        return 1;
    }
    or_mac_rhs(n, n, n, h, bx, by, bz, b0, ux, uy, uz, seff, rhs);
    int cycles = 0;
    double rel = 1.0;
    if (or_solve(n, n, n, h, bx, by, bz, cx, cy, cz, rhs, phi, 1e-10, 100, 2, 2, &cycles, &rel)) return 1;
    or_velocity_correct(n, n, n, h, bx, by, bz, cx, cy, cz, b0, phi, ux, uy, uz);
    /* w0 on the faces from the planar or uniform base state */
    long ne = geometry == 0 ? n + 1 : n1d + 1;
    double *rc = malloc(sizeof(double) * (ne - 1)), *re = malloc(sizeof(double) * ne), *w = malloc(sizeof(double) * ne);
    double step = geometry == 0 ? h : dr;
    for (long e = 0; e < ne; e++) re[e] = e * step;
    for (long j = 0; j + 1 < ne; j++) rc[j] = (j + 0.5) * step;
    double *bt = malloc(sizeof(double) * (ne - 1)), *sb = malloc(sizeof(double) * (ne - 1));
    for (long j = 0; j + 1 < ne; j++) {
        bt[j] = exp(-rc[j]);
        sb[j] = cos(rc[j]);
    }
    if (or_w0(geometry == 0 ? 0 : 1, ne - 1, rc, re, bt, sb, NULL, w)) return 1;
    if (geometry != 2 && (geometry != 0 || bz) &&
        or_add_w0(n, n, n, h, bx, by, bz, geometry == 0 ? 0 : 1, w, re, ne, center, ux, uy, uz))
        return 1;
    printf("geometry %d bc %d%d%d: %d cycles, relative residual %.2e\n", geometry, bx, by, bz, cycles, rel);
    int bad = !(rel <= 1e-10);
    free(tab), free(rho), free(b0), free(cx), free(cy), free(cz), free(ux), free(uy), free(uz), free(S), free(rhs);
    free(phi), free(seff), free(sbar), free(rc), free(re), free(w), free(bt), free(sb);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= project(16, 0, 0, 0, 1);
    bad |= project(16, 1, 1, 1, 1);
    bad |= project(12, 3, 1, 1, 1);
    bad |= project(16, 2, 1, 0, 1);
    long nm = or_radius_count(16, 16, 16);
    double *rc = malloc(sizeof(double) * nm), *re = malloc(sizeof(double) * (nm + 1));
    double *rho0 = malloc(sizeof(double) * nm), *g = malloc(sizeof(double) * (nm + 1));
    double *p0 = malloc(sizeof(double) * nm), *gam = malloc(sizeof(double) * nm), *b = malloc(sizeof(double) * nm);
    or_irregular_radii(nm, 1.0 / 16, rc, re);
    for (long m = 0; m < nm; m++) {
        rho0[m] = exp(-rc[m] * 4.0);
        gam[m] = 5.0 / 3.0;
    }
    for (long m = 0; m <= nm; m++) g[m] = 1.0;
    long jc = or_enforce_hse(nm, rc, rho0, g, 1.0, 0.05, p0);
    or_beta0_from_p0(nm, 1.0, p0, gam, b);
    double phi[16 * 16 * 16], avg[2000], cnt[2000];
    unsigned s = 7u;
    for (int q = 0; q < 16 * 16 * 16; q++) phi[q] = urand(&s);
    bad |= or_average_irregular(16, 16, 16, phi, nm, avg, cnt);
    bad |= or_average_uniform(16, 16, 16, 1.0 / 16, phi, 140, 1.0 / 80, avg);
    printf("cutoff %ld of %ld radii; %s\n", jc, nm, bad ? "FAILED" : "ok");
    free(rc), free(re), free(rho0), free(g), free(p0), free(gam), free(b);
    return bad;
}
