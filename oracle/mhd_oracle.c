/*
 * FP64 CPU oracle for forced, isothermal, resistive MHD on a triply periodic grid.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  The solver does not link, call or
 * read anything from here, and nothing here comes from the solver: the two share
 * no code, headers, tables or constants.
 *
 * It is meant to be read against the paper, not to be fast:
 *   - Section 4, Eqs. continuity, navierstokes, magnetic: the right-hand sides for
 *     ln(rho), u and A (diffusive gauge), with B = curl A, j = curl B / mu0, S the
 *     traceless rate-of-strain tensor;
 *   - Section 4, Eqs. forcing, fnorm, feigen: the forcing term;
 *   - Section 2 (numerical methods) and Section 3.1 / Fig. stencils: sixth-order
 *     central finite differences of radius 3 for first, second and mixed
 *     derivatives (the 2-D cut of the stencil is the two axes and both diagonals);
 *   - Section 2: the third-order 2N (low-storage) Runge-Kutta scheme, taken with an
 *     explicit second register w.
 * Every derivative is evaluated by direct indexing with periodic wrap; nothing is
 * fused, blocked or reordered beyond the loops written here.
 *
 * Readings where the paper is silent (listed with reasons in the design notes):
 *   - RK3 coefficients: Williamson (1980) third-order 2N scheme,
 *     alpha = (0, -5/9, -153/128), beta = (1/3, 15/16, 8/15).
 *   - the forcing record of a step is held fixed over that step's three substeps.
 *   - grid points sit at x_i = i * L / N, i = 0 .. N-1.
 *   - mixed derivatives use the diagonal stencil drawn in Fig. stencils.
 *   - j = grad(div A) - lap A, written with the same second-derivative stencils; the
 *     d_i d_i A_i term appears in both parts and cancels identically, so it is left out.
 *   - upwinding of the continuity equation (Section 4, after the fifth-order scheme
 *     it cites): off unless the run's upwind coefficient c is set; then each
 *     advective product u_a d_a ln(rho) is taken with the fifth-order stencil biased
 *     against the flow, which equals the central sixth-order product minus
 *     |u_a| delta6_a ln(rho) / (60 h_a), delta6 the seven-point sixth difference; c
 *     scales that correction (c = 1: full upwinding).
 *   - an optional uniform field B_ext is added to B (zero unless set).
 *   - mu0 = 1, rho = exp(ln rho).
 *
 * State layout: 7 contiguous arrays (ln rho, ux, uy, uz, Ax, Ay, Az), each
 * nx*ny*nz doubles with x fastest: index i + nx*(j + ny*l).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NF 7
#define NTERM 7

typedef struct {
    int32_t nx, ny, nz, pad;
    double lx, ly, lz;
    double cs, nu, eta, dt;
    double bext[3];
    double upwind;       /* upwinding coefficient of the continuity advection (0: off) */
} ora_params;

typedef struct {
    int32_t k[3], pad;   /* integer wave vector, in units of 2 pi / L per axis */
    double e[3];         /* random unit vector (need not be perpendicular to k) */
    double phi;          /* phase */
    double sigma;        /* helicity fraction */
    double f0;           /* amplitude factor */
} ora_forcing;

/* A window onto 7 field arrays.  wrap = 1: indices are periodic in (mx, my, mz).
 * wrap = 0: indices must already lie inside the arrays (a local patch).
 * (ox, oy, oz) is the global grid index of local (0,0,0); the forcing phase uses
 * global indices reduced into [0, N). */
typedef struct {
    const double *f[NF];
    int mx, my, mz;
    int wrap;
    int ox, oy, oz;
} view;

static int imod(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }

static double at(const view *v, int fld, int i, int j, int l)
{
    if (v->wrap) { i = imod(i, v->mx); j = imod(j, v->my); l = imod(l, v->mz); }
    return v->f[fld][(size_t)i + (size_t)v->mx * ((size_t)j + (size_t)v->my * (size_t)l)];
}

/* unit offsets per axis */
static const int AX[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

/* Sixth-order central first derivative along axis a: the 7-point stencil whose
 * weights make it exact for polynomials of degree <= 6 (Taylor expansion). */
static double d1(const view *v, int fld, int i, int j, int l, int a, double h)
{
    static const double c[4] = {0.0, 3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0};
    double s = 0.0;
    for (int m = 1; m <= 3; m++) {
        double fp = at(v, fld, i + m * AX[a][0], j + m * AX[a][1], l + m * AX[a][2]);
        double fm = at(v, fld, i - m * AX[a][0], j - m * AX[a][1], l - m * AX[a][2]);
        s += c[m] * (fp - fm);
    }
    return s / h;
}

/* Seven-point sixth difference along axis a: sum_m (-1)^(m+3) binom(6, m+3) f_m,
 * i.e. h^6 times the sixth derivative to leading order. */
static double d6(const view *v, int fld, int i, int j, int l, int a)
{
    static const double c[4] = {-20.0, 15.0, -6.0, 1.0};
    double s = c[0] * at(v, fld, i, j, l);
    for (int m = 1; m <= 3; m++) {
        double fp = at(v, fld, i + m * AX[a][0], j + m * AX[a][1], l + m * AX[a][2]);
        double fm = at(v, fld, i - m * AX[a][0], j - m * AX[a][1], l - m * AX[a][2]);
        s += c[m] * (fp + fm);
    }
    return s;
}

/* Sixth-order central second derivative along axis a (exact for degree <= 7). */
static const double C2[4] = {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0};

static double d2(const view *v, int fld, int i, int j, int l, int a, double h)
{
    double s = C2[0] * at(v, fld, i, j, l);
    for (int m = 1; m <= 3; m++) {
        double fp = at(v, fld, i + m * AX[a][0], j + m * AX[a][1], l + m * AX[a][2]);
        double fm = at(v, fld, i - m * AX[a][0], j - m * AX[a][1], l - m * AX[a][2]);
        s += C2[m] * (fp + fm);
    }
    return s / (h * h);
}

/* Mixed derivative d_a d_b (a != b) from the two diagonals of the (a, b) plane:
 * the second difference along (h_a, h_b) minus that along (h_a, -h_b) equals
 * 4 h_a h_b f_ab; each second difference is the sixth-order stencil above (its
 * centre weight cancels between the two).  These are the diagonal points of
 * Fig. stencils. */
static double dab(const view *v, int fld, int i, int j, int l, int a, int b,
                  double ha, double hb)
{
    double s = 0.0;
    for (int m = 1; m <= 3; m++) {
        int pa[3] = {m * AX[a][0], m * AX[a][1], m * AX[a][2]};
        int pb[3] = {m * AX[b][0], m * AX[b][1], m * AX[b][2]};
        double fpp = at(v, fld, i + pa[0] + pb[0], j + pa[1] + pb[1], l + pa[2] + pb[2]);
        double fmm = at(v, fld, i - pa[0] - pb[0], j - pa[1] - pb[1], l - pa[2] - pb[2]);
        double fpm = at(v, fld, i + pa[0] - pb[0], j + pa[1] - pb[1], l + pa[2] - pb[2]);
        double fmp = at(v, fld, i - pa[0] + pb[0], j - pa[1] + pb[1], l - pa[2] + pb[2]);
        s += C2[m] * ((fpp + fmm) - (fpm + fmp));
    }
    return s / (4.0 * ha * hb);
}

static void cross3(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* Forcing at global grid index (gi, gj, gl) (Section 4):
 *   f(x) = Re{ N f_k exp[i (k.x + phi)] },  N = f0 cs sqrt(|k| cs / dt),
 *   f_k = [k x (k x e) - i sigma |k| (k x e)] / [sqrt(1+sigma^2) k^2 sqrt(1 - (k.e)^2/k^2)]. */
static void forcing_at(const ora_params *p, const ora_forcing *fr, int gi, int gj, int gl,
                       double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    if (fr->f0 == 0.0) return;
    const double twopi = 6.283185307179586476925286766559;
    double K[3] = {twopi * fr->k[0] / p->lx, twopi * fr->k[1] / p->ly, twopi * fr->k[2] / p->lz};
    double kk = K[0] * K[0] + K[1] * K[1] + K[2] * K[2];
    double kn = sqrt(kk);
    double ke = K[0] * fr->e[0] + K[1] * fr->e[1] + K[2] * fr->e[2];
    double kxe[3], kxkxe[3];
    cross3(K, fr->e, kxe);
    cross3(K, kxe, kxkxe);
    double denom = sqrt(1.0 + fr->sigma * fr->sigma) * kk * sqrt(1.0 - ke * ke / kk);
    double norm = fr->f0 * p->cs * sqrt(kn * p->cs / p->dt);
    double x[3] = {gi * (p->lx / p->nx), gj * (p->ly / p->ny), gl * (p->lz / p->nz)};
    double theta = K[0] * x[0] + K[1] * x[1] + K[2] * x[2] + fr->phi;
    double complex ph = cexp(I * theta);
    for (int c = 0; c < 3; c++) {
        double complex fk = (kxkxe[c] - I * fr->sigma * kn * kxe[c]) / denom;
        out[c] = creal(norm * fk * ph);
    }
}

/* Right-hand side at one cell.  R[7] receives d/dt of (ln rho, u, A).  If tabs is
 * not NULL, tabs[f*NTERM + t] receives |term t| of field f at this cell. */
static void rhs_cell(const view *v, const ora_params *p, const ora_forcing *fr,
                     int i, int j, int l, double R[NF], double *tabs)
{
    const double h[3] = {p->lx / p->nx, p->ly / p->ny, p->lz / p->nz};
    double lnr = at(v, 0, i, j, l);
    double u[3];
    for (int c = 0; c < 3; c++) u[c] = at(v, 1 + c, i, j, l);

    double glnr[3], du[3][3], dA[3][3], d2u[3][3], d2A[3][3];
    for (int a = 0; a < 3; a++) glnr[a] = d1(v, 0, i, j, l, a, h[a]);
    for (int c = 0; c < 3; c++)
        for (int a = 0; a < 3; a++) {
            du[c][a] = d1(v, 1 + c, i, j, l, a, h[a]);   /* d_a u_c */
            dA[c][a] = d1(v, 4 + c, i, j, l, a, h[a]);   /* d_a A_c */
            d2u[c][a] = d2(v, 1 + c, i, j, l, a, h[a]);  /* d_a d_a u_c */
            d2A[c][a] = d2(v, 4 + c, i, j, l, a, h[a]);
        }

    /* grad(div u)_c = sum_b d_c d_b u_b */
    double gdu[3], lapu[3], lapA[3], jc[3];
    for (int c = 0; c < 3; c++) {
        gdu[c] = 0.0;
        for (int b = 0; b < 3; b++) {
            if (b == c) gdu[c] += d2u[c][c];
            else gdu[c] += dab(v, 1 + b, i, j, l, c, b, h[c], h[b]);
        }
        lapu[c] = d2u[c][0] + d2u[c][1] + d2u[c][2];
        lapA[c] = d2A[c][0] + d2A[c][1] + d2A[c][2];
    }
    /* j = curl curl A = grad(div A) - lap A; the d_c d_c A_c parts cancel exactly */
    for (int c = 0; c < 3; c++) {
        jc[c] = 0.0;
        for (int b = 0; b < 3; b++) {
            if (b == c) continue;
            jc[c] += dab(v, 4 + b, i, j, l, c, b, h[c], h[b]) - d2A[c][b];
        }
    }

    double divu = du[0][0] + du[1][1] + du[2][2];
    double B[3] = {dA[2][1] - dA[1][2] + p->bext[0],
                   dA[0][2] - dA[2][0] + p->bext[1],
                   dA[1][0] - dA[0][1] + p->bext[2]};
    double S[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            S[a][b] = 0.5 * (du[a][b] + du[b][a]) - (a == b ? divu / 3.0 : 0.0);

    double jxB[3], uxB[3], F[3];
    cross3(jc, B, jxB);
    cross3(u, B, uxB);
    int gi = imod(i + v->ox, p->nx), gj = imod(j + v->oy, p->ny), gl = imod(l + v->oz, p->nz);
    forcing_at(p, fr, gi, gj, gl, F);
    double rinv = exp(-lnr);
    double cs2 = p->cs * p->cs;

    double ugl = u[0] * glnr[0] + u[1] * glnr[1] + u[2] * glnr[2];
    /* upwinding: -(u_a d_a lnr)_upwind = -u_a d_a lnr + |u_a| delta6_a lnr / (60 h_a) */
    double upw = 0.0;
    if (p->upwind != 0.0) {
        for (int a = 0; a < 3; a++) upw += fabs(u[a]) * d6(v, 0, i, j, l, a) / (60.0 * h[a]);
        upw *= p->upwind;
    }
    R[0] = -ugl - divu + upw;
    if (tabs) {
        for (int t = 0; t < NF * NTERM; t++) tabs[t] = 0.0;
        tabs[0] = fabs(ugl);
        tabs[1] = fabs(du[0][0]) + fabs(du[1][1]) + fabs(du[2][2]);
        tabs[2] = fabs(upw);
    }
    for (int c = 0; c < 3; c++) {
        double adv = u[0] * du[c][0] + u[1] * du[c][1] + u[2] * du[c][2];
        double pres = cs2 * glnr[c];
        double lor = rinv * jxB[c];
        double v_lap = p->nu * lapu[c];
        double v_gd = p->nu * gdu[c] / 3.0;
        double v_s = p->nu * 2.0 * (S[c][0] * glnr[0] + S[c][1] * glnr[1] + S[c][2] * glnr[2]);
        R[1 + c] = -adv - pres + lor + (v_lap + v_gd + v_s) + F[c];
        double ind = uxB[c];
        double dif = p->eta * lapA[c];
        R[4 + c] = ind + dif;
        if (tabs) {
            double *tu = tabs + (1 + c) * NTERM, *ta = tabs + (4 + c) * NTERM;
            tu[0] = fabs(adv); tu[1] = fabs(pres); tu[2] = fabs(lor); tu[3] = fabs(v_lap);
            tu[4] = fabs(v_gd); tu[5] = fabs(v_s); tu[6] = fabs(F[c]);
            ta[0] = fabs(ind); ta[1] = fabs(dif);
        }
    }
}

static const double RK_ALPHA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double RK_BETA[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

static view full_view(const double *state, const ora_params *p)
{
    view v;
    size_t n = (size_t)p->nx * p->ny * p->nz;
    for (int f = 0; f < NF; f++) v.f[f] = state + f * n;
    v.mx = p->nx; v.my = p->ny; v.mz = p->nz;
    v.wrap = 1; v.ox = v.oy = v.oz = 0;
    return v;
}

/* ------------------------------------------------------------------ exports */

void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int ora_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Right-hand side of every cell.  R: 7*ncell doubles.  termmax (7*NTERM, may be
 * NULL) receives the largest |term| over the grid, per field and term. */
int ora_rhs(const double *state, const ora_params *p, const ora_forcing *fr, double *R,
            double *termmax)
{
    view v = full_view(state, p);
    size_t n = (size_t)p->nx * p->ny * p->nz;
    int nz = p->nz;
    double *pm = termmax ? calloc((size_t)nz * NF * NTERM, sizeof(double)) : NULL;
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nz; l++) {
        double tabs[NF * NTERM];
        for (int j = 0; j < p->ny; j++)
            for (int i = 0; i < p->nx; i++) {
                double r[NF];
                rhs_cell(&v, p, fr, i, j, l, r, pm ? tabs : NULL);
                size_t idx = (size_t)i + (size_t)p->nx * ((size_t)j + (size_t)p->ny * l);
                for (int f = 0; f < NF; f++) R[f * n + idx] = r[f];
                if (pm)
                    for (int t = 0; t < NF * NTERM; t++)
                        if (tabs[t] > pm[(size_t)l * NF * NTERM + t]) pm[(size_t)l * NF * NTERM + t] = tabs[t];
            }
    }
    if (pm) {
        for (int t = 0; t < NF * NTERM; t++) termmax[t] = 0.0;
        for (int l = 0; l < nz; l++)
            for (int t = 0; t < NF * NTERM; t++)
                if (pm[(size_t)l * NF * NTERM + t] > termmax[t]) termmax[t] = pm[(size_t)l * NF * NTERM + t];
        free(pm);
    }
    return 0;
}

/* Advance the state in place by nsteps full RK3 steps; step s uses fr[s].
 * tscale (nsteps*7, may be NULL) receives, per step and field, the sum over the
 * field's RHS terms of max|term| (largest over the three substeps). */
int ora_step(double *state, const ora_params *p, const ora_forcing *fr, int64_t nsteps,
             double *tscale)
{
    size_t n = (size_t)p->nx * p->ny * p->nz;
    double *w = calloc(NF * n, sizeof(double));
    double *R = malloc(NF * n * sizeof(double));
    if (!w || !R) { free(w); free(R); return -1; }
    double tm[NF * NTERM];
    for (int64_t s = 0; s < nsteps; s++) {
        double tsum[NF] = {0};
        for (int sub = 0; sub < 3; sub++) {
            ora_rhs(state, p, &fr[s], R, tscale ? tm : NULL);
            if (tscale)
                for (int f = 0; f < NF; f++) {
                    double acc = 0.0;
                    for (int t = 0; t < NTERM; t++) acc += tm[f * NTERM + t];
                    if (acc > tsum[f]) tsum[f] = acc;
                }
#pragma omp parallel for schedule(static)
            for (size_t q = 0; q < NF * n; q++) {
                w[q] = RK_ALPHA[sub] * w[q] + p->dt * R[q];
                state[q] = state[q] + RK_BETA[sub] * w[q];
            }
        }
        if (tscale)
            for (int f = 0; f < NF; f++) tscale[s * NF + f] = tsum[f];
    }
    free(w);
    free(R);
    return 0;
}

/* One full RK3 step evaluated only at the listed cells (global linear indices),
 * from the periodic state, by integrating the dependency cone of each cell: a
 * 19^3 patch around it (radius 9 = 3 substeps x stencil radius 3), substep 1 on
 * the inner 13^3 cells, substep 2 on the inner 7^3, substep 3 on the centre.
 * out: ncells*7 values (field fastest). */
int ora_step_cells(const double *state, const ora_params *p, const ora_forcing *fr,
                   int64_t ncells, const int64_t *cells, double *out)
{
    const int W = 19, C = 9;
    const size_t pn = (size_t)W * W * W;
    view g = full_view(state, p);
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < ncells; q++) {
        double *loc = malloc(NF * pn * sizeof(double));
        double *w = calloc(NF * pn, sizeof(double));
        double *R = malloc(NF * pn * sizeof(double));
        if (!loc || !w || !R) { free(loc); free(w); free(R); fail = 1; continue; }
        int64_t c = cells[q];
        int ci = (int)(c % p->nx), cj = (int)((c / p->nx) % p->ny), cl = (int)(c / ((int64_t)p->nx * p->ny));
        for (int f = 0; f < NF; f++)
            for (int l = 0; l < W; l++)
                for (int j = 0; j < W; j++)
                    for (int i = 0; i < W; i++)
                        loc[f * pn + i + (size_t)W * (j + (size_t)W * l)] =
                            at(&g, f, ci - C + i, cj - C + j, cl - C + l);
        view v;
        for (int f = 0; f < NF; f++) v.f[f] = loc + f * pn;
        v.mx = v.my = v.mz = W; v.wrap = 0;
        v.ox = ci - C; v.oy = cj - C; v.oz = cl - C;
        for (int sub = 0; sub < 3; sub++) {
            int rr = 6 - 3 * sub;
            for (int l = C - rr; l <= C + rr; l++)
                for (int j = C - rr; j <= C + rr; j++)
                    for (int i = C - rr; i <= C + rr; i++) {
                        double r[NF];
                        rhs_cell(&v, p, fr, i, j, l, r, NULL);
                        for (int f = 0; f < NF; f++) R[f * pn + i + (size_t)W * (j + (size_t)W * l)] = r[f];
                    }
            for (int l = C - rr; l <= C + rr; l++)
                for (int j = C - rr; j <= C + rr; j++)
                    for (int i = C - rr; i <= C + rr; i++)
                        for (int f = 0; f < NF; f++) {
                            size_t x = f * pn + i + (size_t)W * (j + (size_t)W * l);
                            w[x] = RK_ALPHA[sub] * w[x] + p->dt * R[x];
                            loc[x] = loc[x] + RK_BETA[sub] * w[x];
                        }
        }
        for (int f = 0; f < NF; f++) out[q * NF + f] = loc[f * pn + C + (size_t)W * (C + (size_t)W * C)];
        free(loc); free(w); free(R);
    }
    return fail ? -1 : 0;
}

/* |term| of every RHS term at the listed cells of the periodic state (the scale
 * that roundoff of one step is measured against).  out: ncells*7*NTERM. */
int ora_terms_cells(const double *state, const ora_params *p, const ora_forcing *fr,
                    int64_t ncells, const int64_t *cells, double *out)
{
    view v = full_view(state, p);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < ncells; q++) {
        int64_t c = cells[q];
        int i = (int)(c % p->nx), j = (int)((c / p->nx) % p->ny), l = (int)(c / ((int64_t)p->nx * p->ny));
        double r[NF];
        rhs_cell(&v, p, fr, i, j, l, r, out + q * NF * NTERM);
    }
    return 0;
}

/* Single derivative operators on one scalar array of dims (nx, ny, nz), spacing
 * (hx, hy, hz).  kind 1: d_a, kind 2: d_a d_a, kind 3: d_a d_b.  wrap = 1:
 * periodic; wrap = 0: cells within 3 of a face are set to NaN. */
int ora_deriv(const double *f, int nx, int ny, int nz, double hx, double hy, double hz,
              int kind, int a, int b, int wrap, double *out)
{
    view v;
    v.f[0] = f;
    for (int q = 1; q < NF; q++) v.f[q] = f;
    v.mx = nx; v.my = ny; v.mz = nz; v.wrap = wrap; v.ox = v.oy = v.oz = 0;
    const double h[3] = {hx, hy, hz};
    for (int l = 0; l < nz; l++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t idx = (size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * l);
                if (!wrap && (i < 3 || j < 3 || l < 3 || i >= nx - 3 || j >= ny - 3 || l >= nz - 3)) {
                    out[idx] = NAN;
                    continue;
                }
                if (kind == 1) out[idx] = d1(&v, 0, i, j, l, a, h[a]);
                else if (kind == 2) out[idx] = d2(&v, 0, i, j, l, a, h[a]);
                else out[idx] = dab(&v, 0, i, j, l, a, b, h[a], h[b]);
            }
    return 0;
}

/* The forcing field of one record on the whole grid: out = 3*ncell (x, y, z). */
int ora_forcing_field(const ora_params *p, const ora_forcing *fr, double *out)
{
    size_t n = (size_t)p->nx * p->ny * p->nz;
    for (int l = 0; l < p->nz; l++)
        for (int j = 0; j < p->ny; j++)
            for (int i = 0; i < p->nx; i++) {
                double F[3];
                forcing_at(p, fr, i, j, l, F);
                size_t idx = (size_t)i + (size_t)p->nx * ((size_t)j + (size_t)p->ny * l);
                for (int c = 0; c < 3; c++) out[c * n + idx] = F[c];
            }
    return 0;
}

/* Neumaier-compensated accumulator */
typedef struct { double s, c; } csum;
static void cadd(csum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double cval(const csum *a) { return a->s + a->c; }

/* Global diagnostics of a state (Section 4 and the time series of Section 2):
 * out[0] E_M = <|B|^2>/2        out[1] E_K = <rho |u|^2>/2
 * out[2] u_rms = sqrt<|u|^2>    out[3] B_rms = sqrt<|B|^2>
 * out[4] max |u|                out[5] <ln rho>
 * out[6..8] <B>                 out[9] number of cells with a non-finite field value
 * B = curl A (+ B_ext) with the same first-derivative stencil as the RHS.
 * Sums are compensated per z-plane and the plane sums combined in plane order. */
#define ND 8
int ora_diag(const double *state, const ora_params *p, double *out)
{
    view v = full_view(state, p);
    const double h[3] = {p->lx / p->nx, p->ly / p->ny, p->lz / p->nz};
    int nz = p->nz;
    csum *ps = calloc((size_t)nz * ND, sizeof(csum));
    double *pmax = calloc((size_t)nz, sizeof(double));
    double *pnf = calloc((size_t)nz, sizeof(double));
    if (!ps || !pmax || !pnf) { free(ps); free(pmax); free(pnf); return -1; }
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nz; l++) {
        csum *a = ps + (size_t)l * ND;
        for (int j = 0; j < p->ny; j++)
            for (int i = 0; i < p->nx; i++) {
                double lnr = at(&v, 0, i, j, l);
                double u[3] = {at(&v, 1, i, j, l), at(&v, 2, i, j, l), at(&v, 3, i, j, l)};
                int bad = 0;
                for (int f = 0; f < NF; f++) if (!isfinite(at(&v, f, i, j, l))) bad = 1;
                double dA[3][3];
                for (int c = 0; c < 3; c++)
                    for (int b = 0; b < 3; b++) dA[c][b] = d1(&v, 4 + c, i, j, l, b, h[b]);
                double B[3] = {dA[2][1] - dA[1][2] + p->bext[0],
                               dA[0][2] - dA[2][0] + p->bext[1],
                               dA[1][0] - dA[0][1] + p->bext[2]};
                double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                double b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
                cadd(&a[0], b2);
                cadd(&a[1], u2);
                cadd(&a[2], exp(lnr) * u2);
                cadd(&a[3], lnr);
                cadd(&a[4], B[0]);
                cadd(&a[5], B[1]);
                cadd(&a[6], B[2]);
                if (u2 > pmax[l]) pmax[l] = u2;
                if (bad) pnf[l] += 1.0;
            }
    }
    csum tot[ND];
    memset(tot, 0, sizeof tot);
    double umax2 = 0.0, nf = 0.0;
    for (int l = 0; l < nz; l++) {
        for (int q = 0; q < ND; q++) cadd(&tot[q], cval(&ps[(size_t)l * ND + q]));
        if (pmax[l] > umax2) umax2 = pmax[l];
        nf += pnf[l];
    }
    double ncell = (double)p->nx * p->ny * p->nz;
    out[0] = 0.5 * cval(&tot[0]) / ncell;
    out[1] = 0.5 * cval(&tot[2]) / ncell;
    out[2] = sqrt(cval(&tot[1]) / ncell);
    out[3] = sqrt(cval(&tot[0]) / ncell);
    out[4] = sqrt(umax2);
    out[5] = cval(&tot[3]) / ncell;
    out[6] = cval(&tot[4]) / ncell;
    out[7] = cval(&tot[5]) / ncell;
    out[8] = cval(&tot[6]) / ncell;
    out[9] = nf;
    free(ps); free(pmax); free(pnf);
    return 0;
}
