/*
 * Oracle O2-O4: a plain FP64 CPU solver for the variable-coefficient Stokes
 * system on the MAC grid.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is built into liboracle.so, which only
 * tests/, the smoke check and the CPU-baseline leg of the benchmark load.  It
 * shares no code, header or table with the HIP library.
 *
 * What it computes (Sec. 4.2.2, eq_c_discrete_momentum / eq_c_discrete_continuity,
 * with the staggered layout of Sec. 3.1 and harmonic edge viscosity, Sec. 4.2):
 *
 *   x-momentum at interior x-face (i,j,k):
 *     (rho_x/dt) u - theta * { [2 mu_c(i)(u(i+1)-u(i)) - 2 mu_c(i-1)(u(i)-u(i-1))]/hx^2
 *        + [mu_xy(i,j+1)((u(j+1)-u)/hy + (v(i,j+1)-v(i-1,j+1))/hx)
 *           - mu_xy(i,j)((u-u(j-1))/hy + (v(i,j)-v(i-1,j))/hx)]/hy
 *        + the same in z with mu_xz and w }  + (p(i)-p(i-1))/hx  = f_x
 *   (y and z rows by symmetry), and at every cell
 *     -[(u(i+1)-u(i))/hx + (v(j+1)-v(j))/hy + (w(k+1)-w(k))/hz] = g.
 *
 * Walls on every side: normal face velocity 0 (stored, never an unknown),
 * tangential ghost = -interior, pressure gradient on interior faces only.
 *
 * Solver (used only to reach that solution on grids too big for a direct
 * factorisation): restarted right-preconditioned flexible GMRES with modified
 * Gram-Schmidt (the FGMRES of Sec. 4.2.4), preconditioned by a projection step
 * whose two subsolves are multigrid V-cycles with lexicographic Gauss-Seidel.
 *
 * Layout: C order, x fastest. u (nz,ny,nx+1), v (nz,ny+1,nx), w (nz+1,ny,nx),
 * p and mu (nz,ny,nx).  2D: nz = 1, no w.
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int dim, nx, ny, nz;
    double hx, hy, hz;
} Grid;

/* one multigrid level: coefficients of both subproblems */
typedef struct {
    Grid g;
    long nu, nv, nw, nc;
    double *rho[3];      /* face density (velocity mass term) */
    double *beta[3];     /* face 1/rho for the pressure Poisson operator */
    double *mu;          /* cell viscosity */
    double *mxy, *mxz, *myz; /* edge viscosity (harmonic) */
    /* work arrays */
    double *eu[3], *ru[3], *tu[3];  /* velocity correction, rhs, temp */
    double *ep, *rp, *tp;           /* pressure correction, rhs, temp */
} Level;

typedef struct {
    int nlev;
    Level L[32];
    double dt, theta;
    int nu1, nu2, vel_cycles, p_cycles, coarse_sweeps;
} Hier;

/* ------------------------------------------------------------------ sizes */
static long n_u(const Grid *g) { return (long)(g->nx + 1) * g->ny * g->nz; }
static long n_v(const Grid *g) { return (long)g->nx * (g->ny + 1) * g->nz; }
static long n_w(const Grid *g) { return g->dim == 3 ? (long)g->nx * g->ny * (g->nz + 1) : 0; }
static long n_c(const Grid *g) { return (long)g->nx * g->ny * g->nz; }

/* ------------------------------------------------------------- addressing */
#define IU(g, i, j, k) ((((long)(k)) * (g)->ny + (j)) * ((g)->nx + 1) + (i))
#define IV(g, i, j, k) ((((long)(k)) * ((g)->ny + 1) + (j)) * (g)->nx + (i))
#define IW(g, i, j, k) ((((long)(k)) * (g)->ny + (j)) * (g)->nx + (i))
#define IC(g, i, j, k) ((((long)(k)) * (g)->ny + (j)) * (g)->nx + (i))
#define IXY(g, i, j, k) ((((long)(k)) * ((g)->ny + 1) + (j)) * ((g)->nx + 1) + (i))
#define IXZ(g, i, j, k) ((((long)(k)) * (g)->ny + (j)) * ((g)->nx + 1) + (i))
#define IYZ(g, i, j, k) ((((long)(k)) * ((g)->ny + 1) + (j)) * (g)->nx + (i))

/* velocity values with the no-slip ghost rule for tangential neighbours */
static double U(const Grid *g, const double *u, int i, int j, int k) {
    if (i <= 0 || i >= g->nx) return 0.0;                 /* wall-normal face */
    if (j < 0) return -U(g, u, i, 0, k);
    if (j >= g->ny) return -U(g, u, i, g->ny - 1, k);
    if (g->dim == 3) {
        if (k < 0) return -U(g, u, i, j, 0);
        if (k >= g->nz) return -U(g, u, i, j, g->nz - 1);
    }
    return u[IU(g, i, j, k)];
}
static double V(const Grid *g, const double *v, int i, int j, int k) {
    if (j <= 0 || j >= g->ny) return 0.0;
    if (i < 0) return -V(g, v, 0, j, k);
    if (i >= g->nx) return -V(g, v, g->nx - 1, j, k);
    if (g->dim == 3) {
        if (k < 0) return -V(g, v, i, j, 0);
        if (k >= g->nz) return -V(g, v, i, j, g->nz - 1);
    }
    return v[IV(g, i, j, k)];
}
static double W(const Grid *g, const double *w, int i, int j, int k) {
    if (k <= 0 || k >= g->nz) return 0.0;
    if (i < 0) return -W(g, w, 0, j, k);
    if (i >= g->nx) return -W(g, w, g->nx - 1, j, k);
    if (j < 0) return -W(g, w, i, 0, k);
    if (j >= g->ny) return -W(g, w, i, g->ny - 1, k);
    return w[IW(g, i, j, k)];
}
static int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* harmonic mean of mu over the 4 cells around an edge; out-of-domain cells mirror */
static void edge_viscosity(const Grid *g, const double *mu, double *mxy, double *mxz, double *myz) {
    int nx = g->nx, ny = g->ny, nz = g->nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double s = 0.0;
                for (int a = i - 1; a <= i; ++a)
                    for (int b = j - 1; b <= j; ++b)
                        s += 1.0 / mu[IC(g, clampi(a, 0, nx - 1), clampi(b, 0, ny - 1), k)];
                mxy[IXY(g, i, j, k)] = 4.0 / s;
            }
    if (g->dim < 3) return;
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double s = 0.0;
                for (int a = i - 1; a <= i; ++a)
                    for (int c = k - 1; c <= k; ++c)
                        s += 1.0 / mu[IC(g, clampi(a, 0, nx - 1), j, clampi(c, 0, nz - 1))];
                mxz[IXZ(g, i, j, k)] = 4.0 / s;
            }
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double s = 0.0;
                for (int b = j - 1; b <= j; ++b)
                    for (int c = k - 1; c <= k; ++c)
                        s += 1.0 / mu[IC(g, i, clampi(b, 0, ny - 1), clampi(c, 0, nz - 1))];
                myz[IYZ(g, i, j, k)] = 4.0 / s;
            }
}

/* ------------------------------------------------ momentum rows (no p) */
/* A u at an interior x-face, and the row's diagonal coefficient */
static double row_x(const Level *L, double dt, double th, const double *u, const double *v,
                    const double *w, int i, int j, int k, double *diag) {
    const Grid *g = &L->g;
    double hx = g->hx, hy = g->hy, hz = g->hz;
    double uc = u[IU(g, i, j, k)];
    double m0 = L->mu[IC(g, i - 1, j, k)], m1 = L->mu[IC(g, i, j, k)];
    double lap = (2.0 * m1 * (U(g, u, i + 1, j, k) - uc) - 2.0 * m0 * (uc - U(g, u, i - 1, j, k))) / (hx * hx);
    double mN = L->mxy[IXY(g, i, j + 1, k)], mS = L->mxy[IXY(g, i, j, k)];
    double sN = (U(g, u, i, j + 1, k) - uc) / hy + (V(g, v, i, j + 1, k) - V(g, v, i - 1, j + 1, k)) / hx;
    double sS = (uc - U(g, u, i, j - 1, k)) / hy + (V(g, v, i, j, k) - V(g, v, i - 1, j, k)) / hx;
    lap += (mN * sN - mS * sS) / hy;
    double d = L->rho[0][IU(g, i, j, k)] / dt + th * (2.0 * (m0 + m1) / (hx * hx)
               + (mN * (j + 1 >= g->ny ? 2.0 : 1.0) + mS * (j - 1 < 0 ? 2.0 : 1.0)) / (hy * hy));
    if (g->dim == 3) {
        double mT = L->mxz[IXZ(g, i, j, k + 1)], mB = L->mxz[IXZ(g, i, j, k)];
        double sT = (U(g, u, i, j, k + 1) - uc) / hz + (W(g, w, i, j, k + 1) - W(g, w, i - 1, j, k + 1)) / hx;
        double sB = (uc - U(g, u, i, j, k - 1)) / hz + (W(g, w, i, j, k) - W(g, w, i - 1, j, k)) / hx;
        lap += (mT * sT - mB * sB) / hz;
        d += th * (mT * (k + 1 >= g->nz ? 2.0 : 1.0) + mB * (k - 1 < 0 ? 2.0 : 1.0)) / (hz * hz);
    }
    if (diag) *diag = d;
    return L->rho[0][IU(g, i, j, k)] / dt * uc - th * lap;
}

static double row_y(const Level *L, double dt, double th, const double *u, const double *v,
                    const double *w, int i, int j, int k, double *diag) {
    const Grid *g = &L->g;
    double hx = g->hx, hy = g->hy, hz = g->hz;
    double vc = v[IV(g, i, j, k)];
    double m0 = L->mu[IC(g, i, j - 1, k)], m1 = L->mu[IC(g, i, j, k)];
    double lap = (2.0 * m1 * (V(g, v, i, j + 1, k) - vc) - 2.0 * m0 * (vc - V(g, v, i, j - 1, k))) / (hy * hy);
    double mE = L->mxy[IXY(g, i + 1, j, k)], mW = L->mxy[IXY(g, i, j, k)];
    double sE = (V(g, v, i + 1, j, k) - vc) / hx + (U(g, u, i + 1, j, k) - U(g, u, i + 1, j - 1, k)) / hy;
    double sW = (vc - V(g, v, i - 1, j, k)) / hx + (U(g, u, i, j, k) - U(g, u, i, j - 1, k)) / hy;
    lap += (mE * sE - mW * sW) / hx;
    double d = L->rho[1][IV(g, i, j, k)] / dt + th * (2.0 * (m0 + m1) / (hy * hy)
               + (mE * (i + 1 >= g->nx ? 2.0 : 1.0) + mW * (i - 1 < 0 ? 2.0 : 1.0)) / (hx * hx));
    if (g->dim == 3) {
        double mT = L->myz[IYZ(g, i, j, k + 1)], mB = L->myz[IYZ(g, i, j, k)];
        double sT = (V(g, v, i, j, k + 1) - vc) / hz + (W(g, w, i, j, k + 1) - W(g, w, i, j - 1, k + 1)) / hy;
        double sB = (vc - V(g, v, i, j, k - 1)) / hz + (W(g, w, i, j, k) - W(g, w, i, j - 1, k)) / hy;
        lap += (mT * sT - mB * sB) / hz;
        d += th * (mT * (k + 1 >= g->nz ? 2.0 : 1.0) + mB * (k - 1 < 0 ? 2.0 : 1.0)) / (hz * hz);
    }
    if (diag) *diag = d;
    return L->rho[1][IV(g, i, j, k)] / dt * vc - th * lap;
}

static double row_z(const Level *L, double dt, double th, const double *u, const double *v,
                    const double *w, int i, int j, int k, double *diag) {
    const Grid *g = &L->g;
    double hx = g->hx, hy = g->hy, hz = g->hz;
    double wc = w[IW(g, i, j, k)];
    double m0 = L->mu[IC(g, i, j, k - 1)], m1 = L->mu[IC(g, i, j, k)];
    double lap = (2.0 * m1 * (W(g, w, i, j, k + 1) - wc) - 2.0 * m0 * (wc - W(g, w, i, j, k - 1))) / (hz * hz);
    double mE = L->mxz[IXZ(g, i + 1, j, k)], mW = L->mxz[IXZ(g, i, j, k)];
    double sE = (W(g, w, i + 1, j, k) - wc) / hx + (U(g, u, i + 1, j, k) - U(g, u, i + 1, j, k - 1)) / hz;
    double sW = (wc - W(g, w, i - 1, j, k)) / hx + (U(g, u, i, j, k) - U(g, u, i, j, k - 1)) / hz;
    lap += (mE * sE - mW * sW) / hx;
    double mN = L->myz[IYZ(g, i, j + 1, k)], mS = L->myz[IYZ(g, i, j, k)];
    double sN = (W(g, w, i, j + 1, k) - wc) / hy + (V(g, v, i, j + 1, k) - V(g, v, i, j + 1, k - 1)) / hz;
    double sS = (wc - W(g, w, i, j - 1, k)) / hy + (V(g, v, i, j, k) - V(g, v, i, j, k - 1)) / hz;
    lap += (mN * sN - mS * sS) / hy;
    double d = L->rho[2][IW(g, i, j, k)] / dt + th * (2.0 * (m0 + m1) / (hz * hz)
               + (mE * (i + 1 >= g->nx ? 2.0 : 1.0) + mW * (i - 1 < 0 ? 2.0 : 1.0)) / (hx * hx)
               + (mN * (j + 1 >= g->ny ? 2.0 : 1.0) + mS * (j - 1 < 0 ? 2.0 : 1.0)) / (hy * hy));
    if (diag) *diag = d;
    return L->rho[2][IW(g, i, j, k)] / dt * wc - th * lap;
}

/* ------------------------------------------------------ full operator */
/* y = K x with K = [A G; -D 0] on a level (the fine level in practice). */
static void apply_K(const Level *L, double dt, double th, double *const x[4], double *const y[4]) {
    const Grid *g = &L->g;
    int nx = g->nx, ny = g->ny, nz = g->nz;
    const double *u = x[0], *v = x[1], *w = x[2], *p = x[3];
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double r = 0.0;
                if (i > 0 && i < nx)
                    r = row_x(L, dt, th, u, v, w, i, j, k, NULL) + (p[IC(g, i, j, k)] - p[IC(g, i - 1, j, k)]) / g->hx;
                y[0][IU(g, i, j, k)] = r;
            }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double r = 0.0;
                if (j > 0 && j < ny)
                    r = row_y(L, dt, th, u, v, w, i, j, k, NULL) + (p[IC(g, i, j, k)] - p[IC(g, i, j - 1, k)]) / g->hy;
                y[1][IV(g, i, j, k)] = r;
            }
    if (g->dim == 3) {
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    double r = 0.0;
                    if (k > 0 && k < nz)
                        r = row_z(L, dt, th, u, v, w, i, j, k, NULL) + (p[IC(g, i, j, k)] - p[IC(g, i, j, k - 1)]) / g->hz;
                    y[2][IW(g, i, j, k)] = r;
                }
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double dv = (u[IU(g, i + 1, j, k)] - u[IU(g, i, j, k)]) / g->hx
                          + (v[IV(g, i, j + 1, k)] - v[IV(g, i, j, k)]) / g->hy;
                if (g->dim == 3) dv += (w[IW(g, i, j, k + 1)] - w[IW(g, i, j, k)]) / g->hz;
                y[3][IC(g, i, j, k)] = -dv;
            }
}

/* ------------------------------------------------------ pressure operator */
/* (-D beta G phi) at one cell; wall faces carry no flux */
static double prow(const Level *L, const double *ph, int i, int j, int k, double *diag) {
    const Grid *g = &L->g;
    double c = ph[IC(g, i, j, k)], s = 0.0, d = 0.0, b;
    double ix2 = 1.0 / (g->hx * g->hx), iy2 = 1.0 / (g->hy * g->hy), iz2 = 1.0 / (g->hz * g->hz);
    if (i > 0)         { b = L->beta[0][IU(g, i, j, k)] * ix2;     s += b * (c - ph[IC(g, i - 1, j, k)]); d += b; }
    if (i < g->nx - 1) { b = L->beta[0][IU(g, i + 1, j, k)] * ix2; s += b * (c - ph[IC(g, i + 1, j, k)]); d += b; }
    if (j > 0)         { b = L->beta[1][IV(g, i, j, k)] * iy2;     s += b * (c - ph[IC(g, i, j - 1, k)]); d += b; }
    if (j < g->ny - 1) { b = L->beta[1][IV(g, i, j + 1, k)] * iy2; s += b * (c - ph[IC(g, i, j + 1, k)]); d += b; }
    if (g->dim == 3) {
        if (k > 0)         { b = L->beta[2][IW(g, i, j, k)] * iz2;     s += b * (c - ph[IC(g, i, j, k - 1)]); d += b; }
        if (k < g->nz - 1) { b = L->beta[2][IW(g, i, j, k + 1)] * iz2; s += b * (c - ph[IC(g, i, j, k + 1)]); d += b; }
    }
    if (diag) *diag = d;
    return s;
}

static double mean_c(const Grid *g, const double *a) {
    long n = n_c(g);
    double s = 0.0;
    for (long q = 0; q < n; ++q) s += a[q];
    return s / (double)n;
}
static void sub_mean(const Grid *g, double *a) {
    double m = mean_c(g, a);
    long n = n_c(g);
    for (long q = 0; q < n; ++q) a[q] -= m;
}

/* lexicographic Gauss-Seidel sweeps on -L_rho phi = s */
static void p_gs(const Level *L, double *ph, const double *s, int sweeps) {
    const Grid *g = &L->g;
    for (int it = 0; it < sweeps; ++it)
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    double d;
                    double a = prow(L, ph, i, j, k, &d);
                    if (d > 0.0) ph[IC(g, i, j, k)] += (s[IC(g, i, j, k)] - a) / d;
                }
}

static void p_residual(const Level *L, const double *ph, const double *s, double *r) {
    const Grid *g = &L->g;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i)
                r[IC(g, i, j, k)] = s[IC(g, i, j, k)] - prow(L, ph, i, j, k, NULL);
}

/* restriction: coarse cell value = average of its 2^d children */
static void restrict_c(const Grid *f, const Grid *c, const double *a, double *b) {
    int kk = f->dim == 3 ? 2 : 1;
    double wgt = f->dim == 3 ? 0.125 : 0.25;
    for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) {
                double s = 0.0;
                for (int dk = 0; dk < kk; ++dk)
                    for (int dj = 0; dj < 2; ++dj)
                        for (int di = 0; di < 2; ++di)
                            s += a[IC(f, 2 * i + di, 2 * j + dj, kk * k + dk)];
                b[IC(c, i, j, k)] = wgt * s;
            }
}

/* prolongation: every child takes its parent's value, added to a */
static void prolong_c_add(const Grid *f, const Grid *c, const double *b, double *a) {
    int kk = f->dim == 3 ? 2 : 1;
    for (int k = 0; k < f->nz; ++k)
        for (int j = 0; j < f->ny; ++j)
            for (int i = 0; i < f->nx; ++i)
                a[IC(f, i, j, k)] += b[IC(c, i / 2, j / 2, k / kk)];
}

static void p_vcycle(Hier *H, int l, double *ph, const double *s) {
    Level *L = &H->L[l];
    if (l == H->nlev - 1) {
        /* coarsest: Gauss-Seidel until the residual stops changing */
        double r0 = 0.0;
        p_residual(L, ph, s, L->tp);
        for (long q = 0; q < L->nc; ++q) r0 += L->tp[q] * L->tp[q];
        for (int it = 0; it < H->coarse_sweeps; it += 10) {
            p_gs(L, ph, s, 10);
            sub_mean(&L->g, ph);
            p_residual(L, ph, s, L->tp);
            double rr = 0.0;
            for (long q = 0; q < L->nc; ++q) rr += L->tp[q] * L->tp[q];
            if (rr <= 1e-28 * r0) break;
        }
        return;
    }
    Level *C = &H->L[l + 1];
    p_gs(L, ph, s, H->nu1);
    p_residual(L, ph, s, L->tp);
    restrict_c(&L->g, &C->g, L->tp, C->rp);
    memset(C->ep, 0, sizeof(double) * C->nc);
    p_vcycle(H, l + 1, C->ep, C->rp);
    prolong_c_add(&L->g, &C->g, C->ep, ph);
    p_gs(L, ph, s, H->nu2);
}

/* ------------------------------------------------------ velocity multigrid */
static void v_gs(const Level *L, double dt, double th, double *const e[3], double *const r[3], int sweeps) {
    const Grid *g = &L->g;
    double *u = e[0], *v = e[1], *w = e[2];
    for (int it = 0; it < sweeps; ++it) {
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 1; i < g->nx; ++i) {
                    double d, a = row_x(L, dt, th, u, v, w, i, j, k, &d);
                    u[IU(g, i, j, k)] += (r[0][IU(g, i, j, k)] - a) / d;
                }
        for (int k = 0; k < g->nz; ++k)
            for (int j = 1; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    double d, a = row_y(L, dt, th, u, v, w, i, j, k, &d);
                    v[IV(g, i, j, k)] += (r[1][IV(g, i, j, k)] - a) / d;
                }
        if (g->dim == 3)
            for (int k = 1; k < g->nz; ++k)
                for (int j = 0; j < g->ny; ++j)
                    for (int i = 0; i < g->nx; ++i) {
                        double d, a = row_z(L, dt, th, u, v, w, i, j, k, &d);
                        w[IW(g, i, j, k)] += (r[2][IW(g, i, j, k)] - a) / d;
                    }
    }
}

static void v_residual(const Level *L, double dt, double th, double *const e[3], double *const r[3], double *const out[3]) {
    const Grid *g = &L->g;
    memset(out[0], 0, sizeof(double) * L->nu);
    memset(out[1], 0, sizeof(double) * L->nv);
    if (g->dim == 3) memset(out[2], 0, sizeof(double) * L->nw);
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 1; i < g->nx; ++i)
                out[0][IU(g, i, j, k)] = r[0][IU(g, i, j, k)] - row_x(L, dt, th, e[0], e[1], e[2], i, j, k, NULL);
    for (int k = 0; k < g->nz; ++k)
        for (int j = 1; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i)
                out[1][IV(g, i, j, k)] = r[1][IV(g, i, j, k)] - row_y(L, dt, th, e[0], e[1], e[2], i, j, k, NULL);
    if (g->dim == 3)
        for (int k = 1; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i)
                    out[2][IW(g, i, j, k)] = r[2][IW(g, i, j, k)] - row_z(L, dt, th, e[0], e[1], e[2], i, j, k, NULL);
}

/* Face restriction for component `a` (0,1,2) between grids: the coarse face
 * takes weight 2 from each coincident fine face and weight 1 from each fine
 * face half a coarse cell to either side, normalised to a unit sum.  Applied to
 * interior coarse faces only; coarse wall faces are set to zero. */
static double face_get(const Grid *g, const double *a, int comp, int i, int j, int k) {
    if (comp == 0) return a[IU(g, i, j, k)];
    if (comp == 1) return a[IV(g, i, j, k)];
    return a[IW(g, i, j, k)];
}
static long face_idx(const Grid *g, int comp, int i, int j, int k) {
    if (comp == 0) return IU(g, i, j, k);
    if (comp == 1) return IV(g, i, j, k);
    return IW(g, i, j, k);
}
static void restrict_f(const Grid *f, const Grid *c, int comp, const double *a, double *b, int keep_walls) {
    int nI = c->nx + (comp == 0), nJ = c->ny + (comp == 1), nK = c->nz + (comp == 2 && c->dim == 3);
    int d3 = f->dim == 3;
    for (int K = 0; K < nK; ++K)
        for (int J = 0; J < nJ; ++J)
            for (int I = 0; I < nI; ++I) {
                int cc[3] = {I, J, K};
                int ncomp = comp == 0 ? c->nx : (comp == 1 ? c->ny : c->nz);
                long ci = face_idx(c, comp, I, J, K);
                if (cc[comp] == 0 || cc[comp] == ncomp) {
                    if (!keep_walls) { b[ci] = 0.0; continue; }
                }
                double s = 0.0, wsum = 0.0;
                /* transverse children */
                int t1 = comp == 0 ? 1 : 0, t2 = comp == 2 ? 1 : 2;
                int nt2 = d3 ? 2 : 1;
                for (int a1 = 0; a1 < 2; ++a1)
                    for (int a2 = 0; a2 < nt2; ++a2)
                        for (int off = -1; off <= 1; ++off) {
                            int fi[3];
                            fi[comp] = 2 * cc[comp] + off;
                            fi[t1] = 2 * cc[t1] + a1;
                            fi[t2] = d3 ? 2 * cc[t2] + a2 : 0;
                            int nfa = comp == 0 ? f->nx : (comp == 1 ? f->ny : f->nz);
                            if (fi[comp] < 0 || fi[comp] > nfa) continue;
                            double wt = off == 0 ? 2.0 : 1.0;
                            s += wt * face_get(f, a, comp, fi[0], fi[1], fi[2]);
                            wsum += wt;
                        }
                b[ci] = s / wsum;
            }
}

/* face prolongation for component comp: linear along the normal, constant
 * across; fine wall faces stay zero.  Adds into a. */
static void prolong_f_add(const Grid *f, const Grid *c, int comp, const double *b, double *a) {
    int nI = f->nx + (comp == 0), nJ = f->ny + (comp == 1), nK = f->nz + (comp == 2 && f->dim == 3);
    int kk = f->dim == 3 ? 2 : 1;
    int nfa = comp == 0 ? f->nx : (comp == 1 ? f->ny : f->nz);
    for (int k = 0; k < nK; ++k)
        for (int j = 0; j < nJ; ++j)
            for (int i = 0; i < nI; ++i) {
                int fi[3] = {i, j, k};
                if (fi[comp] == 0 || fi[comp] == nfa) continue;
                int ci[3] = {i / 2, j / 2, k / kk};
                double val;
                if (fi[comp] % 2 == 0) {
                    ci[comp] = fi[comp] / 2;
                    val = face_get(c, b, comp, ci[0], ci[1], ci[2]);
                } else {
                    int c0[3] = {ci[0], ci[1], ci[2]}, c1[3] = {ci[0], ci[1], ci[2]};
                    c0[comp] = (fi[comp] - 1) / 2;
                    c1[comp] = (fi[comp] + 1) / 2;
                    val = 0.5 * (face_get(c, b, comp, c0[0], c0[1], c0[2]) + face_get(c, b, comp, c1[0], c1[1], c1[2]));
                }
                a[face_idx(f, comp, i, j, k)] += val;
            }
}

static void v_vcycle(Hier *H, int l, double *const e[3], double *const r[3]) {
    Level *L = &H->L[l];
    int d = L->g.dim;
    if (l == H->nlev - 1) {
        v_gs(L, H->dt, H->theta, e, r, H->coarse_sweeps);
        return;
    }
    Level *C = &H->L[l + 1];
    v_gs(L, H->dt, H->theta, e, r, H->nu1);
    v_residual(L, H->dt, H->theta, e, r, L->tu);
    for (int a = 0; a < d; ++a) restrict_f(&L->g, &C->g, a, L->tu[a], C->ru[a], 0);
    memset(C->eu[0], 0, sizeof(double) * C->nu);
    memset(C->eu[1], 0, sizeof(double) * C->nv);
    if (d == 3) memset(C->eu[2], 0, sizeof(double) * C->nw);
    v_vcycle(H, l + 1, C->eu, C->ru);
    for (int a = 0; a < d; ++a) prolong_f_add(&L->g, &C->g, a, C->eu[a], e[a]);
    v_gs(L, H->dt, H->theta, e, r, H->nu2);
}

/* ------------------------------------------------------ hierarchy setup */
static int can_coarsen(const Grid *g) {
    int ok = g->nx % 2 == 0 && g->ny % 2 == 0 && g->nx >= 4 && g->ny >= 4;
    if (g->dim == 3) ok = ok && g->nz % 2 == 0 && g->nz >= 4;
    long cells = n_c(g);
    return ok && cells > 64;
}

static void level_alloc(Level *L, const Grid *g) {
    L->g = *g;
    L->nu = n_u(g); L->nv = n_v(g); L->nw = n_w(g); L->nc = n_c(g);
    long nf[3] = {L->nu, L->nv, L->nw};
    for (int a = 0; a < 3; ++a) {
        long m = nf[a] > 0 ? nf[a] : 1;
        L->rho[a] = calloc(m, sizeof(double));
        L->beta[a] = calloc(m, sizeof(double));
        L->eu[a] = calloc(m, sizeof(double));
        L->ru[a] = calloc(m, sizeof(double));
        L->tu[a] = calloc(m, sizeof(double));
    }
    L->mu = calloc(L->nc, sizeof(double));
    L->mxy = calloc((long)(g->nx + 1) * (g->ny + 1) * g->nz, sizeof(double));
    if (g->dim == 3) {
        L->mxz = calloc((long)(g->nx + 1) * g->ny * (g->nz + 1), sizeof(double));
        L->myz = calloc((long)g->nx * (g->ny + 1) * (g->nz + 1), sizeof(double));
    } else {
        L->mxz = L->myz = NULL;
    }
    L->ep = calloc(L->nc, sizeof(double));
    L->rp = calloc(L->nc, sizeof(double));
    L->tp = calloc(L->nc, sizeof(double));
}

static void level_free(Level *L) {
    for (int a = 0; a < 3; ++a) {
        free(L->rho[a]); free(L->beta[a]); free(L->eu[a]); free(L->ru[a]); free(L->tu[a]);
    }
    free(L->mu); free(L->mxy); free(L->mxz); free(L->myz);
    free(L->ep); free(L->rp); free(L->tp);
}

static void hier_build(Hier *H, const Grid *g, double *const rho[3], const double *mu) {
    Level *F = &H->L[0];
    level_alloc(F, g);
    for (int a = 0; a < g->dim; ++a) {
        long m = a == 0 ? F->nu : (a == 1 ? F->nv : F->nw);
        memcpy(F->rho[a], rho[a], sizeof(double) * m);
        for (long q = 0; q < m; ++q) F->beta[a][q] = 1.0 / rho[a][q];
    }
    memcpy(F->mu, mu, sizeof(double) * F->nc);
    edge_viscosity(g, F->mu, F->mxy, F->mxz, F->myz);
    H->nlev = 1;
    while (H->nlev < 32 && can_coarsen(&H->L[H->nlev - 1].g)) {
        Level *f = &H->L[H->nlev - 1];
        Level *c = &H->L[H->nlev];
        Grid cg = f->g;
        cg.nx /= 2; cg.ny /= 2; if (cg.dim == 3) cg.nz /= 2;
        cg.hx *= 2; cg.hy *= 2; if (cg.dim == 3) cg.hz *= 2;
        level_alloc(c, &cg);
        int d3 = cg.dim == 3;
        /* viscosity: harmonic mean of the children */
        for (int k = 0; k < cg.nz; ++k)
            for (int j = 0; j < cg.ny; ++j)
                for (int i = 0; i < cg.nx; ++i) {
                    double s = 0.0; int cnt = 0;
                    for (int dk = 0; dk < (d3 ? 2 : 1); ++dk)
                        for (int dj = 0; dj < 2; ++dj)
                            for (int di = 0; di < 2; ++di) {
                                s += 1.0 / f->mu[IC(&f->g, 2 * i + di, 2 * j + dj, (d3 ? 2 * k + dk : 0))];
                                cnt++;
                            }
                    c->mu[IC(&cg, i, j, k)] = cnt / s;
                }
        edge_viscosity(&cg, c->mu, c->mxy, c->mxz, c->myz);
        /* velocity mass density: face restriction of rho (interior and wall faces) */
        for (int a = 0; a < cg.dim; ++a) restrict_f(&f->g, &cg, a, f->rho[a], c->rho[a], 1);
        /* Poisson coefficient: arithmetic mean of the coincident fine beta */
        for (int a = 0; a < cg.dim; ++a) {
            int nI = cg.nx + (a == 0), nJ = cg.ny + (a == 1), nK = cg.nz + (a == 2 && d3);
            for (int K = 0; K < nK; ++K)
                for (int J = 0; J < nJ; ++J)
                    for (int I = 0; I < nI; ++I) {
                        int cc[3] = {I, J, K};
                        double s = 0.0; int cnt = 0;
                        int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
                        for (int a1 = 0; a1 < 2; ++a1)
                            for (int a2 = 0; a2 < (d3 ? 2 : 1); ++a2) {
                                int fi[3];
                                fi[a] = 2 * cc[a];
                                fi[t1] = 2 * cc[t1] + a1;
                                fi[t2] = d3 ? 2 * cc[t2] + a2 : 0;
                                s += face_get(&f->g, f->beta[a], a, fi[0], fi[1], fi[2]);
                                cnt++;
                            }
                        c->beta[a][face_idx(&cg, a, I, J, K)] = s / cnt;
                    }
        }
        H->nlev++;
    }
}

static void hier_free(Hier *H) {
    for (int l = 0; l < H->nlev; ++l) level_free(&H->L[l]);
}

/* ------------------------------------------------------ vectors */
typedef struct { double *f[4]; } Vec;   /* u, v, w, p on the fine grid */

static long vlen(const Level *L, int c) {
    return c == 0 ? L->nu : c == 1 ? L->nv : c == 2 ? L->nw : L->nc;
}
static Vec vnew(const Level *L) {
    Vec x;
    for (int c = 0; c < 4; ++c) x.f[c] = calloc(vlen(L, c) > 0 ? vlen(L, c) : 1, sizeof(double));
    return x;
}
static void vfree(Vec *x) { for (int c = 0; c < 4; ++c) free(x->f[c]); }
/* inner product with the continuity/pressure block weighted by w2 */
static double vdot(const Level *L, const Vec *a, const Vec *b, double w2) {
    double s = 0.0;
    for (int c = 0; c < 4; ++c) {
        long n = vlen(L, c);
        const double *x = a->f[c], *y = b->f[c];
        double t = 0.0;
#pragma omp parallel for reduction(+ : t) schedule(static)
        for (long q = 0; q < n; ++q) t += x[q] * y[q];
        s += c == 3 ? w2 * t : t;
    }
    return s;
}
static void vaxpy(const Level *L, double al, const Vec *x, Vec *y) {
    for (int c = 0; c < 4; ++c) {
        long n = vlen(L, c);
        double *yy = y->f[c];
        const double *xx = x->f[c];
#pragma omp parallel for schedule(static)
        for (long q = 0; q < n; ++q) yy[q] += al * xx[q];
    }
}
static void vscale_copy(const Level *L, double al, const Vec *x, Vec *y) {
    for (int c = 0; c < 4; ++c) {
        long n = vlen(L, c);
#pragma omp parallel for schedule(static)
        for (long q = 0; q < n; ++q) y->f[c][q] = al * x->f[c][q];
    }
}

/* ------------------------------------------------------ preconditioner */
/* Projection-method preconditioner with a local-viscosity pressure update:
 *  1. u~ ~= A^{-1} r_u                    (velocity V-cycles)
 *  2. s = (r_p + D u~)/dt, mean removed
 *  3. phi ~= L_rho^{-1} s, L_rho = D beta G   (pressure V-cycles on -L_rho)
 *  4. u = u~ - dt beta G phi
 *  5. p = phi - 2 theta mu (r_p + D u~), mean removed                      */
static void precond(Hier *H, const Vec *r, Vec *z) {
    Level *F = &H->L[0];
    const Grid *g = &F->g;
    double dt = H->dt, th = H->theta;
    int d = g->dim;
    double *eu[3] = {z->f[0], z->f[1], z->f[2]};
    double *ru[3] = {r->f[0], r->f[1], r->f[2]};
    memset(z->f[0], 0, sizeof(double) * F->nu);
    memset(z->f[1], 0, sizeof(double) * F->nv);
    if (d == 3) memset(z->f[2], 0, sizeof(double) * F->nw);
    for (int c = 0; c < H->vel_cycles; ++c) {
        if (c == 0) {
            v_vcycle(H, 0, eu, ru);
        } else {
            /* further cycles act on the remaining residual; the level-0 ru/eu
             * arrays are free here (a V-cycle on level 0 uses only tu there) */
            v_residual(F, dt, th, eu, ru, F->ru);
            double *cu[3] = {F->eu[0], F->eu[1], F->eu[2]};
            memset(cu[0], 0, sizeof(double) * F->nu);
            memset(cu[1], 0, sizeof(double) * F->nv);
            if (d == 3) memset(cu[2], 0, sizeof(double) * F->nw);
            v_vcycle(H, 0, cu, F->ru);
            for (int a = 0; a < d; ++a)
                for (long q = 0; q < vlen(F, a); ++q) eu[a][q] += cu[a][q];
        }
    }
    /* divergence of u~ plus r_p (a V-cycle on level 0 overwrites tp, so q is its own array) */
    double *q = malloc(sizeof(double) * F->nc);   /* r_p + D u~ */
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                double dv = (eu[0][IU(g, i + 1, j, k)] - eu[0][IU(g, i, j, k)]) / g->hx
                          + (eu[1][IV(g, i, j + 1, k)] - eu[1][IV(g, i, j, k)]) / g->hy;
                if (d == 3) dv += (eu[2][IW(g, i, j, k + 1)] - eu[2][IW(g, i, j, k)]) / g->hz;
                q[IC(g, i, j, k)] = r->f[3][IC(g, i, j, k)] + dv;
            }
    double *s = F->rp, *phi = F->ep;
    /* the Poisson problem is -L_rho phi = -s */
    for (long c = 0; c < F->nc; ++c) s[c] = -q[c] / dt;
    sub_mean(g, s);
    memset(phi, 0, sizeof(double) * F->nc);
    double *cor = malloc(sizeof(double) * F->nc);
    double *res = malloc(sizeof(double) * F->nc);
    for (int c = 0; c < H->p_cycles; ++c) {
        if (c == 0) {
            p_vcycle(H, 0, phi, s);
        } else {
            p_residual(F, phi, s, res);
            memset(cor, 0, sizeof(double) * F->nc);
            p_vcycle(H, 0, cor, res);
            for (long t = 0; t < F->nc; ++t) phi[t] += cor[t];
        }
        sub_mean(g, phi);
    }
    free(cor);
    free(res);
    /* velocity correction u = u~ - dt beta G phi on interior faces */
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 1; i < g->nx; ++i)
                eu[0][IU(g, i, j, k)] -= dt * F->beta[0][IU(g, i, j, k)] * (phi[IC(g, i, j, k)] - phi[IC(g, i - 1, j, k)]) / g->hx;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 1; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i)
                eu[1][IV(g, i, j, k)] -= dt * F->beta[1][IV(g, i, j, k)] * (phi[IC(g, i, j, k)] - phi[IC(g, i, j - 1, k)]) / g->hy;
    if (d == 3)
        for (int k = 1; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i)
                    eu[2][IW(g, i, j, k)] -= dt * F->beta[2][IW(g, i, j, k)] * (phi[IC(g, i, j, k)] - phi[IC(g, i, j, k - 1)]) / g->hz;
    /* local-viscosity pressure update */
    for (long c = 0; c < F->nc; ++c) z->f[3][c] = phi[c] - 2.0 * th * F->mu[c] * q[c];
    sub_mean(g, z->f[3]);
    free(q);
}

/* ------------------------------------------------------ FGMRES */
typedef struct {
    int iters, restarts, status;
    double rel_res_est, rel_res_true, bnorm, gmean;
} SolveInfo;

/* Weight of the continuity rows in the residual norm.  The momentum rows scale
 * like a = rho/dt (plus viscosity) and the continuity rows like 1/h, which
 * leaves the plain 2-norm with a condition number near 1e14 and the pressure
 * barely determined by it.  Weighting the continuity rows (and, equivalently,
 * measuring the pressure in units of sigma) by sigma = a_ref * l / pi, where
 * pi/l is the smallest pressure wavenumber (l the longest side) and a_ref the
 * geometric mean of the smallest and largest rho/dt plus the viscous term at
 * that wavenumber, balances both blocks at the slowest pressure mode. */
static double auto_sigma(const Level *F, double dt, double th) {
    const Grid *g = &F->g;
    double rmin = INFINITY, rmax = 0.0, mmax = 0.0;
    long nf[3] = {F->nu, F->nv, F->nw};
    for (int a = 0; a < g->dim; ++a)
        for (long q = 0; q < nf[a]; ++q) {
            double r = F->rho[a][q];
            if (r < rmin) rmin = r;
            if (r > rmax) rmax = r;
        }
    for (long q = 0; q < F->nc; ++q) if (F->mu[q] > mmax) mmax = F->mu[q];
    double l = g->nx * g->hx;
    if (g->ny * g->hy > l) l = g->ny * g->hy;
    if (g->dim == 3 && g->nz * g->hz > l) l = g->nz * g->hz;
    double k = 3.14159265358979323846 / l;
    double aref = sqrt(rmin * rmax) / dt + th * mmax * k * k;
    return aref / k;
}

static void residual_vec(Hier *H, const Vec *b, const Vec *x, Vec *r) {
    double *xi[4] = {x->f[0], x->f[1], x->f[2], x->f[3]};
    double *ro[4] = {r->f[0], r->f[1], r->f[2], r->f[3]};
    apply_K(&H->L[0], H->dt, H->theta, xi, ro);
    for (int c = 0; c < 4; ++c) {
        long n = vlen(&H->L[0], c);
        for (long q = 0; q < n; ++q) r->f[c][q] = b->f[c][q] - r->f[c][q];
    }
}

static void fgmres(Hier *H, Vec *b, Vec *x, double tol, int m, int max_iters, double w2, SolveInfo *info) {
    Level *F = &H->L[0];
    Vec *V = malloc(sizeof(Vec) * (m + 1));
    Vec *Z = malloc(sizeof(Vec) * m);
    for (int j = 0; j <= m; ++j) V[j] = vnew(F);
    for (int j = 0; j < m; ++j) Z[j] = vnew(F);
    Vec w = vnew(F), r = vnew(F);
    double *Hm = calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = calloc(m, sizeof(double)), *sn = calloc(m, sizeof(double));
    double *gv = calloc(m + 1, sizeof(double)), *y = calloc(m, sizeof(double));
#define HH(i, j) Hm[(size_t)(i) * m + (j)]
    double bnorm = sqrt(vdot(F, b, b, w2));
    info->bnorm = bnorm;
    info->iters = 0;
    info->restarts = 0;
    info->status = 1;
    if (bnorm == 0.0) {
        for (int c = 0; c < 4; ++c) memset(x->f[c], 0, sizeof(double) * (vlen(F, c) > 0 ? vlen(F, c) : 1));
        info->rel_res_est = info->rel_res_true = 0.0;
        info->status = 0;
        goto done;
    }
    sub_mean(&F->g, x->f[3]);
    double prev_cycle_res = INFINITY;
    for (;;) {
        residual_vec(H, b, x, &r);
        double beta = sqrt(vdot(F, &r, &r, w2));
        info->rel_res_true = beta / bnorm;
        if (beta <= tol * bnorm) { info->status = 0; break; }
        if (info->iters >= max_iters) break;
        if (beta >= 0.999 * prev_cycle_res) break;          /* stagnation across restarts */
        prev_cycle_res = beta;
        if (info->iters > 0) info->restarts++;
        vscale_copy(F, 1.0 / beta, &r, &V[0]);
        memset(gv, 0, sizeof(double) * (m + 1));
        gv[0] = beta;
        int j, nj = 0;
        for (j = 0; j < m && info->iters < max_iters; ++j) {
            precond(H, &V[j], &Z[j]);
            double *zi[4] = {Z[j].f[0], Z[j].f[1], Z[j].f[2], Z[j].f[3]};
            double *wo[4] = {w.f[0], w.f[1], w.f[2], w.f[3]};
            apply_K(F, H->dt, H->theta, zi, wo);
            for (int i = 0; i <= j; ++i) {          /* modified Gram-Schmidt */
                HH(i, j) = vdot(F, &w, &V[i], w2);
                vaxpy(F, -HH(i, j), &V[i], &w);
            }
            double hn = sqrt(vdot(F, &w, &w, w2));
            HH(j + 1, j) = hn;
            if (hn > 0.0) vscale_copy(F, 1.0 / hn, &w, &V[j + 1]);
            for (int i = 0; i < j; ++i) {           /* previous rotations */
                double t = cs[i] * HH(i, j) + sn[i] * HH(i + 1, j);
                HH(i + 1, j) = -sn[i] * HH(i, j) + cs[i] * HH(i + 1, j);
                HH(i, j) = t;
            }
            double a = HH(j, j), bb = HH(j + 1, j);
            double den = sqrt(a * a + bb * bb);
            cs[j] = den > 0.0 ? a / den : 1.0;
            sn[j] = den > 0.0 ? bb / den : 0.0;
            HH(j, j) = den;
            HH(j + 1, j) = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            info->iters++;
            nj = j + 1;
            info->rel_res_est = fabs(gv[j + 1]) / bnorm;
            if (fabs(gv[j + 1]) <= tol * bnorm || hn == 0.0) break;
        }
        /* least squares: upper-triangular solve */
        for (int i = nj - 1; i >= 0; --i) {
            double s = gv[i];
            for (int k = i + 1; k < nj; ++k) s -= HH(i, k) * y[k];
            y[i] = HH(i, i) != 0.0 ? s / HH(i, i) : 0.0;
        }
        for (int i = 0; i < nj; ++i) vaxpy(F, y[i], &Z[i], x);
        sub_mean(&F->g, x->f[3]);
    }
done:
    for (int j = 0; j <= m; ++j) vfree(&V[j]);
    for (int j = 0; j < m; ++j) vfree(&Z[j]);
    vfree(&w); vfree(&r);
    free(V); free(Z); free(Hm); free(cs); free(sn); free(gv); free(y);
#undef HH
}

/* ------------------------------------------------------ exported API */
static double wall_seconds(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

static int make_grid(Grid *g, int dim, const int *n, const double *h) {
    if (dim != 2 && dim != 3) return -1;
    g->dim = dim;
    g->nx = n[0]; g->ny = n[1]; g->nz = dim == 3 ? n[2] : 1;
    g->hx = h[0]; g->hy = h[1]; g->hz = dim == 3 ? h[2] : h[0];
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return -1;
    return 0;
}

/* y = K x.  x[4], y[4]: u, v, w (NULL in 2D), p in the layout above. */
int oracle_apply(int dim, const int *n, const double *h, double dt, double theta,
                 double *const rho[3], const double *mu, double *const x[4], double *const y[4]) {
    Grid g;
    if (make_grid(&g, dim, n, h)) return -1;
    Level L;
    memset(&L, 0, sizeof(L));
    L.g = g;
    L.nu = n_u(&g); L.nv = n_v(&g); L.nw = n_w(&g); L.nc = n_c(&g);
    for (int a = 0; a < 3; ++a) L.rho[a] = a < dim ? rho[a] : NULL;
    L.mu = (double *)mu;
    L.mxy = calloc((long)(g.nx + 1) * (g.ny + 1) * g.nz, sizeof(double));
    if (dim == 3) {
        L.mxz = calloc((long)(g.nx + 1) * g.ny * (g.nz + 1), sizeof(double));
        L.myz = calloc((long)g.nx * (g.ny + 1) * (g.nz + 1), sizeof(double));
    }
    edge_viscosity(&g, L.mu, L.mxy, L.mxz, L.myz);
    apply_K(&L, dt, theta, x, y);
    free(L.mxy); free(L.mxz); free(L.myz);
    return 0;
}

/* The continuity weight auto_sigma picks for these coefficients (*out). */
int oracle_auto_sigma(int dim, const int *n, const double *h, double dt, double theta,
                      double *const rho[3], const double *mu, double *out) {
    Grid g;
    if (make_grid(&g, dim, n, h)) return -1;
    Level L;
    memset(&L, 0, sizeof(L));
    L.g = g;
    L.nu = n_u(&g); L.nv = n_v(&g); L.nw = n_w(&g); L.nc = n_c(&g);
    for (int a = 0; a < 3; ++a) L.rho[a] = a < dim ? rho[a] : NULL;
    L.mu = (double *)mu;
    *out = auto_sigma(&L, dt, theta);
    return 0;
}

/* Solve K x = (f, g) to ||b - K x||_s <= tol ||b||_s, where ||(a, c)||_s^2 =
 * ||a||^2 + sigma^2 ||c||^2 weights the continuity rows (cont_scale > 0 gives
 * sigma; 0 picks auto_sigma; 1 is the plain 2-norm).  x holds the initial guess
 * on entry and the solution on exit (zero-mean p).  opts: restart, max_iters,
 * nu1, nu2, vel_cycles, p_cycles, coarse_sweeps.  out: iters, restarts, status,
 * rel_res_est, rel_res_true, mean removed from g, levels, sigma, setup seconds,
 * FGMRES seconds (out needs 10 entries). */
int oracle_solve(int dim, const int *n, const double *h, double dt, double theta,
                 double *const rho[3], const double *mu, double *const f[4], double tol,
                 const int *opts, double cont_scale, double *const x[4], double *out) {
    Grid g;
    if (make_grid(&g, dim, n, h)) return -1;
    double t0 = wall_seconds();
    Hier *H = calloc(1, sizeof(Hier));
    H->dt = dt; H->theta = theta;
    H->nu1 = opts[2]; H->nu2 = opts[3];
    H->vel_cycles = opts[4]; H->p_cycles = opts[5]; H->coarse_sweeps = opts[6];
    hier_build(H, &g, rho, mu);
    Level *F = &H->L[0];
    Vec b = vnew(F), xv = vnew(F);
    for (int c = 0; c < 4; ++c) {
        long m = vlen(F, c);
        if (m == 0) continue;
        memcpy(b.f[c], f[c], sizeof(double) * m);
        memcpy(xv.f[c], x[c], sizeof(double) * m);
    }
    /* wall-normal faces are not unknowns: zero them in b and x */
    for (int k = 0; k < g.nz; ++k) for (int j = 0; j < g.ny; ++j) {
        b.f[0][IU(&g, 0, j, k)] = b.f[0][IU(&g, g.nx, j, k)] = 0.0;
        xv.f[0][IU(&g, 0, j, k)] = xv.f[0][IU(&g, g.nx, j, k)] = 0.0;
    }
    for (int k = 0; k < g.nz; ++k) for (int i = 0; i < g.nx; ++i) {
        b.f[1][IV(&g, i, 0, k)] = b.f[1][IV(&g, i, g.ny, k)] = 0.0;
        xv.f[1][IV(&g, i, 0, k)] = xv.f[1][IV(&g, i, g.ny, k)] = 0.0;
    }
    if (dim == 3) for (int j = 0; j < g.ny; ++j) for (int i = 0; i < g.nx; ++i) {
        b.f[2][IW(&g, i, j, 0)] = b.f[2][IW(&g, i, j, g.nz)] = 0.0;
        xv.f[2][IW(&g, i, j, 0)] = xv.f[2][IW(&g, i, j, g.nz)] = 0.0;
    }
    double gm = mean_c(&g, b.f[3]);
    sub_mean(&g, b.f[3]);
    SolveInfo info;
    memset(&info, 0, sizeof(info));
    double sigma = cont_scale > 0.0 ? cont_scale : auto_sigma(F, dt, theta);
    double t1 = wall_seconds();
    fgmres(H, &b, &xv, tol, opts[0], opts[1], sigma * sigma, &info);
    double t2 = wall_seconds();
    for (int c = 0; c < 4; ++c) {
        long m = vlen(F, c);
        if (m == 0) continue;
        memcpy(x[c], xv.f[c], sizeof(double) * m);
    }
    out[0] = info.iters; out[1] = info.restarts; out[2] = info.status;
    out[3] = info.rel_res_est; out[4] = info.rel_res_true; out[5] = gm; out[6] = H->nlev;
    out[7] = sigma;
    out[8] = t1 - t0;      /* setup seconds (hierarchy, copies) */
    out[9] = t2 - t1;      /* FGMRES seconds */
    vfree(&b); vfree(&xv);
    hier_free(H);
    free(H);
    return 0;
}

/* Apply the projection preconditioner once (for tests of its algebra). */
int oracle_precond(int dim, const int *n, const double *h, double dt, double theta,
                   double *const rho[3], const double *mu, const int *opts,
                   double *const r[4], double *const z[4]) {
    Grid g;
    if (make_grid(&g, dim, n, h)) return -1;
    Hier *H = calloc(1, sizeof(Hier));
    H->dt = dt; H->theta = theta;
    H->nu1 = opts[2]; H->nu2 = opts[3];
    H->vel_cycles = opts[4]; H->p_cycles = opts[5]; H->coarse_sweeps = opts[6];
    hier_build(H, &g, rho, mu);
    Level *F = &H->L[0];
    Vec rv = vnew(F), zv = vnew(F);
    for (int c = 0; c < 4; ++c) {
        long m = vlen(F, c);
        if (m) memcpy(rv.f[c], r[c], sizeof(double) * m);
    }
    precond(H, &rv, &zv);
    for (int c = 0; c < 4; ++c) {
        long m = vlen(F, c);
        if (m) memcpy(z[c], zv.f[c], sizeof(double) * m);
    }
    vfree(&rv); vfree(&zv);
    hier_free(H);
    free(H);
    return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* OpenMP threads of the following calls (n < 1: leave unchanged). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
