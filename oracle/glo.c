/*
 * glo.c -- CPU FP64 oracle for the oblate-planet transit light curve.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library.  Plain C, IEEE FP64,
 * round-to-nearest, built with floating-point contraction off.
 *
 * The quantity (Section 2, "Ellipsoid Transit Model", and its limb-darkening
 * paragraph): the limb-darkening-weighted area of the stellar disk covered by
 * the projected ellipse, divided by the total weighted area of the disk.  The
 * paper evaluates it as Green's-theorem line integrals; Green's theorem turns
 * those back into exactly this area integral, which is what is written out
 * here, with no boundary integral, no intersection quartic and no shared
 * geometry with the GPU path.
 *
 * Readings of the paper this oracle rests on (each one is a choice the paper
 * leaves open):
 *  - The intensity law is the quadratic one, I = 1 - u1(1-mu) - u2(1-mu)^2,
 *    normalised by its integral over the disk (the paper names only the three
 *    Green's integrands and never states the normalisation).
 *  - k is the equatorial radius ratio, the polar radius is k(1-f) (eq. 1).
 *  - theta is the angle between the spin axis and the line of sight, i.e. the
 *    paper's eta = pi/2 - theta; phi is the paper's xi; zeta = 0 for an
 *    oblate spheroid (Appendix A: b = c, the third angle drops out).
 *  - The orbit is circular, alpha = 2 pi (t - t0)/P is the mean anomaly and
 *    sin(beta) = b/d with d = a/R* (Section 2, eq. coord-map).
 *  - The planet occults only when it is on the observer's side (z < 0).
 *  - Exposure smearing is a box average over n_ss midpoint sub-samples.
 *
 * Method (the plain definition as an iterated integral):
 *   In the ellipse frame p = c + w u_hat + v s_hat, the ellipse is
 *   (w/k)^2 + (v/kq)^2 <= 1.  Outer variable psi in [-pi/2, pi/2] with
 *   w = k sin(psi); for each psi the ellipse chord in v is intersected with
 *   the disk chord (limits clipped, never an indicator function) and the
 *   integral of I along the clipped chord is taken in closed form (or, in the
 *   cross-check mode, by adaptive quadrature).  The outer integral is global
 *   adaptive Gauss-Legendre (10/20-point pairs, bisection of the panel with the
 *   largest error estimate), split beforehand at every kink of the integrand:
 *   where an active chord limit switches between ellipse and circle, where the
 *   clipped chord closes, and where the disk chord itself appears.
 */
#include "glo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rules on [-1, 1], computed once by Newton's method on the  */
/* three-term Legendre recurrence (textbook construction).                   */
/* ------------------------------------------------------------------------ */
#define NLO 10
#define NHI 20
static double gl_lo_x[NLO], gl_lo_w[NLO];
static double gl_hi_x[NHI], gl_hi_w[NHI];

static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; i++) {
        long double z = cosl((long double)M_PI * (i + 0.75L) / (n + 0.5L));
        long double dp = 1.0L;
        for (int it = 0; it < 200; it++) {
            long double p0 = 1.0L, p1 = z;
            for (int j = 2; j <= n; j++) {
                long double p2 = ((2.0L * j - 1.0L) * z * p1 - (j - 1.0L) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) {
                /* recompute the derivative at the converged node */
                p0 = 1.0L;
                p1 = z;
                for (int j = 2; j <= n; j++) {
                    long double p2 = ((2.0L * j - 1.0L) * z * p1 - (j - 1.0L) * p0) / j;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0L);
                break;
            }
        }
        x[i] = (double)z;
        w[i] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
    }
}

__attribute__((constructor)) static void glo_init(void)
{
    gauss_legendre(NLO, gl_lo_x, gl_lo_w);
    gauss_legendre(NHI, gl_hi_x, gl_hi_w);
}

/* ------------------------------------------------------------------------ */
/* Global adaptive quadrature of f over [a, b] to absolute tolerance tol.    */
/* ------------------------------------------------------------------------ */
typedef double (*glo_fn)(double x, const void *ctx);

typedef struct {
    double a, b, val, err;
} panel;

static void rule_pair(glo_fn f, const void *ctx, double a, double b,
                      double *val, double *err)
{
    double m = 0.5 * (a + b), h = 0.5 * (b - a);
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < NLO; i++) lo += gl_lo_w[i] * f(m + h * gl_lo_x[i], ctx);
    for (int i = 0; i < NHI; i++) hi += gl_hi_w[i] * f(m + h * gl_hi_x[i], ctx);
    *val = h * hi;
    *err = fabs(h * (hi - lo));
}

#define MAXPANEL 6000

/* integrals that stopped at MAXPANEL panels (or at panels too narrow to
 * split) with their error estimate still above the target; reported by
 * glo_unconverged so that a test can require none */
static long glo_n_unconverged = 0;

static double adapt(glo_fn f, const void *ctx, double a, double b, double tol)
{
    if (!(b > a)) return 0.0;
    panel *P = (panel *)malloc(sizeof(panel) * MAXPANEL);
    int n = 1;
    P[0].a = a;
    P[0].b = b;
    rule_pair(f, ctx, a, b, &P[0].val, &P[0].err);
    for (;;) {
        double etot = 0.0;
        int worst = 0;
        for (int i = 0; i < n; i++) {
            etot += P[i].err;
            if (P[i].err > P[worst].err) worst = i;
        }
        if (etot <= tol) break;
        double pa = P[worst].a, pb = P[worst].b, pm = 0.5 * (pa + pb);
        if (n + 1 >= MAXPANEL || !(pm > pa && pm < pb)) {
            /* out of panels, or the worst panel cannot be split further */
#ifdef _OPENMP
#pragma omp atomic
#endif
            glo_n_unconverged++;
            break;
        }
        P[worst].b = pm;
        rule_pair(f, ctx, pa, pm, &P[worst].val, &P[worst].err);
        P[n].a = pm;
        P[n].b = pb;
        rule_pair(f, ctx, pm, pb, &P[n].val, &P[n].err);
        n++;
    }
    /* sum in ascending order of the panel's left end for reproducibility */
    double s = 0.0;
    for (int i = 0; i < n; i++) s += P[i].val;
    free(P);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Limb darkening                                                            */
/* ------------------------------------------------------------------------ */
int glo_kipping(double q1, double q2, double *u1, double *u2)
{
    if (!(q1 >= 0.0 && q1 <= 1.0 && q2 >= 0.0 && q2 <= 1.0)) return -1;
    double s = sqrt(q1);
    *u1 = 2.0 * s * q2;
    *u2 = s * (1.0 - 2.0 * q2);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Geometry (Section 2, eq. coord-map and the rotation matrices)             */
/* ------------------------------------------------------------------------ */
static void mat3_mul(const double A[3][3], const double B[3][3], double C[3][3])
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int m = 0; m < 3; m++) s += A[i][m] * B[m][j];
            C[i][j] = s;
        }
}

static void rot_x(double a, double R[3][3])
{
    double c = cos(a), s = sin(a);
    double M[3][3] = {{1, 0, 0}, {0, c, -s}, {0, s, c}};
    memcpy(R, M, sizeof(M));
}

static void rot_y(double a, double R[3][3])
{
    double c = cos(a), s = sin(a);
    double M[3][3] = {{c, 0, s}, {0, 1, 0}, {-s, 0, c}};
    memcpy(R, M, sizeof(M));
}

static void rot_z(double a, double R[3][3])
{
    double c = cos(a), s = sin(a);
    double M[3][3] = {{c, -s, 0}, {s, c, 0}, {0, 0, 1}};
    memcpy(R, M, sizeof(M));
}

int glo_geometry(const double p[GLO_NPARAM], double t, double out[9])
{
    const double k = p[GLO_K], f = p[GLO_F], theta = p[GLO_THETA];
    const double phi = p[GLO_PHI], b = p[GLO_B], d = p[GLO_ARS];
    const double P = p[GLO_P], t0 = p[GLO_T0];

    /* orbit: the planet centre x solves R(x + Ry(-beta) Rx(alpha) (0,0,d)) = 0 */
    double alpha = 2.0 * M_PI * (t - t0) / P;
    double beta = asin(b / d);
    double Ry[3][3], Rx[3][3], Rb[3][3];
    rot_y(-beta, Ry);
    rot_x(alpha, Rx);
    mat3_mul(Ry, Rx, Rb);
    double xc = -Rb[0][2] * d, yc = -Rb[1][2] * d, zc = -Rb[2][2] * d;

    /* spin (polar) axis in the observer frame: the body x' axis, i.e. the
     * first row of R(zeta=0, eta, xi) = Rx(0) Ry(eta) Rz(xi) */
    double eta = 0.5 * M_PI - theta;
    double Re[3][3], Rz[3][3], R0[3][3], R[3][3];
    rot_y(eta, Re);
    rot_z(phi, Rz);
    rot_x(0.0, R0);
    double T[3][3];
    mat3_mul(Re, Rz, T);
    mat3_mul(R0, T, R);
    double nx = R[0][0], ny = R[0][1], nz = R[0][2];

    /* orthographic silhouette of a spheroid with equatorial radius k and
     * polar radius k(1-f) along n: semi-axis k perpendicular to the projected
     * axis, sqrt(k^2 nz^2 + (k(1-f))^2 (1 - nz^2)) along it */
    double ap = k * (1.0 - f);
    double along = sqrt(k * k * nz * nz + ap * ap * (nx * nx + ny * ny));
    double nxy = sqrt(nx * nx + ny * ny);
    double sx = 1.0, sy = 0.0;
    if (nxy > 0.0) {
        sx = nx / nxy;
        sy = ny / nxy;
    }
    out[0] = xc;
    out[1] = yc;
    out[2] = zc;
    out[3] = -sy; /* u_hat: s_hat turned by +90 degrees */
    out[4] = sx;
    out[5] = sx; /* s_hat: projected spin axis */
    out[6] = sy;
    out[7] = k;
    out[8] = along;
    return zc < 0.0 ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Occulted fraction as an iterated area integral                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    double k, kq;       /* ellipse semi-axes along u_hat and s_hat */
    double cu, cs;      /* star-centre offsets: c.u_hat, c.s_hat (c = ellipse centre) */
    double c0, c1, c2;  /* I(r) = c0 + c1 mu + c2 r^2 */
    int mode;
    double tol_inner;
} occ_ctx;

/* integral over s in [sL, sU] of I along a chord at distance h from the star
 * centre, s measured from the foot of the perpendicular, R2 = 1 - h^2 */
static double chord_closed(const occ_ctx *c, double h, double R2, double sL, double sU)
{
    double R = sqrt(R2);
    /* R^2 - s^2 as (R - s)(R + s) with the same rounded R that clipped the
     * chord, so a limit on the limb gives exactly zero rather than the square
     * root of a rounding residue */
    double rL = (R - sL) * (R + sL), rU = (R - sU) * (R + sU);
    if (rL < 0.0) rL = 0.0;
    if (rU < 0.0) rU = 0.0;
    rL = sqrt(rL);
    rU = sqrt(rU);
    /* antiderivative of sqrt(R^2 - s^2): (s sqrt(R^2 - s^2) + R^2 asin(s/R))/2,
     * with asin(s/R) = atan2(s, sqrt(R^2 - s^2)) so that both terms use the
     * same rounded square root near the limb */
    double mu_int = 0.5 * ((sU * rU + R2 * atan2(sU, rU)) - (sL * rL + R2 * atan2(sL, rL)));
    double len = sU - sL;
    double r2_int = h * h * len + (sU * sU * sU - sL * sL * sL) / 3.0;
    return c->c0 * len + c->c1 * mu_int + c->c2 * r2_int;
}

typedef struct {
    const occ_ctx *c;
    double h2;
} chord_ctx;

static double intensity_on_chord(double s, const void *vp)
{
    const chord_ctx *q = (const chord_ctx *)vp;
    double r2 = q->h2 + s * s;
    double mu2 = 1.0 - r2;
    double mu = mu2 > 0.0 ? sqrt(mu2) : 0.0;
    return q->c->c0 + q->c->c1 * mu + q->c->c2 * r2;
}

/* clipped chord at outer abscissa psi; returns 0 when empty */
static int chord_limits(const occ_ctx *c, double psi, double *h, double *R2,
                        double *sL, double *sU)
{
    double w = c->k * sin(psi);
    double half = c->kq * cos(psi);
    if (half < 0.0) half = 0.0;
    double hh = c->cu + w;
    if (!(fabs(hh) < 1.0)) return 0;
    double r2 = (1.0 - hh) * (1.0 + hh);
    double R = sqrt(r2);
    /* chord coordinate s = cs + v: ellipse gives v in [-half, half],
     * disk gives s in [-R, R] */
    double lo = c->cs - half, hi = c->cs + half;
    if (lo < -R) lo = -R;
    if (hi > R) hi = R;
    if (!(hi > lo)) return 0;
    *h = hh;
    *R2 = r2;
    *sL = lo;
    *sU = hi;
    return 1;
}

static double outer_integrand(double psi, const void *vp)
{
    const occ_ctx *c = (const occ_ctx *)vp;
    double h, R2, sL, sU;
    if (!chord_limits(c, psi, &h, &R2, &sL, &sU)) return 0.0;
    double v;
    if (c->mode == GLO_INNER_CLOSED) {
        v = chord_closed(c, h, R2, sL, sU);
    } else {
        chord_ctx q = {c, h * h};
        v = adapt(intensity_on_chord, &q, sL, sU, c->tol_inner);
    }
    return v * c->k * cos(psi);
}

/* the four limit-crossing functions whose zeros are kinks of the integrand:
 * ellipse upper/lower limit against disk upper/lower limit (s coordinates) */
static int kink_values(const occ_ctx *c, double psi, double e[4])
{
    double w = c->k * sin(psi);
    double half = c->kq * cos(psi);
    double hh = c->cu + w;
    /* the disk chord exists for |hh| <= 1; a point at the disk's vertical
     * tangent (a scan abscissa there, up to its rounding) has R = 0 */
    if (!(fabs(hh) <= 1.0 + 1e-12)) return 0;
    double r2 = (1.0 - hh) * (1.0 + hh);
    double R = r2 > 0.0 ? sqrt(r2) : 0.0;
    double eU = c->cs + half, eL = c->cs - half;
    e[0] = eU - R;
    e[1] = eL + R;
    e[2] = eU + R;
    e[3] = eL - R;
    return 1;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

#define NGRID 1024
#define MAXBRK 64

/* zero of limit-crossing function j in [a, b], where it changes sign (fa: its
 * value at a), by bisection */
static double kink_bisect(const occ_ctx *c, int j, double a, double b, double fa)
{
    for (int it = 0; it < 80; it++) {
        double m = 0.5 * (a + b), em[4];
        if (!kink_values(c, m, em)) break;
        if ((em[j] < 0.0) == (fa < 0.0)) {
            a = m;
            fa = em[j];
        } else {
            b = m;
        }
    }
    return 0.5 * (a + b);
}

/* golden-section search on [a, b] for the point where dir * (function j) is
 * smallest (dir = +1: its minimum, -1: its maximum) */
static double kink_extremum(const occ_ctx *c, int j, double a, double b, double dir)
{
    const double g = 0.6180339887498949; /* (sqrt(5) - 1)/2 */
    double x1 = b - g * (b - a), x2 = a + g * (b - a), e1[4], e2[4];
    double f1 = kink_values(c, x1, e1) ? dir * e1[j] : HUGE_VAL;
    double f2 = kink_values(c, x2, e2) ? dir * e2[j] : HUGE_VAL;
    for (int it = 0; it < 90; it++) {
        if (f1 < f2) {
            b = x2;
            x2 = x1;
            f2 = f1;
            x1 = b - g * (b - a);
            f1 = kink_values(c, x1, e1) ? dir * e1[j] : HUGE_VAL;
        } else {
            a = x1;
            x1 = x2;
            f1 = f2;
            x2 = a + g * (b - a);
            f2 = kink_values(c, x2, e2) ? dir * e2[j] : HUGE_VAL;
        }
    }
    return 0.5 * (a + b);
}

double glo_occulted(double cx, double cy, double ux, double uy, double k,
                    double q, double u1, double u2, double tol, int mode)
{
    if (cx * cx + cy * cy >= (1.0 + k) * (1.0 + k)) return 0.0;
    occ_ctx c;
    c.k = k;
    c.kq = k * q;
    c.cu = cx * ux + cy * uy;  /* c . u_hat */
    c.cs = cx * uy - cy * ux;  /* c . s_hat, s_hat = (uy, -ux) */
    c.c0 = 1.0 - u1 - 2.0 * u2;
    c.c1 = u1 + 2.0 * u2;
    c.c2 = u2;
    c.mode = mode;
    double Phi = M_PI * (1.0 - u1 / 3.0 - u2 / 6.0);
    double tol_abs = tol * fabs(Phi);
    c.tol_inner = tol_abs * 1e-2;

    /* breakpoints */
    double brk[MAXBRK];
    int nb = 0;
    brk[nb++] = -0.5 * M_PI;
    brk[nb++] = 0.5 * M_PI;
    for (int sgn = -1; sgn <= 1; sgn += 2) {
        double sv = (sgn - c.cu) / k;
        if (sv > -1.0 && sv < 1.0) brk[nb++] = asin(sv);
    }
    /* sign scan of the four limit-crossing functions on a grid; a sign change
     * in a cell is refined by bisection.  Two zeros inside one cell (a
     * near-tangency) leave no sign change, so wherever a function has a
     * local extremum between three grid points without a sign change there,
     * the extremum is located and, if it lies across zero, both zeros are
     * refined. */
    /* scan abscissae: the uniform grid and the disk's vertical tangents (the
     * ends of the range where the disk chord exists), so that a zero between
     * the last grid point and such an end is seen as a sign change */
    double scan[NGRID + 3];
    int ns = 0;
    for (int i = 0; i <= NGRID; i++) scan[ns++] = -0.5 * M_PI + M_PI * (double)i / NGRID;
    for (int i = 2; i < nb; i++) scan[ns++] = brk[i];
    qsort(scan, (size_t)ns, sizeof(double), cmp_double);
    double pp_psi = 0.0, prev_psi = 0.0, pp_e[4], prev_e[4];
    int pp_ok = 0, prev_ok = 0;
    for (int i = 0; i < ns && nb < MAXBRK - 8; i++) {
        double psi = scan[i];
        double e[4];
        int ok = kink_values(&c, psi, e);
        if (ok && prev_ok) {
            for (int j = 0; j < 4 && nb < MAXBRK - 4; j++) {
                if ((prev_e[j] < 0.0) != (e[j] < 0.0)) {
                    brk[nb++] = kink_bisect(&c, j, prev_psi, psi, prev_e[j]);
                } else if (pp_ok && (pp_e[j] < 0.0) == (prev_e[j] < 0.0) &&
                           (prev_e[j] - pp_e[j]) * (e[j] - prev_e[j]) < 0.0) {
                    /* extremum near prev_psi: pull it toward zero */
                    double dir = (prev_e[j] < 0.0) ? -1.0 : 1.0;
                    double ps = kink_extremum(&c, j, pp_psi, psi, dir);
                    double es[4];
                    if (kink_values(&c, ps, es) && (es[j] < 0.0) != (prev_e[j] < 0.0)) {
                        brk[nb++] = kink_bisect(&c, j, pp_psi, ps, pp_e[j]);
                        brk[nb++] = kink_bisect(&c, j, ps, psi, es[j]);
                    }
                }
            }
        }
        pp_ok = prev_ok;
        pp_psi = prev_psi;
        if (prev_ok) memcpy(pp_e, prev_e, sizeof(e));
        prev_ok = ok;
        prev_psi = psi;
        if (ok) memcpy(prev_e, e, sizeof(e));
    }
    qsort(brk, (size_t)nb, sizeof(double), cmp_double);

    double total = 0.0;
    for (int i = 0; i + 1 < nb; i++) {
        double a = brk[i], b = brk[i + 1];
        if (!(b > a)) continue;
        total += adapt(outer_integrand, &c, a, b, tol_abs * (b - a) / M_PI);
    }
    return total / Phi;
}

/* ------------------------------------------------------------------------ */
/* Flux                                                                      */
/* ------------------------------------------------------------------------ */
static int params_ok(const double p[GLO_NPARAM])
{
    for (int i = 0; i < GLO_NPARAM; i++)
        if (!isfinite(p[i])) return 0;
    const double k = p[GLO_K], f = p[GLO_F], d = p[GLO_ARS];
    if (!(k > 0.0 && k < 1.0)) return 0;
    if (!(f >= 0.0 && f < 1.0)) return 0;
    if (!(d > 1.0 + k)) return 0;
    if (!(fabs(p[GLO_B]) < d)) return 0;
    if (!(p[GLO_P] > 0.0)) return 0;
    if (!(p[GLO_Q1] >= 0.0 && p[GLO_Q1] <= 1.0)) return 0;
    if (!(p[GLO_Q2] >= 0.0 && p[GLO_Q2] <= 1.0)) return 0;
    return 1;
}

static double flux_instant(const double p[GLO_NPARAM], double u1, double u2,
                           double t, double tol)
{
    double g[9];
    if (!glo_geometry(p, t, g)) return 1.0;
    double q = g[8] / g[7];
    double delta = glo_occulted(g[0], g[1], g[3], g[4], g[7], q, u1, u2, tol,
                                GLO_INNER_CLOSED);
    return 1.0 - delta;
}

int glo_flux(const double p[GLO_NPARAM], double t, double t_exp, int n_ss,
             double tol, double *out)
{
    double u1, u2;
    if (!params_ok(p) || !isfinite(t) || !isfinite(t_exp) || t_exp < 0.0 ||
        n_ss < 1 || n_ss > 64 || glo_kipping(p[GLO_Q1], p[GLO_Q2], &u1, &u2)) {
        *out = NAN;
        return -1;
    }
    double sum = 0.0;
    for (int j = 0; j < n_ss; j++) {
        double tj = t + (((double)j + 0.5) / (double)n_ss - 0.5) * t_exp;
        sum += flux_instant(p, u1, u2, tj, tol);
    }
    *out = sum / (double)n_ss;
    return 0;
}

static void gather_params(const double *params, int64_t n_sets, int64_t s,
                          double p[GLO_NPARAM])
{
    for (int i = 0; i < GLO_NPARAM; i++) p[i] = params[(int64_t)i * n_sets + s];
}

static int64_t set_of_index(const int64_t *offsets, int64_t n_sets,
                            int64_t n_times, int64_t idx)
{
    if (!offsets) return idx / n_times;
    int64_t lo = 0, hi = n_sets; /* offsets[lo] <= idx < offsets[hi] */
    while (hi - lo > 1) {
        int64_t m = (lo + hi) / 2;
        if (offsets[m] <= idx) lo = m;
        else hi = m;
    }
    return lo;
}

int64_t glo_flux_select(const double *params, int64_t n_sets,
                        const double *times, const int64_t *offsets,
                        int64_t n_times, const int32_t *n_ss,
                        const double *t_exp, double tol, const int64_t *sel,
                        int64_t n_sel, double *out_sel, int nthreads)
{
    int64_t nerr = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads) reduction(+ : nerr)
#endif
    for (int64_t i = 0; i < n_sel; i++) {
        int64_t idx = sel[i];
        int64_t s = set_of_index(offsets, n_sets, n_times, idx);
        double p[GLO_NPARAM];
        gather_params(params, n_sets, s, p);
        double t = offsets ? times[idx] : times[idx % n_times];
        int nss = n_ss ? n_ss[s] : 1;
        double te = t_exp ? t_exp[s] : 0.0;
        if (glo_flux(p, t, te, nss, tol, &out_sel[i])) nerr++;
    }
    return nerr;
}

int64_t glo_flux_batch(const double *params, int64_t n_sets,
                       const double *times, const int64_t *offsets,
                       int64_t n_times, const int32_t *n_ss,
                       const double *t_exp, double tol, double *out,
                       int nthreads)
{
    int64_t nerr = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : nerr)
#endif
    for (int64_t s = 0; s < n_sets; s++) {
        double p[GLO_NPARAM];
        gather_params(params, n_sets, s, p);
        int64_t a = offsets ? offsets[s] : s * n_times;
        int64_t b = offsets ? offsets[s + 1] : (s + 1) * n_times;
        int nss = n_ss ? n_ss[s] : 1;
        double te = t_exp ? t_exp[s] : 0.0;
        for (int64_t i = a; i < b; i++) {
            double t = offsets ? times[i] : times[i - a];
            if (glo_flux(p, t, te, nss, tol, &out[i])) nerr++;
        }
    }
    return nerr;
}

/* ------------------------------------------------------------------------ */
/* General ellipsoids (a, b, c; angles zeta, eta, xi), optionally tidally   */
/* locked                                                                    */
/* ------------------------------------------------------------------------ */
/* Silhouette as the Schur complement of the body quadric: with M the
 * rotation from observer offsets y = x - x_c to body coordinates
 * (x' = M y; Section 2 eq. coord-map gives M = R(zeta, eta, xi), the
 * tidally-locked map of Appendix B gives M = R(zeta, eta, xi) Rx(-alpha)
 * Ry(beta)), the ellipsoid is y^T Q y <= 1 with Q = M^T diag(a^-2, b^-2,
 * c^-2) M, and its orthographic shadow on the sky plane is u^T S u <= 1 with
 * S = Q_xy,xy - Q_xy,z Q_zz^-1 Q_z,xy.  The shadow's semi-axes and the
 * direction of the major one come from the eigen-decomposition of S.  (The
 * GPU path uses the paper's parametric eqs. dx, dy1, dy2 instead.) */
static int ell_params_ok(const double p[GLO_E_NPARAM])
{
    for (int i = 0; i < GLO_E_NPARAM; i++)
        if (!isfinite(p[i])) return 0;
    double amax = 0.0;
    for (int i = GLO_E_RA; i <= GLO_E_RC; i++) {
        if (!(p[i] > 0.0 && p[i] < 1.0)) return 0;
        if (p[i] > amax) amax = p[i];
    }
    const double d = p[GLO_E_ARS];
    if (!(d > 1.0 + amax)) return 0;
    if (!(fabs(p[GLO_E_B]) < d)) return 0;
    if (!(p[GLO_E_P] > 0.0)) return 0;
    if (!(p[GLO_E_Q1] >= 0.0 && p[GLO_E_Q1] <= 1.0)) return 0;
    if (!(p[GLO_E_Q2] >= 0.0 && p[GLO_E_Q2] <= 1.0)) return 0;
    if (!(p[GLO_E_LOCKED] == 0.0 || p[GLO_E_LOCKED] == 1.0)) return 0;
    return 1;
}

int glo_geometry_ell(const double p[GLO_E_NPARAM], double t, double out[9])
{
    const double b = p[GLO_E_B], d = p[GLO_E_ARS], P = p[GLO_E_P], t0 = p[GLO_E_T0];
    double alpha = 2.0 * M_PI * (t - t0) / P;
    double beta = asin(b / d);
    double Ry[3][3], Rx[3][3], Rb[3][3];
    rot_y(-beta, Ry);
    rot_x(alpha, Rx);
    mat3_mul(Ry, Rx, Rb);
    double xc = -Rb[0][2] * d, yc = -Rb[1][2] * d, zc = -Rb[2][2] * d;

    double Rzeta[3][3], Reta[3][3], Rxi[3][3], T[3][3], M[3][3];
    rot_x(p[GLO_E_ZETA], Rzeta);
    rot_y(p[GLO_E_ETA], Reta);
    rot_z(p[GLO_E_XI], Rxi);
    mat3_mul(Reta, Rxi, T);
    mat3_mul(Rzeta, T, M); /* R(zeta, eta, xi) */
    if (p[GLO_E_LOCKED] != 0.0) {
        double Rma[3][3], Rpb[3][3], L[3][3], M2[3][3];
        rot_x(-alpha, Rma);
        rot_y(beta, Rpb);
        mat3_mul(Rma, Rpb, L);
        mat3_mul(M, L, M2);
        memcpy(M, M2, sizeof(M));
    }
    const double inv2[3] = {1.0 / (p[GLO_E_RA] * p[GLO_E_RA]), 1.0 / (p[GLO_E_RB] * p[GLO_E_RB]),
                            1.0 / (p[GLO_E_RC] * p[GLO_E_RC])};
    double Q[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += M[k][i] * inv2[k] * M[k][j];
            Q[i][j] = acc;
        }
    const double s11 = Q[0][0] - Q[0][2] * Q[2][0] / Q[2][2];
    const double s12 = Q[0][1] - Q[0][2] * Q[2][1] / Q[2][2];
    const double s22 = Q[1][1] - Q[1][2] * Q[2][1] / Q[2][2];
    const double half_tr = 0.5 * (s11 + s22);
    const double rad = hypot(0.5 * (s11 - s22), s12);
    const double lo = half_tr - rad, hi = half_tr + rad; /* lo: major axis */
    /* eigenvector of the smaller eigenvalue, from the better-conditioned row */
    double ux, uy;
    if (rad == 0.0) {
        ux = 1.0;
        uy = 0.0;
    } else if (fabs(s11 - lo) >= fabs(s22 - lo)) {
        ux = -s12;
        uy = s11 - lo;
    } else {
        ux = s22 - lo;
        uy = -s12;
    }
    const double nu = hypot(ux, uy);
    ux /= nu;
    uy /= nu;
    out[0] = xc;
    out[1] = yc;
    out[2] = zc;
    out[3] = ux; /* u_hat: major axis */
    out[4] = uy;
    out[5] = uy; /* s_hat = (uy, -ux): minor axis */
    out[6] = -ux;
    out[7] = 1.0 / sqrt(lo);
    out[8] = 1.0 / sqrt(hi);
    return zc < 0.0 ? 1 : 0;
}

static double flux_instant_ell(const double p[GLO_E_NPARAM], double u1, double u2, double t, double tol)
{
    double g[9];
    if (!glo_geometry_ell(p, t, g)) return 1.0;
    return 1.0 - glo_occulted(g[0], g[1], g[3], g[4], g[7], g[8] / g[7], u1, u2, tol, GLO_INNER_CLOSED);
}

int glo_flux_ell(const double p[GLO_E_NPARAM], double t, double t_exp, int n_ss, double tol, double *out)
{
    double u1, u2;
    if (!ell_params_ok(p) || !isfinite(t) || !isfinite(t_exp) || t_exp < 0.0 || n_ss < 1 || n_ss > 64 ||
        glo_kipping(p[GLO_E_Q1], p[GLO_E_Q2], &u1, &u2)) {
        *out = NAN;
        return -1;
    }
    double sum = 0.0;
    for (int j = 0; j < n_ss; j++) {
        double tj = t + (((double)j + 0.5) / (double)n_ss - 0.5) * t_exp;
        sum += flux_instant_ell(p, u1, u2, tj, tol);
    }
    *out = sum / (double)n_ss;
    return 0;
}

int64_t glo_flux_batch_ell(const double *params, int64_t n_sets, const double *times, const int64_t *offsets,
                           int64_t n_times, const int32_t *n_ss, const double *t_exp, double tol, double *out,
                           int nthreads)
{
    int64_t nerr = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : nerr)
#endif
    for (int64_t s = 0; s < n_sets; s++) {
        double p[GLO_E_NPARAM];
        for (int i = 0; i < GLO_E_NPARAM; i++) p[i] = params[(int64_t)i * n_sets + s];
        int64_t a = offsets ? offsets[s] : s * n_times;
        int64_t b = offsets ? offsets[s + 1] : (s + 1) * n_times;
        int nss = n_ss ? n_ss[s] : 1;
        double te = t_exp ? t_exp[s] : 0.0;
        for (int64_t i = a; i < b; i++) {
            double t = offsets ? times[i] : times[i - a];
            if (glo_flux_ell(p, t, te, nss, tol, &out[i])) nerr++;
        }
    }
    return nerr;
}

long glo_unconverged(void)
{
    long n;
#ifdef _OPENMP
#pragma omp atomic read
#endif
    n = glo_n_unconverged;
    return n;
}

int glo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
