// gl_device.h -- per-sample FP64 flux of an oblate planet (device and host).
//
// Computes, for one parameter set and one time, the fraction of quadratically
// limb-darkened stellar flux blocked by the sky-projected ellipse of an oblate
// spheroid on a circular orbit (Price et al. 2024, Section 2).
//
// Method (the paper's Green's-theorem boundary form, Section 2, with exact
// intersections instead of limb snapping):
//  * The projected ellipse is the paper's parametric curve
//      x = x0 + dx cos(th),  y = y0 + dy1 cos(th) + dy2 sin(th)      (eqs. dx, dy1, dy2)
//    with x0 = d cos(alpha) sin(beta), y0 = d sin(alpha).
//  * The occulted region E cap D is bounded by ellipse arcs inside the stellar
//    disk and limb arcs inside the ellipse.  Ellipse/limb intersections are the
//    real roots of |p(th)|^2 - 1, a quartic in t = tan((th - th0)/2); they are
//    isolated between the critical points of the quartic (roots of its cubic
//    derivative, themselves isolated by the roots of the quadratic second
//    derivative) and polished by safeguarded Newton, so no root is missed.
//  * The three Green's integrands of the paper (f_flat, f_lin, f_quad) give the
//    integrals of 1, mu and r^2 over the region.  On ellipse arcs they are
//    integrated by Gauss-Legendre in a tangent half-angle variable with nodes
//    clustered at both arc ends (the f_lin integrand behaves like
//    (th - th_root)^(3/2) there); on limb arcs they have closed forms.  When
//    the whole ellipse is on the star the flat and r^2 integrals are closed
//    forms (ellipse area and second moment) and f_lin uses a full-turn rule
//    clustered at the point nearest the limb.
//  * The quadratic law I = 1 - u1(1-mu) - u2(1-mu)^2 = c0 + c1 mu + c2 r^2,
//    normalised by Phi = pi (1 - u1/3 - u2/6), gives the occulted fraction.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "gl_tables.h"

#define GL_HD __host__ __device__ __forceinline__
// heavy stages keep their own register allocation on the GPU
#define GL_HD_CALL static __host__ __device__ __attribute__((noinline))

namespace gl {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;

// Derived per-parameter-set constants (built once per set, kept in LDS/SGPRs).
struct SetConst {
    double A, B, C;        // dx, dy1, dy2 of the projected ellipse
    double AC;             // dx * dy2 = k^2 q (area / pi)
    double M2;             // dx^2 + dy1^2 + dy2^2 = k^2 (1 + q^2)
    double K3, K4;         // (dx^2 + dy1^2 - dy2^2)/2 and dy1 * dy2
    double k;              // largest semi-axis
    double xb;             // d sin(beta) = b: x0 = xb cos(alpha)
    double d;              // orbital distance: y0 = d sin(alpha)
    double w_orb;          // 2 pi / P
    double P, t0;
    double inv_P;          // 1 / P
    double zA, z2A_inv, zC0;  // k^2 - kq^2, 1 / (2 (k^2 - kq^2)) (0 when tiny), kq^2 - 1 (kq: minor semi-axis)
    double half_win;       // instantaneous overlap needs |t - t0 - nP| < half_win
    double c0, c1, c2;     // I = c0 + c1 mu + c2 r^2
    double inv_phi;        // 1 / Phi
    double t_exp;          // exposure (days)
    double sx, sy;         // unit vector of the projected spin axis (minor axis direction)
    // general ellipsoids (zero for the oblate parameter block)
    double rot[9];         // R(zeta, eta, xi) = Rx Ry Rz, row major (r1..r9)
    double ax2[3];         // a^2, b^2, c^2
    double sb, cb;         // sin(beta), cos(beta)
    int n_ss;              // midpoint sub-samples per output
    int valid;             // 0: domain error, outputs are NaN
    int locked;            // 1: tidally locked, the shadow turns with the orbit
};

// ---------------------------------------------------------------- helpers
GL_HD double sqr(double x) { return x * x; }

// finite (not NaN, not +-inf); NaN fails every comparison
GL_HD bool finite_d(double x) { return fabs(x) <= 1.7976931348623157e308; }

// 1/x for the quadrature nodes: the hardware FP64 reciprocal estimate refined
// by two Newton steps (relative error near one ulp; x is never 0, inf or
// denormal here).  The host build uses the IEEE division.
GL_HD double rcp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
#else
    return 1.0 / x;
#endif
}

// sqrt(x) for x >= 0 from the hardware reciprocal-square-root estimate and
// two Goldschmidt/Newton refinements; arguments below 1e-300 return 0.
GL_HD double sqrt_nn(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    // branch-free: the refinement runs on a clamped argument and the result
    // is selected afterwards (zero for x <= 1e-300 and for NaN)
    const bool pos = x > 1e-300;
    const double xc = pos ? x : 1.0;
    const double y = __builtin_amdgcn_rsq(xc);
    double g = xc * y, h = 0.5 * y;
    const double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    const double d = fma(-g, g, xc);
    g = fma(d, h, g);
    const double d2 = fma(-g, g, xc);
    const double r = fma(d2, h, g);
    return pos ? r : 0.0;
#else
    return x > 0.0 ? sqrt(x) : 0.0;
#endif
}

// Integrand-grade forms for quadrature nodes, where a relative error of a few
// 1e-15 per node is far below the rules' own error: the hardware estimates
// (relative error below 2^-24, measured) after one Newton step each, which
// squares that error: about 2e-15 for the reciprocal and 1.5 x 2^-48 = 4e-15
// for the square root.  Host builds use the IEEE forms.
GL_HD double rcp_q(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
#else
    return 1.0 / x;
#endif
}

// (x >= 0: the estimate is taken at max(x, 1e-300), so that x = 0 gives
// g = 0 and a result of exactly 0 with no select; below 1e-300 the result is
// merely tiny.)  With y = (1 + eps)/sqrt(x): g = x y, e = 1/2 - g y/2 =
// -eps - eps^2/2, and g (1 + e) = sqrt(x) (1 - 3 eps^2/2 - eps^3/2).
GL_HD double sqrt_q(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(fmax(x, 1e-300));
    const double g = x * y;
    return fma(g, fma(-g, 0.5 * y, 0.5), g);
#else
    return x > 0.0 ? sqrt(x) : 0.0;
#endif
}

// As sqrt_q for an argument known to be positive and normal: nodes of the
// whole-ellipse trapezoid rule, which stay a bounded distance inside the disk.
GL_HD double sqrt_qp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
    const double g = x * y;
    return fma(g, fma(-g, 0.5 * y, 0.5), g);
#else
    return sqrt(x);
#endif
}

// Single-precision estimates (the hardware instructions on the device, the
// IEEE functions on the host): the FP32 integrator of Section 2 and the
// first iterates of the quartic solver.
GL_HD float rsqrt_f(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}

GL_HD float sqrt_f(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}

GL_HD float rcp_f(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// Cube root with the sign of x, as 2^(log2|x| / 3) from the hardware base-2
// logarithm and exponential (x = 0 gives 0).
GL_HD float cbrt_f(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return copysignf(__builtin_amdgcn_exp2f(__builtin_amdgcn_logf(fabsf(x)) * (1.0f / 3.0f)), x);
#else
    return cbrtf(x);
#endif
}

// sin and cos of a in [-pi, pi] (orbital phase): a = k pi/2 + r with
// |r| <= pi/4 (pi/2 split in two parts, Cody-Waite style), Taylor series of
// sin r and cos r to r^17 and r^16 (the next terms are below 1e-17), then the
// quadrant turn.
GL_HD void sincos_pi(double a, double& sn, double& cs)
{
    const double k = rint(a * 0.63661977236758134308);  // 2/pi
    const double r = fma(-k, 1.5707963267948966e+00, fma(-k, 6.123233995736766e-17, a));
    const double r2 = r * r;
    double ps = 1.0 / 355687428096000.0;                       // 1/17!
    ps = fma(ps, -r2, 1.0 / 1307674368000.0);                  // 1/15!
    ps = fma(ps, r2, -1.0 / 6227020800.0);                     // 1/13!
    ps = fma(ps, r2, 1.0 / 39916800.0);                        // 1/11!
    ps = fma(ps, r2, -1.0 / 362880.0);                         // 1/9!
    ps = fma(ps, r2, 1.0 / 5040.0);                            // 1/7!
    ps = fma(ps, r2, -1.0 / 120.0);                            // 1/5!
    ps = fma(ps, r2, 1.0 / 6.0);                               // 1/3!
    const double s0 = fma(-r * r2, ps, r);
    double pc = 1.0 / 20922789888000.0;                        // 1/16!
    pc = fma(pc, -r2, 1.0 / 87178291200.0);                    // 1/14!
    pc = fma(pc, r2, -1.0 / 479001600.0);                      // 1/12!
    pc = fma(pc, r2, 1.0 / 3628800.0);                         // 1/10!
    pc = fma(pc, r2, -1.0 / 40320.0);                          // 1/8!
    pc = fma(pc, r2, 1.0 / 720.0);                             // 1/6!
    pc = fma(pc, r2, -1.0 / 24.0);                             // 1/4!
    pc = fma(pc, r2, 0.5);                                     // 1/2!
    const double c0 = fma(-r2, pc, 1.0);
    const int q = ((int)k) & 3;
    sn = (q == 0) ? s0 : (q == 1) ? c0 : (q == 2) ? -s0 : -c0;
    cs = (q == 0) ? c0 : (q == 1) ? -s0 : (q == 2) ? -c0 : s0;
}

// 1/31, 1/29, ..., 1/3, 1: the Taylor series of atan(u) / u in powers of -u^2.
static constexpr double kAtanInvOdd[16] = {1.0 / 31, 1.0 / 29, 1.0 / 27, 1.0 / 25, 1.0 / 23, 1.0 / 21,
                                           1.0 / 19, 1.0 / 17, 1.0 / 15, 1.0 / 13, 1.0 / 11, 1.0 / 9,
                                           1.0 / 7,  1.0 / 5,  1.0 / 3,  1.0};

// atan(z) for |z| <= 1: atan z = pi/6 + atan((z - 1/sqrt 3)/(1 + z/sqrt 3))
// brings |z| below tan(pi/12); then the Taylor series to z^31.  No branches:
// the reduced argument is always computed and selected, so that the lanes of
// a wavefront never run the series twice.
GL_HD double atan_unit(double z)
{
    const double az = fabs(z);
    const bool red = az > 0.26794919243112270;      // tan(pi/12)
    const double is3 = 0.57735026918962576451;       // 1/sqrt(3)
    const double q = (az - is3) / fma(az, is3, 1.0);
    const double u = red ? q : az;
    const double base = red ? 0.52359877559829887308 : 0.0;  // pi/6
    const double u2 = u * u;
    // coefficients read from a table, five per pass of a loop that is not
    // unrolled: unrolled, the compiler keeps the 15 doubles in registers
    // across a caller's whole sample loop (and spills them)
    double p = kAtanInvOdd[0];
#pragma unroll 1
    for (int i = 1; i < 16; i += 5) {
#pragma unroll
        for (int j = 0; j < 5; ++j) p = fma(p, -u2, kAtanInvOdd[i + j]);
    }
    const double r = base + u * p;
    return z < 0.0 ? -r : r;
}

// atan2(y, x) in (-pi, pi] from atan_unit, one call per argument pair.
GL_HD double atan2_d(double y, double x)
{
    const double ay = fabs(y), ax = fabs(x);
    const bool steep = ay > ax;
    const double num = steep ? ax : ay, den = steep ? ay : ax;  // num <= den
    const double t = atan_unit(num / (den > 0.0 ? den : 1.0));  // 0 when x = y = 0
    double a = steep ? 1.57079632679489661923 - t : t;
    if (x < 0.0) a = 3.14159265358979323846 - a;
    return (y < 0.0) ? -a : a;
}

// a reduced to [-pi, pi] for sincos_pi (the angles of a parameter block may lie
// outside it): a - 2 pi rint(a / 2 pi).
GL_HD double wrap_pi(double a) { return fma(-kTwoPi, rint(a * (1.0 / kTwoPi)), a); }

// The paper's rotation R(zeta=0, eta, xi) = Ry(eta) Rz(xi) entries r1..r9 and
// eqs. dx, dy1, dy2 with polar semi-axis a = k(1-f) (body x') and b = c = k.
GL_HD void projected_ellipse(double k, double f, double theta, double phi,
                             double& A, double& B, double& C)
{
    double se, ce, sx, cx;
    sincos_pi(wrap_pi(0.5 * kPi - theta), se, ce);  // eta = pi/2 - theta
    sincos_pi(wrap_pi(phi), sx, cx);
    // R = Ry(eta) Rz(xi)
    const double r1 = ce * cx, r2 = -ce * sx, r3 = se;
    const double r4 = sx, r5 = cx, r6 = 0.0;
    const double r7 = -se * cx, r8 = se * sx, r9 = ce;
    const double a = k * (1.0 - f), b = k, c = k;
    const double a2 = a * a, b2 = b * b, c2 = c * c;
    A = sqrt(a2 * r1 * r1 + b2 * r4 * r4 + c2 * r7 * r7);
    B = (a2 * r1 * r2 + b2 * r4 * r5 + c2 * r7 * r8) / A;
    C = sqrt(a2 * b2 * r9 * r9 + a2 * c2 * r6 * r6 + b2 * c2 * r3 * r3) / A;
}

// The shape terms derived from (dx, dy1, dy2) and the major semi-axis kmaj of
// the shadow: area, second moments and the coefficients of the singularity
// bound (zero_cosh_bound).
GL_HD void shape_terms(SetConst& s, double kmaj)
{
    s.AC = s.A * s.C;
    s.M2 = s.A * s.A + s.B * s.B + s.C * s.C;
    s.K3 = 0.5 * (s.A * s.A + s.B * s.B - s.C * s.C);
    s.K4 = s.B * s.C;
    s.k = kmaj;
    const double kq = s.AC / kmaj;  // minor semi-axis of the projected ellipse
    s.zA = (kmaj - kq) * (kmaj + kq);
    s.z2A_inv = s.zA > 1e-14 * kmaj * kmaj ? 1.0 / (2.0 * s.zA) : 0.0;
    s.zC0 = kq * kq - 1.0;
}

// Semi-axes of the curve (A cos th, B cos th + C sin th): the square roots of
// the eigenvalues of [[A^2, AB], [AB, B^2 + C^2]] (trace M2, determinant
// (AC)^2).  Returns the major one; (ux, uy) is the unit minor-axis direction.
GL_HD double shadow_axes(double A, double B, double C, double& ux, double& uy)
{
    const double s11 = A * A, s12 = A * B, s22 = B * B + C * C;
    const double rad = sqrt(sqr(0.5 * (s11 - s22)) + s12 * s12);
    const double hi = 0.5 * (s11 + s22) + rad;
    const double lo = (A * C) * (A * C) / hi;
    double vx, vy;  // eigenvector of lo from the better conditioned row
    if (fabs(s11 - lo) >= fabs(s22 - lo)) {
        vx = -s12;
        vy = s11 - lo;
    } else {
        vx = s22 - lo;
        vy = -s12;
    }
    const double n = sqrt(vx * vx + vy * vy);
    ux = n > 0.0 ? vx / n : 1.0;
    uy = n > 0.0 ? vy / n : 0.0;
    return sqrt(hi);
}

// Orbit, transit window and limb darkening of a set: b, d = a/R*, P, t0,
// Kipping q1, q2; kreach bounds the shadow's semi-axes over the orbit.
GL_HD void orbit_and_limb(SetConst& s, double kreach, double b, double d, double P, double t0, double q1,
                          double q2)
{
    // orbit (eq. coord-map): sin(beta) = b/d, x0 = d cos(alpha) sin(beta)
    s.xb = d * (b / d);
    s.d = d;
    s.P = P;
    s.inv_P = 1.0 / P;
    s.t0 = t0;
    s.w_orb = kTwoPi / P;
    // overlap needs rho^2 = b^2 cos^2(alpha) + d^2 sin^2(alpha) < (1 + k)^2 with
    // cos(alpha) > 0, i.e. sin^2(alpha) < ((1+k)^2 - b^2) / (d^2 - b^2)
    const double num = (1.0 + kreach) * (1.0 + kreach) - b * b;
    if (num > 0.0) {
        const double sa = fmin(1.0, sqrt(num / ((d - b) * (d + b))));
        s.half_win = (asin(sa) / s.w_orb) * (1.0 + 1e-9) + 1e-12 * P;
    } else {
        s.half_win = -1e300;  // never overlaps the disk
    }
    // Kipping (2013) q -> u, then I = c0 + c1 mu + c2 r^2
    const double sq = sqrt(q1);
    const double u1 = 2.0 * sq * q2, u2 = sq * (1.0 - 2.0 * q2);
    s.c0 = 1.0 - u1 - 2.0 * u2;
    s.c1 = u1 + 2.0 * u2;
    s.c2 = u2;
    s.inv_phi = 1.0 / (kPi * (1.0 - u1 / 3.0 - u2 / 6.0));
}

// Builds SetConst from the parameter block values (k, f, theta, phi, b, a/R*,
// P, t0, q1, q2).  Returns false on a domain error.
GL_HD bool make_set_const(const double* p, double t_exp, int n_ss, SetConst& s)
{
    const double k = p[0], f = p[1], theta = p[2], phi = p[3], b = p[4];
    const double d = p[5], P = p[6], t0 = p[7], q1 = p[8], q2 = p[9];
    bool ok = true;
    for (int i = 0; i < 10; ++i) ok = ok && finite_d(p[i]);
    ok = ok && (k > 0.0) && (k < 1.0) && (f >= 0.0) && (f < 1.0) && (d > 1.0 + k) &&
         (fabs(b) < d) && (P > 0.0) && (q1 >= 0.0) && (q1 <= 1.0) && (q2 >= 0.0) &&
         (q2 <= 1.0) && finite_d(t_exp) && (t_exp >= 0.0) && (n_ss >= 1) && (n_ss <= 64);
    s.valid = ok ? 1 : 0;
    s.n_ss = n_ss;
    s.t_exp = t_exp;
    s.locked = 0;
    for (int i = 0; i < 9; ++i) s.rot[i] = 0.0;
    s.ax2[0] = s.ax2[1] = s.ax2[2] = 0.0;
    s.sb = s.cb = 0.0;
    if (!ok) return false;
    projected_ellipse(k, f, theta, phi, s.A, s.B, s.C);
    {
        double sp, cp;
        sincos_pi(wrap_pi(phi), sp, cp);
        s.sx = cp;
        s.sy = -sp;
    }
    // the equatorial radius k is the shadow's major semi-axis (f >= 0)
    shape_terms(s, k);
    orbit_and_limb(s, k, b, d, P, t0, q1, q2);
    return true;
}

// ---------------------------------------------------------------- MCMC walkers
// The fitting parameters of Section 3 (r, mu, nu, xi, b, d/R*, P, t0, q1, q2)
// to the oblate parameter block (Appendix A): f = f_min + (1 - f_min) nu with
// f_min = 1 - sqrt((mu + 1) / 2); cos(2 eta) = (mu - (f - 1)^2) / (f (f - 2))
// from eq. mu, eta in [0, pi/2] (0 for a sphere); theta = pi/2 - eta; the
// equatorial radius k = r / cbrt(1 - f) (r^3 = k^3 (1 - f)); the other rows
// carry over.
constexpr int kWalkParams = 10;

GL_HD void walker_to_params(const double* w, double* p)
{
    const double r = w[0], mu = w[1], nu = w[2];
    const double f_min = 1.0 - sqrt(0.5 * (mu + 1.0));
    const double f = f_min + (1.0 - f_min) * nu;
    const double den = f * (f - 2.0);
    double c2 = den != 0.0 ? (mu - (f - 1.0) * (f - 1.0)) / den : 1.0;
    c2 = fmin(1.0, fmax(-1.0, c2));
    p[0] = r / cbrt(1.0 - f);
    p[1] = f;
    p[2] = 0.5 * kPi - 0.5 * acos(c2);
    for (int i = 3; i < kWalkParams; ++i) p[i] = w[i];
}

// ---------------------------------------------------------------- general ellipsoids
// Rows of the general parameter block: semi-axes a, b, c (stellar radii)
// along x', y', z'; orientation zeta, eta, xi (R = Rx(zeta) Ry(eta) Rz(xi),
// Section 2 eq. coord-map); impact parameter, a/R*, P, t0, Kipping q1, q2;
// `locked` = 1 for the tidally-locked coordinate map of Appendix B.
constexpr int kEllParams = 13;

// (dx, dy1, dy2) of the shadow of the body whose body coordinates are
// M (x - x_c), from the first two columns u, v and the third w of M:
// dx = |D u|, dy1 = (D u . D v) / dx, dy2 = |D u x D v| / dx with
// D = diag(a, b, c), and D u x D v = abc (w_x / a, w_y / b, w_z / c).  With
// M = R these are eqs. dx, dy1, dy2; with M = R Rx(-alpha) Ry(beta) they are
// eqs. dx-locked, dy1-locked, dy2-locked.
GL_HD void deltas_of_map(const double* ax2, const double* u, const double* v, const double* w,
                         double& A, double& B, double& C)
{
    const double a2 = ax2[0], b2 = ax2[1], c2 = ax2[2];
    A = sqrt(a2 * u[0] * u[0] + b2 * u[1] * u[1] + c2 * u[2] * u[2]);
    B = (a2 * u[0] * v[0] + b2 * u[1] * v[1] + c2 * u[2] * v[2]) / A;
    C = sqrt(a2 * b2 * w[2] * w[2] + a2 * c2 * w[1] * w[1] + b2 * c2 * w[0] * w[0]) / A;
}

GL_HD bool make_set_const_ell(const double* p, double t_exp, int n_ss, SetConst& s)
{
    const double ra = p[0], rb = p[1], rc = p[2], zeta = p[3], eta = p[4], xi = p[5];
    const double b = p[6], d = p[7], P = p[8], t0 = p[9], q1 = p[10], q2 = p[11], lk = p[12];
    bool ok = true;
    for (int i = 0; i < kEllParams; ++i) ok = ok && finite_d(p[i]);
    const double amax = fmax(ra, fmax(rb, rc));
    ok = ok && (ra > 0.0) && (ra < 1.0) && (rb > 0.0) && (rb < 1.0) && (rc > 0.0) && (rc < 1.0) &&
         (d > 1.0 + amax) && (fabs(b) < d) && (P > 0.0) && (q1 >= 0.0) && (q1 <= 1.0) && (q2 >= 0.0) &&
         (q2 <= 1.0) && (lk == 0.0 || lk == 1.0) && finite_d(t_exp) && (t_exp >= 0.0) && (n_ss >= 1) &&
         (n_ss <= 64);
    s.valid = ok ? 1 : 0;
    s.n_ss = n_ss;
    s.t_exp = t_exp;
    s.locked = lk == 1.0 ? 1 : 0;
    if (!ok) return false;
    double sz, cz, se, ce, sx, cx;
    sincos_pi(wrap_pi(zeta), sz, cz);
    sincos_pi(wrap_pi(eta), se, ce);
    sincos_pi(wrap_pi(xi), sx, cx);
    // Ry(eta) Rz(xi), then Rx(zeta) mixes its second and third rows
    const double m1[3] = {ce * cx, -ce * sx, se};
    const double m2[3] = {sx, cx, 0.0};
    const double m3[3] = {-se * cx, se * sx, ce};
    for (int j = 0; j < 3; ++j) {
        s.rot[j] = m1[j];
        s.rot[3 + j] = cz * m2[j] - sz * m3[j];
        s.rot[6 + j] = sz * m2[j] + cz * m3[j];
    }
    s.ax2[0] = ra * ra;
    s.ax2[1] = rb * rb;
    s.ax2[2] = rc * rc;
    s.sb = b / d;
    s.cb = sqrt((1.0 - s.sb) * (1.0 + s.sb));
    // the set-level shadow: exact when not locked; when locked, the shadow at
    // mid-transit (the per-sample one comes from lock_at)
    const double* R = s.rot;
    double u[3], v[3], w[3];
    for (int i = 0; i < 3; ++i) {
        const double r1 = R[3 * i], r2 = R[3 * i + 1], r3 = R[3 * i + 2];
        if (s.locked) {  // M = R Rx(0) Ry(beta)
            u[i] = r1 * s.cb - r3 * s.sb;
            v[i] = r2;
            w[i] = r1 * s.sb + r3 * s.cb;
        } else {
            u[i] = r1;
            v[i] = r2;
            w[i] = r3;
        }
    }
    deltas_of_map(s.ax2, u, v, w, s.A, s.B, s.C);
    const double kmaj = shadow_axes(s.A, s.B, s.C, s.sx, s.sy);
    shape_terms(s, kmaj);
    // a locked shadow changes over the orbit: its window uses the largest semi-axis
    orbit_and_limb(s, s.locked ? amax : kmaj, b, d, P, t0, q1, q2);
    return true;
}


// Time offset from the nearest mid-transit, in (-P/2, P/2].
GL_HD double phase_time(const SetConst& s, double t)
{
    // (the transit index from dt / P or dt * (1/P) can differ only where dt
    // is half a period from a transit, with the planet behind the star)
    const double dt = t - s.t0;
    return dt - s.P * rint(dt * s.inv_P);
}

// Per-sample shadow of a locked set at time t (Appendix B): body coordinates
// R Rx(-alpha) Ry(beta) (x - x_c) at the sample's orbital phase alpha; the
// centre follows from centre_at with the same alpha.
GL_HD void lock_at(const SetConst& s, double t, SetConst& o)
{
    o = s;
    const double alpha = s.w_orb * phase_time(s, t);
    double sa, ca;
    sincos_pi(alpha, sa, ca);
    const double sb = s.sb, cb = s.cb;
    double u[3], v[3], w[3];
    for (int i = 0; i < 3; ++i) {
        const double r1 = s.rot[3 * i], r2 = s.rot[3 * i + 1], r3 = s.rot[3 * i + 2];
        const double g = r2 * sa + r3 * ca;
        u[i] = r1 * cb - sb * g;
        v[i] = r2 * ca - r3 * sa;
        w[i] = r1 * sb + cb * g;
    }
    deltas_of_map(s.ax2, u, v, w, o.A, o.B, o.C);
    const double kmaj = shadow_axes(o.A, o.B, o.C, o.sx, o.sy);
    shape_terms(o, kmaj);
}

// ---------------------------------------------------------------- work census
// The census variant counts the work a sample really does (used to turn the
// kernel time into an algorithmic FLOP rate); the default does nothing.
// Both count the arcs that the arc rule accepted at its last level with the
// Gauss-Kronrod difference still above its tolerance (rare; reported, never
// silent).
struct NoCensus {
    int unconv = 0;
    GL_HD void iter() {}
    GL_HD void arc() {}
    GL_HD void trap(int) {}
    GL_HD void limb() {}
    GL_HD void unconverged() { ++unconv; }
};
struct Census {
    int iters = 0, arcs = 0, trap_nodes = 0, limbs = 0, unconv = 0;
    GL_HD void iter() { ++iters; }
    GL_HD void arc() { ++arcs; }           // one 21-node Gauss-Kronrod piece
    GL_HD void trap(int n) { trap_nodes += n; }
    GL_HD void limb() { ++limbs; }
    GL_HD void unconverged() { ++unconv; }
};

// ---------------------------------------------------------------- quartic
struct Poly4 {
    double a0, a1, a2, a3, a4;
};

GL_HD double p4(const Poly4& q, double t)
{
    return fma(fma(fma(fma(q.a4, t, q.a3), t, q.a2), t, q.a1), t, q.a0);
}
GL_HD double dp4(const Poly4& q, double t)
{
    return fma(fma(fma(4.0 * q.a4, t, 3.0 * q.a3), t, 2.0 * q.a2), t, q.a1);
}
GL_HD double ddp4(const Poly4& q, double t)
{
    return fma(fma(12.0 * q.a4, t, 6.0 * q.a3), t, 2.0 * q.a2);
}

// Root of a function that is monotone on [lo, hi] with values flo, fhi of
// opposite sign at the ends: Newton from the given first iterate (from the
// regula-falsi point when that is missing or outside the bracket), with
// bisection whenever a step leaves the bracket; stops when the step is below
// its tolerance or the bracket at rounding level, or (a root of q) when |f| is
// below the rounding noise of its own evaluation.
template <int Deriv, class CT>
GL_HD double bracket_root(const Poly4& q, double lo, double hi, double flo, double fhi, CT& ct,
                          double start = __builtin_nan(""))
{
    const double a0 = fabs(q.a0), a1 = fabs(q.a1), a2 = fabs(q.a2), a3 = fabs(q.a3),
                 a4 = fabs(q.a4);
    // first iterate: the given start when it lies inside the bracket, else the
    // secant through the ends, else the midpoint
    double x = (start > lo && start < hi) ? start : lo - flo * (hi - lo) / (fhi - flo);
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        ct.iter();
        double f, df;
        const double ax = fabs(x);
        if (Deriv == 0) {
            f = p4(q, x);
            df = dp4(q, x);
            // a root of q may stop at the rounding noise of its evaluation; a
            // critical point stops on its step alone (the 1e-4 tolerance below)
            const double noise = fma(fma(fma(fma(a4, ax, a3), ax, a2), ax, a1), ax, a0);
            if (fabs(f) <= 8e-16 * noise) return x;
        } else {
            f = dp4(q, x);
            df = ddp4(q, x);
        }
        if ((f < 0.0) == (flo < 0.0)) lo = x;
        else hi = x;
        double xn = x - f * rcp(df);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        // a Newton step below 1e-4 leaves an error near its square, 1e-8 in t
        // (quadratic convergence).  That is enough for both kinds: a critical
        // point only brackets roots and places a cluster break point (the
        // integral does not depend on where an arc is split), and a crossing
        // that is off by d only swaps a sliver between ellipse and limb whose
        // area is of order d^2 times the crossing angle: the limb arc starts at
        // the polar angle of the ellipse point at the computed root, so the
        // contour closes along a ray, where the integrands of the polar form
        // vanish.  Started from the closed-form guesses of the solver, the
        // first step is usually below 1e-6 and ends the iteration
        constexpr double step_tol = 1e-4;
        if (fabs(xn - x) <= step_tol * fmax(1.0, ax) || hi - lo <= 2e-16 * fmax(1.0, ax)) return xn;
        x = xn;
    }
    return x;
}

// First iterates from closed forms: coefficients in FP64, cube and square
// roots in FP32.  A guess is used only when it lies inside its bracket, so an
// inaccurate or missing one costs Newton steps, never accuracy; NaN marks a
// missing guess (every comparison with it fails).

// The real root of the cubic q'(t) = 4 a4 t^3 + 3 a3 t^2 + 2 a2 t + a1 when it
// has only one: Cardano's formula for the cubic depressed about its
// inflection point, y^3 + P y + R = 0, y = u + v with u^3 the larger of
// -R/2 +- sqrt(R^2/4 + P^3/27) in magnitude and v = -P / (3u) (no
// cancellation); NaN when the cubic has three real roots.
GL_HD double cubic_one_root(const Poly4& q)
{
    const double ia = rcp(4.0 * q.a4);
    const double b = 3.0 * q.a3 * ia, c = 2.0 * q.a2 * ia, d = q.a1 * ia;
    const double P = fma(b * b, -1.0 / 3.0, c);
    const double R = fma(b * fma(2.0 * b, b, -9.0 * c), 1.0 / 27.0, d);
    const double disc = fma(0.25 * R, R, P * P * P * (1.0 / 27.0));
    const float hr = (float)(-0.5 * R), sd = sqrt_f((float)fmax(disc, 0.0));
    const float u = cbrt_f(hr >= 0.0f ? hr + sd : hr - sd);
    const double v = u != 0.0f ? -P * (double)rcp_f(3.0f * u) : 0.0;
    const double y = (double)u + v - b * (1.0 / 3.0);
    return disc >= 0.0 ? y : __builtin_nan("");
}

// Real roots of the quartic q when it has exactly two (Ferrari's method):
// with t = y - b/4 the monic quartic becomes y^4 + p y^2 + r1 y + r0; a root
// m >= 0 of the resolvent m^3 + p m^2 + (p^2/4 - r0) m - r1^2/8 (Cardano,
// then one FP64 Newton step: a small m loses its relative accuracy to
// cancellation in the formula) splits it into y^2 - s y + (p/2 + m + w) and
// y^2 + s y + (p/2 + m - w), s = sqrt(2m), w = r1 / (2s), taken as
// sign(r1) sqrt(m^2 + p m + p^2/4 - r0), which holds at the resolvent root and
// stays finite as m -> 0 (the biquadratic limit).  Two real roots of the
// quartic go with a resolvent of one real root (equal discriminants, up to a
// positive factor); with three (no real root of the quartic, or four) every
// guess is NaN.  out[0..3] in no particular order, NaN for a quadratic
// without real roots.
GL_HD void quartic_guesses(const Poly4& q, float* out)
{
    const double ia = rcp(q.a4);
    const double b = q.a3 * ia, c = q.a2 * ia, d = q.a1 * ia, e = q.a0 * ia;
    const double b2 = b * b;
    const double p = fma(-0.375, b2, c);
    const double r1 = fma(0.125 * b2, b, fma(-0.5 * b, c, d));
    const double r0 = fma(-3.0 / 256.0 * b2, b2, fma(0.0625 * b2, c, fma(-0.25 * b, d, e)));
    const double C = fma(0.25 * p, p, -r0), D = -0.125 * r1 * r1;
    const double P3 = fma(p * p, -1.0 / 3.0, C);
    const double R3 = fma(p * fma(2.0 * p, p, -9.0 * C), 1.0 / 27.0, D);
    const double disc = fma(0.25 * R3, R3, P3 * P3 * P3 * (1.0 / 27.0));
    const float hr = (float)(-0.5 * R3), sd = sqrt_f((float)fmax(disc, 0.0));
    const float u = cbrt_f(hr >= 0.0f ? hr + sd : hr - sd);
    double m = (double)u + (u != 0.0f ? -P3 * (double)rcp_f(3.0f * u) : 0.0) - p * (1.0 / 3.0);
    const double fm = fma(fma(m + p, m, C), m, D), dfm = fma(fma(3.0, m, 2.0 * p), m, C);
    m = fmax(m - fm * rcp(dfm != 0.0 ? dfm : 1.0), 0.0);
    const float s = sqrt_f((float)(2.0 * m));
    const float w = copysignf(sqrt_f((float)fmax(fma(m + p, m, C), 0.0)), (float)r1);
    const float h = (float)(fma(0.5, p, m)), sh = (float)(-0.25 * b);
    const float d1 = s * s - 4.0f * (h + w), d2 = s * s - 4.0f * (h - w);
    const float w1 = sqrt_f(d1), w2 = sqrt_f(d2);  // NaN for a negative argument
    const bool ok = disc >= 0.0;
    const float nan = __builtin_nanf("");
    out[0] = ok && d1 >= 0.0f ? sh + 0.5f * (s + w1) : nan;
    out[1] = ok && d1 >= 0.0f ? sh + 0.5f * (s - w1) : nan;
    out[2] = ok && d2 >= 0.0f ? sh + 0.5f * (w2 - s) : nan;
    out[3] = ok && d2 >= 0.0f ? sh - 0.5f * (s + w2) : nan;
}

// Real roots and critical points of the quartic in fixed slots, ascending
// among the valid ones.  Every index below is static, so the slots stay in
// registers.
struct QuarticRoots {
    int n_roots;
    double r[4];
    bool rv[4];
    double c[3];
    bool cv[3];
};

template <class CT>
GL_HD void solve_quartic_inl(const Poly4& q, QuarticRoots& out, CT& ct)
{
    // Cauchy bound on all roots of q and of q'
    const double inv = 1.0 / fabs(q.a4);
    const double Bnd = 1.0 + fmax(fmax(fabs(q.a3), fabs(q.a2)), fmax(fabs(q.a1), fabs(q.a0))) * inv;
    // inflection points (roots of q'' = 12 a4 t^2 + 6 a3 t + 2 a2) clamped into
    // [-Bnd, Bnd]; without real ones both sit at -Bnd.  Between consecutive
    // edges q' is monotone (empty intervals never show a sign change).
    double i0 = -Bnd, i1 = -Bnd;
    {
        const double qa = 12.0 * q.a4, qb = 6.0 * q.a3, qc = 2.0 * q.a2;
        const double disc = qb * qb - 4.0 * qa * qc;
        if (disc > 0.0) {
            const double sd = sqrt(disc);
            const double qq = -0.5 * (qb + copysign(sd, qb));
            const double x1 = qq / qa, x2 = (qq != 0.0) ? qc / qq : -x1;
            i0 = fmin(fmax(fmin(x1, x2), -Bnd), Bnd);
            i1 = fmin(fmax(fmax(x1, x2), -Bnd), Bnd);
        }
    }
    const double e[4] = {-Bnd, i0, i1, Bnd};
    // critical points: a root of q' in each interval where it changes sign,
    // solved in a loop over the lane's own sign changes (nearly every sample
    // has exactly one, in a slot that differs from lane to lane: one Newton
    // loop per lane instead of one per slot)
    double fe[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) fe[i] = dp4(q, e[i]);
    unsigned ctodo = 0u;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        out.cv[i] = (fe[i] < 0.0) != (fe[i + 1] < 0.0) && fe[i] != 0.0 && fe[i + 1] != 0.0;
        out.c[i] = e[i];
        ctodo |= (out.cv[i] ? 1u : 0u) << i;
    }
    // first iterate: the cubic's one real root (NaN when it has three)
    const double cstart = cubic_one_root(q);
    while (ctodo) {
        const int i = __builtin_ctz(ctodo);
        ctodo &= ctodo - 1u;
        const double lo = i == 0 ? e[0] : i == 1 ? e[1] : e[2];
        const double hi = i == 0 ? e[1] : i == 1 ? e[2] : e[3];
        const double flo = i == 0 ? fe[0] : i == 1 ? fe[1] : fe[2];
        const double fhi = i == 0 ? fe[1] : i == 1 ? fe[2] : fe[3];
        const double x = bracket_root<1>(q, lo, hi, flo, fhi, ct, cstart);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k == i) out.c[k] = x;
    }
    // roots of q between consecutive critical points; an empty critical slot
    // keeps the left end of its interval, which only splits a stretch where
    // q is monotone
    const double pt[5] = {-Bnd, out.c[0], out.c[1], out.c[2], Bnd};
    double fq[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) fq[i] = p4(q, pt[i]);
    // first iterates: Ferrari's roots, each taken by the bracket it falls in
    // (the secant across the bracket where none does)
    float guess[4];
    quartic_guesses(q, guess);
    // the brackets with a sign change are solved in a loop over the lane's own
    // brackets (one Newton loop per root of the lane, not per bracket slot:
    // the lanes of a wavefront mostly have their two roots in different slots)
    out.n_roots = 0;
    unsigned todo = 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        out.rv[i] = (fq[i] < 0.0) != (fq[i + 1] < 0.0) && fq[i] != 0.0 && fq[i + 1] != 0.0;
        out.r[i] = 0.0;
        out.n_roots += out.rv[i] ? 1 : 0;
        todo |= (out.rv[i] ? 1u : 0u) << i;
    }
    while (todo) {
        const int i = __builtin_ctz(todo);
        todo &= todo - 1u;
        // bracket i by selects (the slots stay in registers)
        const double lo = i == 0 ? pt[0] : i == 1 ? pt[1] : i == 2 ? pt[2] : pt[3];
        const double hi = i == 0 ? pt[1] : i == 1 ? pt[2] : i == 2 ? pt[3] : pt[4];
        const double flo = i == 0 ? fq[0] : i == 1 ? fq[1] : i == 2 ? fq[2] : fq[3];
        const double fhi = i == 0 ? fq[1] : i == 1 ? fq[2] : i == 2 ? fq[3] : fq[4];
        double start = __builtin_nan("");
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double g = (double)guess[k];
            start = (g > lo && g < hi) ? g : start;
        }
        const double x = bracket_root<0>(q, lo, hi, flo, fhi, ct, start);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k == i) out.r[k] = x;
    }
}

// Out-of-line form (keeps the register budget of callers that rarely need it).
template <class CT>
GL_HD_CALL void solve_quartic(const Poly4& q, QuarticRoots& out, CT& ct)
{
    solve_quartic_inl(q, out, ct);
}

// ---------------------------------------------------------------- geometry of one sample
// Ellipse in the rotated angle psi = th - th0:
//   x = x0 + Xc cos(psi) + Xs sin(psi),  y = y0 + Yc cos(psi) + Ys sin(psi)
struct Frame {
    double x0, y0;
    double Xc, Xs, Yc, Ys;
    double P0, P1, P2;     // x y' - y x' = P0 + P1 cos(psi) + P2 sin(psi)
};

GL_HD void make_frame(const SetConst& s, double x0, double y0, double c0a, double s0a, Frame& F)
{
    F.x0 = x0;
    F.y0 = y0;
    F.Xc = s.A * c0a;
    F.Xs = -s.A * s0a;
    F.Yc = s.B * c0a + s.C * s0a;
    F.Ys = s.C * c0a - s.B * s0a;
    F.P0 = s.AC;
    F.P1 = x0 * F.Ys - y0 * F.Xs;
    F.P2 = y0 * F.Xc - x0 * F.Yc;
}

// Sums of the three Green's integrands over E cap D: 1, mu and r^2.
struct Sums {
    double flat, lin, quad;
};

// Tolerances of the self-checking rules (absolute, on the integrals of 1 and
// mu over the region; the flux error is at most about the same size).
#ifndef GL_ARC_TOL
#define GL_ARC_TOL 1e-6
#endif
#ifndef GL_TRAP_TOL
#define GL_TRAP_TOL 1e-8
#endif
constexpr double kArcTol = GL_ARC_TOL;    // |K21 - G10| accepted on an arc
constexpr double kTrapTol = GL_TRAP_TOL;  // |T_2n - T_n| accepted on a whole turn
constexpr int kArcMaxLevel = 4;           // an arc is re-split at most into 16 pieces
// Arcs with h = tan(span/4) above this start at two pieces: on the MCMC-walker
// workload nearly all of them fail the one-piece check (which is then wasted
// work), nearly all shorter ones pass it.
constexpr double kArcStartSplit = 0.7;

GL_HD int arc_start_level(double h) { return h > kArcStartSplit ? 1 : 0; }

// One piece tau in [mid - half, mid + half] of the arc psi = psi_c + 2 atan(tau):
// clustered Gauss-Kronrod 10/21 rule.  Adds the Kronrod sums to K and returns
// the Gauss-Kronrod difference of the integrals of 1 and mu.
// The Gauss-10 nodes of the 21-point rule are the odd ones.
constexpr bool gk21_gauss_odd()
{
    for (int j = 0; j < 21; ++j)
        if ((GK21_WG[j] != 0.0) != (j % 2 == 1)) return false;
    return true;
}
static_assert(gk21_gauss_odd(), "Gauss weights expected at odd nodes only");

template <bool UNROLL = false>
GL_HD double gk_piece(const Frame& F, double cc, double sc, double mid, double half, Sums& K)
{
    // With u = 1 - tau^2 and inv = 1/(1 + tau^2), cos and sin of the angle are
    // (cc u - 2 sc tau) inv and (sc u + 2 cc tau) inv, so every quantity that
    // is linear in them is (a u + b tau) inv with a, b fixed on the piece:
    // x - x0, y - y0, dx, dy and the flat integrand x y' - y x' - P0.
    const double axu = F.Xc * cc + F.Xs * sc, axt = 2.0 * (F.Xs * cc - F.Xc * sc);
    const double ayu = F.Yc * cc + F.Ys * sc, ayt = 2.0 * (F.Ys * cc - F.Yc * sc);
    const double dxu = 0.5 * axt, dxt = -2.0 * axu;
    const double dyu = 0.5 * ayt, dyt = -2.0 * ayu;
    const double fu = F.P1 * cc + F.P2 * sc, ft = 2.0 * (F.P2 * cc - F.P1 * sc);
    double kf = 0.0, kl = 0.0, kq = 0.0, gf = 0.0, gl = 0.0;
    auto node = [&](int j, auto gauss) {
        const double tau = mid + half * GK21_M[j];
        const double d = fma(tau, tau, 1.0);
        const double inv = rcp_q(d);
        const double u = 2.0 - d;
        const double x = fma(inv, fma(axu, u, axt * tau), F.x0);
        const double y = fma(inv, fma(ayu, u, ayt * tau), F.y0);
        const double tdx = fma(dxu, u, dxt * tau), tdy = fma(dyu, u, dyt * tau);  // dx, dy / inv
        const double x2 = x * x, y2 = y * y;
        const double om = fmax(0.0, 1.0 - x2 - y2);
        const double w = sqrt_q(om);
        const double G = 1.0 + om * rcp_q(1.0 + w);         // (1 + w + w^2)/(1 + w)
        const double inv2 = inv * inv;
        const double fl = fma(inv2, fma(fu, u, ft * tau), inv * F.P0);  // (x y' - y x') dpsi/dtau / 2
        const double li = fl * G;
        const double tq = x * (x2 * (1.0 / 3.0) + y2) * tdy - y * (x2 + y2 * (1.0 / 3.0)) * tdx;
        kf += GK21_WK[j] * fl;
        kl += GK21_WK[j] * li;
        kq += GK21_WK[j] * (inv2 * tq);
        if constexpr (decltype(gauss)::value) {
            gf += GK21_WG[j] * fl;
            gl += GK21_WG[j] * li;
        }
    };
    // same nodes in the same order either way; unrolled, the rule's constants
    // become immediates (no table loads inside the loop) and the Kronrod-only
    // nodes (even j, zero Gauss weight) skip the Gauss sums
    if (UNROLL) {
#pragma unroll
        for (int jj = 0; jj < 10; ++jj) {
            node(2 * jj, std::false_type{});
            node(2 * jj + 1, std::true_type{});
        }
        node(20, std::false_type{});
    } else {
#pragma unroll 1
        for (int j = 0; j < 21; ++j) node(j, std::true_type{});
    }
    // dpsi factor 2, f_flat = flat/2, f_lin = (2/3) G flat/2, f_quad = quad/2
    K.flat += half * kf;
    K.lin += half * kl * (2.0 / 3.0);
    K.quad += half * kq;
    return half * (fabs(kf - gf) + (2.0 / 3.0) * fabs(kl - gl));
}

// Whole arc tau in [-h, h]: one or two Gauss-Kronrod pieces (arc_start_level),
// re-split uniformly into 2, 4, ... pieces until the summed Gauss-Kronrod
// difference is below kArcTol (L0 >= 0 forces the starting level).  An arc
// still above it at kArcMaxLevel is accepted there and counted (ct.unconverged).
template <class CT>
GL_HD_CALL void arc_gk(const Frame& F, double cc, double sc, double h, Sums& S, CT& ct, int L0 = -1)
{
    for (int L = L0 < 0 ? arc_start_level(h) : L0;; ++L) {
        const int np = 1 << L;
        const double half = h / np;
        Sums K = {0.0, 0.0, 0.0};
        double err = 0.0;
        for (int p = 0; p < np; ++p) {
            err += gk_piece(F, cc, sc, -h + (2 * p + 1) * half, half, K);
            ct.arc();
        }
        if (err <= kArcTol || L == kArcMaxLevel) {
            if (err > kArcTol) ct.unconverged();
            S.flat += K.flat;
            S.lin += K.lin;
            S.quad += K.quad;
            return;
        }
    }
}

// Orders of the periodic trapezoid rule for a whole ellipse on the star, and
// cos/sin of their steps 2 pi / n.
constexpr int kTrapOrders = 9;
constexpr int kTrapN[kTrapOrders] = {8, 12, 16, 20, 24, 32, 40, 48, 64};

// Weights 2 pi / (3 n) of the trapezoid sums of the mu integral.
constexpr double kTrapW[kTrapOrders] = {
    kTwoPi / (3.0 * 8), kTwoPi / (3.0 * 12), kTwoPi / (3.0 * 16), kTwoPi / (3.0 * 20), kTwoPi / (3.0 * 24),
    kTwoPi / (3.0 * 32), kTwoPi / (3.0 * 40), kTwoPi / (3.0 * 48), kTwoPi / (3.0 * 64)};

// cos and sin of the trapezoid steps 2 pi / n (a table read by index: as
// literals the compiler keeps all of them in registers across a caller's loop).
static constexpr double kTrapStepC[kTrapOrders] = {
    0.70710678118654757, 0.86602540378443860, 0.92387953251128674, 0.95105651629515353, 0.96592582628906831,
    0.98078528040323043, 0.98768834059513777, 0.99144486137381038, 0.99518472667219693};
static constexpr double kTrapStepS[kTrapOrders] = {
    0.70710678118654757, 0.5, 0.38268343236508978, 0.30901699437494740, 0.25881904510252074,
    0.19509032201612825, 0.15643446504023087, 0.13052619222005157, 0.098017140329560604};

GL_HD void trap_step(int i, double& c, double& s)
{
    c = kTrapStepC[i];
    s = kTrapStepS[i];
}

// Smallest trapezoid order n with n * d >= L, where d is the distance of the
// nearest complex zero of 1 - r^2(th) from the real th axis (error ~ exp(-n d)).
// The caller passes r = cosh(d) (or a lower bound of it), compared here with
// cosh(L / n).  Returns -1 if even the largest order is not enough.
constexpr double kTrapL = 24.0;
constexpr double kTrapCosh[9] = {
    // cosh(24 / n) for n = 8, 12, 16, 20, 24, 32, 40, 48, 64
    10.0676619957778, 3.7621956910836, 2.3524096152432, 1.8106555673244, 1.5430806348152,
    1.2946832846768, 1.1854652182423, 1.1276259652064, 1.0711403467046};

GL_HD int trap_order_cosh(double r)
{
    for (int i = 0; i < kTrapOrders; ++i)
        if (r >= kTrapCosh[i]) return i;
    return -1;
}

GL_HD int trap_order(double d)
{
    for (int i = 0; i < kTrapOrders; ++i)
        if (kTrapN[i] * d >= kTrapL) return i;
    return -1;
}

// Whole ellipse, periodic trapezoid with n = kTrapN[oi] equally spaced nodes in
// th (the integrand is periodic and analytic in a strip): mu integral.  Nodes
// come in pairs +-th_j from a rotation recurrence.  (Inlined form; trap_lin
// below is the same rule as an out-of-line call.)
GL_HD double trap_lin_inl(const SetConst& s, double x0, double y0, int oi)
{
    const double P1 = x0 * s.C, P2 = y0 * s.A - x0 * s.B;
    const int n = kTrapN[oi];
    double rc, rs;
    trap_step(oi, rc, rs);
    // (1 - r^2 > 0 at every node: the class guarantees a margin to the limb)
    auto node = [&](double c, double sn) {
        const double x = x0 + s.A * c;
        const double y = y0 + s.B * c + s.C * sn;
        const double om = 1.0 - x * x - y * y;
        const double w = sqrt_qp(om);
        return (1.0 + om * rcp_q(1.0 + w)) * (s.AC + P1 * c + P2 * sn);
    };
    double acc = node(1.0, 0.0) + node(-1.0, 0.0);
    double c = rc, sn = rs;
    for (int j = 1; j < n / 2; ++j) {
        acc += node(c, sn) + node(c, -sn);
        const double cn = c * rc - sn * rs;
        sn = sn * rc + c * rs;
        c = cn;
    }
    return acc * kTrapW[oi];
}

GL_HD_CALL double trap_lin(const SetConst& s, double x0, double y0, int oi)
{
    return trap_lin_inl(s, x0, y0, oi);
}

// Whole ellipse, nested periodic trapezoid: 8, 16, 32, 64 nodes, each level
// adding the midpoints of the previous one.  Returns true (and the mu
// integral) once two successive levels agree to kTrapTol, judged from the
// 16/32 pair on and only while the differences shrink (a coarse level can
// agree with the next by accident before the convergence is exponential).
GL_HD bool trap_lin_nested_inl(const SetConst& s, double x0, double y0, double& out, int& levels)
{
    const double P1 = x0 * s.C, P2 = y0 * s.A - x0 * s.B;
    auto node = [&](double c, double sn) {
        const double x = x0 + s.A * c;
        const double y = y0 + s.B * c + s.C * sn;
        const double om = fmax(0.0, 1.0 - x * x - y * y);
        const double w = sqrt_q(om);
        return (1.0 + om * rcp_q(1.0 + w)) * (s.AC + P1 * c + P2 * sn);
    };
    // level 8: nodes k pi/4
    double sum = node(1.0, 0.0) + node(-1.0, 0.0) + node(0.0, 1.0) + node(0.0, -1.0);
    {
        const double r = TRAP_PI_C[0];  // cos(pi/4) = sin(pi/4)
        sum += node(r, r) + node(r, -r) + node(-r, r) + node(-r, -r);
    }
    int n = 8;
    double wn = kTwoPi / (3.0 * 8);  // 2 pi / (3 n), halved exactly with each level
    double prev = sum * wn;
    double prev_diff = 1e300;
    levels = 1;
#pragma unroll 1
    for (int L = 1; L <= 3; ++L) {
        // midpoints (2j + 1) pi / n, j = 0 .. n/2 - 1, in +- pairs
        const double c0 = TRAP_PI_C[L], s0 = TRAP_PI_S[L];          // pi / n
        const double rc = TRAP_PI_C[L - 1], rs = TRAP_PI_S[L - 1];  // 2 pi / n
        double c = c0, sn = s0, add = 0.0;
#pragma unroll 2
        for (int j = 0; j < n / 2; ++j) {
            add += node(c, sn) + node(c, -sn);
            const double cn = c * rc - sn * rs;
            sn = sn * rc + c * rs;
            c = cn;
        }
        sum += add;
        n *= 2;
        wn *= 0.5;
        const double cur = sum * wn;
        const double diff = fabs(cur - prev);
        ++levels;
        if (n >= 32 && diff <= kTrapTol && diff <= prev_diff) {
            out = cur;
            return true;
        }
        prev = cur;
        prev_diff = diff;
    }
    out = prev;
    return false;
}

GL_HD_CALL bool trap_lin_nested(const SetConst& s, double x0, double y0, double& out, int& levels)
{
    return trap_lin_nested_inl(s, x0, y0, out, levels);
}

// Limb arc, counter-clockwise from unit vector direction (xa, ya) to (xb, yb).
GL_HD void limb_sums(double xa, double ya, double xb, double yb, Sums& S)
{
    const double dl = atan2_d(xa * yb - ya * xb, xa * xb + ya * yb);
    const double ra = rcp(xa * xa + ya * ya), rb = rcp(xb * xb + yb * yb);
    // sin(4 lambda) = 4 x y (x^2 - y^2) / r^4
    const double s4a = 4.0 * xa * ya * (xa * xa - ya * ya) * ra * ra;
    const double s4b = 4.0 * xb * yb * (xb * xb - yb * yb) * rb * rb;
    S.flat += 0.5 * dl;
    S.lin += dl * (1.0 / 3.0);
    S.quad += 0.25 * dl - (s4b - s4a) * (1.0 / 48.0);
}

// Arc between half-angle tangents ta -> tb (counter-clockwise in psi; passes
// through psi = pi when tb < ta), described for the tau rule as a centre
// direction (cc, sc) and h = tan(span/4); arcs longer than pi are split in two.
struct TauArc {
    double cc, sc, h;
};

GL_HD int arc_between(double ta, double tb, TauArc* out)
{
    const double Na = sqrt_nn(1.0 + ta * ta), Nb = sqrt_nn(1.0 + tb * tb);
    const double sg = (tb > ta) ? 1.0 : -1.0;
    // h = tan(span/4), centre psi_c = atan(ta) + atan(tb) (+ pi when wrapping)
    const double h = sg * (tb - ta) / (Na * Nb + sg * (1.0 + ta * tb));
    const double inv = sg / (Na * Nb);
    const double cc = (1.0 - ta * tb) * inv, sc = (ta + tb) * inv;
    if (h <= 1.0) {
        out[0] = {cc, sc, h};
        out[1] = out[0];  // (both slots always written: they stay in registers)
        return 1;
    }
    const double q = sqrt_nn(1.0 + h * h);
    const double r = rcp(q);
    const double cq = r, sq = h * r;                  // quarter-span angle
    const double h2 = h * rcp(1.0 + q);               // tan(span/8)
    out[0] = {cc * cq + sc * sq, sc * cq - cc * sq, h2};
    out[1] = {cc * cq - sc * sq, sc * cq + cc * sq, h2};
    return 2;
}

GL_HD void point_at(const Frame& F, double t, double& x, double& y)
{
    const double t2 = t * t, inv = rcp(1.0 + t2);
    const double cu = (1.0 - t2) * inv, su = 2.0 * t * inv;
    x = F.x0 + F.Xc * cu + F.Xs * su;
    y = F.y0 + F.Yc * cu + F.Ys * su;
}

// A local maximum of r^2 on the star whose nearby pair of complex zeros of
// 1 - r^2 lies closer than this to the real th axis becomes a cluster point.
constexpr double kSplitDist = 0.4;

enum SampleClass : int { CLS_OUT = 0, CLS_FULL = 1, CLS_PARTIAL = 2 };

// Lower bound on cosh(b) for any complex zero th = a + i b of |p(th)|^2 - 1
// when the ellipse lies inside the disk.  With e(th) = cosh b e(a) + i sinh b e'(a),
// p = u + i v where |u| <= rho + k cosh b and |v| >= kq sinh b (kq: minor
// semi-axis); a zero needs |u|^2 - |v|^2 = 1, hence
//   k^2 (1 - q^2) c^2 + 2 rho k c + rho^2 + (kq)^2 - 1 >= 0,  c = cosh b.
// Returns the smallest such c (>= 1), or 1 when no bound applies.  The
// coefficients that depend on the set only come precomputed (zA, z2A_inv, zC0).
GL_HD double zero_cosh_bound(const SetConst& s, double rho2, double rho)
{
    const double B = 2.0 * rho * s.k;
    const double C = rho2 + s.zC0;
    if (C >= 0.0) return 1.0;
    double c;
    if (s.z2A_inv > 0.0) c = (-B + sqrt_nn(B * B - 4.0 * s.zA * C)) * s.z2A_inv;
    else c = B > 0.0 ? -C * rcp(B) : 1e300;
    return fmax(c, 1.0);
}

// Classification of a sample by its ellipse centre: kOffDisk when the ellipse
// cannot touch the disk, the trapezoid order index (>= 0) when the rigorous
// singularity bound proves the whole ellipse lies well inside the disk, kHard
// otherwise.
constexpr int kOffDisk = -2;
constexpr int kHard = -1;

GL_HD int easy_class(const SetConst& s, double x0, double y0)
{
    const double rho2 = x0 * x0 + y0 * y0;
    const double kp = 1.0 + s.k;
    if (rho2 >= kp * kp) return kOffDisk;
    const double rho = sqrt_nn(rho2);
    const double cosh_bound = zero_cosh_bound(s, rho2, rho);
    const int oi = trap_order_cosh(cosh_bound);
    return oi < 0 ? kHard : oi;
}

// Occulted fraction of a whole ellipse on the disk from its mu integral sl:
// the area and the r^2 moment of the ellipse are closed forms.
GL_HD double whole_delta(const SetConst& s, double x0, double y0, double sl)
{
    const double rho2 = x0 * x0 + y0 * y0;
    const double S_flat_whole = kPi * s.AC;
    const double S_quad_whole = kPi * s.AC * (rho2 + 0.25 * s.M2);
    return (s.c0 * S_flat_whole + s.c1 * sl + s.c2 * S_quad_whole) * s.inv_phi;
}

// Easy samples: the ellipse cannot touch the disk, or provably lies well
// inside it (periodic trapezoid, order from the singularity bound).  Returns
// true and the occulted fraction when the sample is easy.
template <class CT = NoCensus>
GL_HD bool occulted_easy(const SetConst& s, double x0, double y0, double& delta, int* cls_out,
                         CT& ct)
{
    const int oi = easy_class(s, x0, y0);
    if (oi == kOffDisk) {
        if (cls_out) *cls_out = CLS_OUT;
        delta = 0.0;
        return true;
    }
    if (oi == kHard) return false;
    if (cls_out) *cls_out = CLS_FULL;
    ct.trap(kTrapN[oi]);
    delta = whole_delta(s, x0, y0, trap_lin(s, x0, y0, oi));
    return true;
}

// What a hard sample needs before its boundary is walked: the intersection
// quartic in t = tan(psi/2) about the anchor th0, its real roots and critical
// points, and the cluster points (local maxima of r^2 on the star whose
// nearby complex zeros come close to the real axis).
struct HardPrep {
    Poly4 q;
    QuarticRoots R;
    double c0a, s0a;  // cos, sin of the anchor th0
    double tc[3];     // cluster points in the slots of their critical points
    bool tv[3];
    int ntc;
    double t_near;    // the local maximum nearest the limb
    bool inf_inside;  // t = +-inf (th = th0 + pi) lies on the star

    // a single cluster point at t (a whole ellipse whose nested rule did not settle)
    GL_HD void single_cluster(double t)
    {
        tc[0] = t;
        tc[1] = tc[2] = 0.0;
        tv[0] = true;
        tv[1] = tv[2] = false;
        ntc = 1;
    }
};

template <class CT, bool INLINE_SOLVE = false>
GL_HD void hard_prepare(const SetConst& s, double x0, double y0, HardPrep& H, CT& ct)
{
    const double rho2 = x0 * x0 + y0 * y0;
    // g(th) = |p(th)|^2 - 1 = K0 + K1 cos + K2 sin + K3 cos 2th + K4 sin 2th
    const double K0 = rho2 - 1.0 + 0.5 * s.M2;
    const double K1 = 2.0 * (x0 * s.A + y0 * s.B);
    const double K2 = 2.0 * y0 * s.C;
    const double nK2 = K1 * K1 + K2 * K2;
    double cf = 1.0, sf = 0.0;  // direction of the far point th_far
    if (nK2 > 1e-300) {
        const double inv = rcp(sqrt_nn(nK2));
        cf = K1 * inv;
        sf = K2 * inv;
    }
    // anchor th0 so that t = +-inf (th = th0 + pi) is where |g| is largest
    // among th_far + {0, pi/2, pi, 3pi/2}
    double best_c = cf, best_s = sf, best_g = 0.0;
    {
        double cc = cf, ss = sf;
        for (int i = 0; i < 4; ++i) {
            const double c2 = cc * cc - ss * ss, s2 = 2.0 * cc * ss;
            const double gv = K0 + K1 * cc + K2 * ss + s.K3 * c2 + s.K4 * s2;
            if (fabs(gv) > fabs(best_g)) {
                best_g = gv;
                best_c = cc;
                best_s = ss;
            }
            const double tmp = cc;
            cc = -ss;
            ss = tmp;
        }
    }
    const double c0a = -best_c, s0a = -best_s;  // th0 = th_best + pi
    H.c0a = c0a;
    H.s0a = s0a;
    // g(th0 + psi) = K0 + K1' cos psi + K2' sin psi + K3' cos 2psi + K4' sin 2psi
    const double K1r = K1 * c0a + K2 * s0a;
    const double K2r = -K1 * s0a + K2 * c0a;
    const double c2a = c0a * c0a - s0a * s0a, s2a = 2.0 * c0a * s0a;
    const double K3r = s.K3 * c2a + s.K4 * s2a;
    const double K4r = -s.K3 * s2a + s.K4 * c2a;
    // (1 + t^2)^2 g as a quartic in t = tan(psi/2)
    Poly4& q = H.q;
    q.a4 = K0 - K1r + K3r;
    q.a3 = 2.0 * K2r - 4.0 * K4r;
    q.a2 = 2.0 * K0 - 6.0 * K3r;
    q.a1 = 2.0 * K2r + 4.0 * K4r;
    q.a0 = K0 + K1r + K3r;
    if (INLINE_SOLVE) solve_quartic_inl(q, H.R, ct);
    else solve_quartic(q, H.R, ct);
    H.inf_inside = q.a4 < 0.0;

    // local maxima of r^2 on the star: the nearby complex zeros of the quartic
    // sit at t_c +- i sqrt(2|p|/|p''|), about 2 sqrt(2|p|/|p''|)/(1+t_c^2) in th
    H.ntc = 0;
    H.t_near = 0.0;
    double d_near = 1e300;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        H.tc[i] = 0.0;
        H.tv[i] = false;
        if (!H.R.cv[i]) continue;
        const double t = H.R.c[i];
        const double pv = p4(q, t), pp = ddp4(q, t);
        if (pv < 0.0 && pp < 0.0) {
            const double dth = 2.0 * sqrt_nn(2.0 * pv * rcp(pp)) * rcp(1.0 + t * t);
            if (dth < d_near) {
                d_near = dth;
                H.t_near = t;
            }
            if (dth < kSplitDist) {
                H.tc[i] = t;
                H.tv[i] = true;
                ++H.ntc;
            }
        }
    }
}

// Class of a prepared hard sample: no crossing with t = inf off the star means
// the ellipse lies off the disk; no crossing otherwise means whole on the disk.
GL_HD int hard_class(const HardPrep& H)
{
    if (H.R.n_roots < 2) return H.inf_inside ? CLS_FULL : CLS_OUT;
    return CLS_PARTIAL;
}

// Break points of the boundary of E cap D in t, ascending (kind 0 = root,
// 1 = cluster point), in bp[0..nb) (nb is returned; the rest of the 7 slots
// hold +huge).  A whole ellipse needs at least one cluster point (a single
// one gets the diametrically opposite point as its partner).  Merged by a
// 16-comparator sorting network so that every index is static.
GL_HD void sort_pair(double& ka, int& da, double& kb, int& db)
{
    const bool sw = kb < ka;
    const double k0 = sw ? kb : ka, k1 = sw ? ka : kb;
    const int d0 = sw ? db : da, d1 = sw ? da : db;
    ka = k0;
    kb = k1;
    da = d0;
    db = d1;
}

GL_HD int hard_breaks(HardPrep& H, double* bp, int* kind)
{
    constexpr double kNone = 1e300;
    const bool whole = H.R.n_roots < 2;
    if (whole && H.ntc == 1) {
        // second break point diametrically opposite: psi + pi <-> -1/t
        // the one cluster point (empty slots hold 0; a sum, not a selection
        // of slots, keeps the slots in registers)
        const double t = H.tc[0] + H.tc[1] + H.tc[2];
        const double o = (t != 0.0) ? -1.0 / t : -1e16;
        H.tc[0] = fmin(t, o);
        H.tc[1] = fmax(t, o);
        H.tc[2] = 0.0;
        H.tv[0] = H.tv[1] = true;
        H.tv[2] = false;
        H.ntc = 2;
    }
    double k[7];
    int d[7];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        k[i] = (!whole && H.R.rv[i]) ? H.R.r[i] : kNone;
        d[i] = 0;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        k[4 + i] = H.tv[i] ? H.tc[i] : kNone;
        d[4 + i] = 1;
    }
    sort_pair(k[0], d[0], k[6], d[6]);
    sort_pair(k[2], d[2], k[3], d[3]);
    sort_pair(k[4], d[4], k[5], d[5]);
    sort_pair(k[0], d[0], k[2], d[2]);
    sort_pair(k[1], d[1], k[4], d[4]);
    sort_pair(k[3], d[3], k[6], d[6]);
    sort_pair(k[0], d[0], k[1], d[1]);
    sort_pair(k[2], d[2], k[5], d[5]);
    sort_pair(k[3], d[3], k[4], d[4]);
    sort_pair(k[1], d[1], k[2], d[2]);
    sort_pair(k[4], d[4], k[6], d[6]);
    sort_pair(k[2], d[2], k[3], d[3]);
    sort_pair(k[4], d[4], k[5], d[5]);
    sort_pair(k[1], d[1], k[2], d[2]);
    sort_pair(k[3], d[3], k[4], d[4]);
    sort_pair(k[5], d[5], k[6], d[6]);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        bp[i] = k[i];
        kind[i] = d[i];
    }
    return (whole ? 0 : H.R.n_roots) + H.ntc;
}

// Walks the boundary between consecutive break points: ellipse arcs on the
// star go to arc(cc, sc, h, level) (as tau-rule arcs, split when longer than
// pi, with the starting level of the arc rule); limb arcs are added to S in
// closed form when `limbs` is set.  Returns the number of ellipse arcs.  Most
// samples have one piece of each kind: the first ellipse piece and the first
// limb piece are taken out of the loop over break points, so that all lanes of
// a wavefront run each kind once together instead of splitting between the two
// kinds at every break point; further pieces (cluster points, four crossings)
// follow in the loop.  Either kind is still taken in ascending order.
template <class ArcFn, class CT>
GL_HD int boundary_walk(const HardPrep& H, const Frame& F, const double* bp, const int* kind,
                        int nb, Sums& S, bool limbs, ArcFn&& arc, CT& ct)
{
    unsigned more = 0u;  // bit i: piece i is not the first of its kind
    bool seen_in = false, seen_out = false;
    double ia = 0.0, ib = 0.0, oa = 0.0, ob = 0.0;  // first ellipse and first limb piece
    unsigned on = 0u;                                // bit i: piece i lies on the star
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        if (i >= nb) break;
        const bool wrap = i + 1 == nb;  // the piece from the last break point back to the first
        const double ta = bp[i], tb = wrap ? bp[0] : bp[i + 1 < 7 ? i + 1 : 0];
        const int ka = kind[i], kb = wrap ? kind[0] : kind[i + 1 < 7 ? i + 1 : 0];
        bool inside;
        if (ka == 1 || kb == 1) inside = true;  // cluster points lie on the star
        else if (!wrap) inside = p4(H.q, 0.5 * (ta + tb)) < 0.0;
        else inside = H.inf_inside;              // the piece through t = inf
        const bool first = inside ? !seen_in : !seen_out;
        if (inside && first) {
            ia = ta;
            ib = tb;
        }
        if (!inside && first) {
            oa = ta;
            ob = tb;
        }
        seen_in = seen_in || inside;
        seen_out = seen_out || !inside;
        on |= (inside ? 1u : 0u) << i;
        more |= (first ? 0u : 1u) << i;
    }
    int n_arcs = 0;
    auto ellipse_piece = [&](double ta, double tb) {
        TauArc arcs[2];
        const int na = arc_between(ta, tb, arcs);
        arc(arcs[0].cc, arcs[0].sc, arcs[0].h, arc_start_level(arcs[0].h));
        if (na == 2) arc(arcs[1].cc, arcs[1].sc, arcs[1].h, arc_start_level(arcs[1].h));
        n_arcs += na;
    };
    auto limb_piece = [&](double ta, double tb) {
        double xa, ya, xb, yb;
        point_at(F, ta, xa, ya);
        point_at(F, tb, xb, yb);
        limb_sums(xa, ya, xb, yb, S);
        ct.limb();
    };
    if (seen_in) ellipse_piece(ia, ib);
    if (more & on) {
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            if (((more & on) >> i) & 1u) {
                const bool wrap = i + 1 == nb;
                ellipse_piece(bp[i], wrap ? bp[0] : bp[i + 1 < 7 ? i + 1 : 0]);
            }
        }
    }
    if (limbs) {
        if (seen_out) limb_piece(oa, ob);
        if (more & ~on) {
#pragma unroll
            for (int i = 0; i < 7; ++i) {
                if (((more & ~on) >> i) & 1u) {
                    const bool wrap = i + 1 == nb;
                    limb_piece(bp[i], wrap ? bp[0] : bp[i + 1 < 7 ? i + 1 : 0]);
                }
            }
        }
    }
    return n_arcs;
}

// Occulted fraction from the three boundary sums.
GL_HD double sums_delta(const SetConst& s, const Sums& S)
{
    return (s.c0 * S.flat + s.c1 * S.lin + s.c2 * S.quad) * s.inv_phi;
}

// Hard samples (everything occulted_easy declines): intersection quartic,
// near-limb whole ellipses, limb and ellipse arcs.
template <class CT = NoCensus>
GL_HD double occulted_hard(const SetConst& s, double x0, double y0, int* cls_out, CT& ct)
{
    HardPrep H;
    hard_prepare(s, x0, y0, H, ct);
    const int cls = hard_class(H);
    if (cls_out) *cls_out = cls;
    if (cls == CLS_OUT) return 0.0;
    if (cls == CLS_FULL && H.ntc == 0) {
        double sl;
        int lev;
        const bool ok = trap_lin_nested(s, x0, y0, sl, lev);
        ct.trap(8 << (lev - 1));
        if (ok) return whole_delta(s, x0, y0, sl);
        H.single_cluster(H.t_near);  // did not settle: cluster at the point nearest the limb
    }
    double bp[7];
    int kind[7];
    const int nb = hard_breaks(H, bp, kind);
    Frame F;
    make_frame(s, x0, y0, H.c0a, H.s0a, F);
    Sums S = {0.0, 0.0, 0.0};
    boundary_walk(H, F, bp, kind, nb, S, true,
                  [&](double cc, double sc, double h, int lev) { arc_gk(F, cc, sc, h, S, ct, lev); }, ct);
    return sums_delta(s, S);
}

// Occulted fraction delta for ellipse centre (x0, y0).
template <class CT = NoCensus>
GL_HD double occulted(const SetConst& s, double x0, double y0, int* cls_out, CT& ct)
{
    double d;
    if (occulted_easy<CT>(s, x0, y0, d, cls_out, ct)) return d;
    return occulted_hard<CT>(s, x0, y0, cls_out, ct);
}

// Planet centre at time t (eq. coord-map with a circular orbit); returns false
// when the planet is behind the star or cannot touch the disk.
GL_HD bool centre_at(const SetConst& s, double t, double& x0, double& y0)
{
    const double tau = phase_time(s, t);
    const double alpha = s.w_orb * tau;
    double sa, ca;
    sincos_pi(alpha, sa, ca);
    x0 = s.xb * ca;
    y0 = s.d * sa;
    return ca > 0.0;
}

// Relative flux of one instantaneous sub-sample.
template <class CT = NoCensus>
GL_HD double flux_instant(const SetConst& s, double t, int* cls_out, CT& ct)
{
    double x0, y0;
    if (!centre_at(s, t, x0, y0)) {
        if (cls_out) *cls_out = CLS_OUT;
        return 1.0;
    }
    return 1.0 - occulted<CT>(s, x0, y0, cls_out, ct);
}

GL_HD double flux_instant(const SetConst& s, double t)
{
    NoCensus nc;
    return flux_instant<NoCensus>(s, t, nullptr, nc);
}

// ---------------------------------------------------------------- the paper's integrator
// Section 2 of the paper evaluates the Green's-theorem line integrals without
// solving for the crossings: the ellipse boundary is sampled at equally
// spaced theta, a point outside the stellar disk is moved radially onto the
// limb (the point at the same angle lambda, with dlambda/dtheta carrying the
// parametrisation), the three integrands f_flat, f_lin, f_quad are evaluated
// at the (possibly moved) point, and each sum is taken by Simpson's rule; in
// single precision.  Kept here beside the exact path for comparison.


// Occulted fraction for ellipse centre (x0, y0) by the snapped boundary and
// a periodic Simpson rule over n (even) nodes: weights 2, 4, 2, ..., 4 times
// h / 3 (the first node is also the last).  FP32 throughout; the set's
// constants and the centre are rounded to FP32 here.
// FP32 operations per node inside the disk, counted from snap_node below and
// the weighted accumulation (FMA = 2, square root and reciprocal = 1); a
// moved node adds 11
constexpr int kFlopSnapNode = 48;

// One node of the rule at (cos, sin) of theta: the integrands f_flat, f_lin
// (without its 2/3) and f_quad at the boundary point, moved onto the limb if
// it lies outside the disk.  snap_delta below runs it in one lane's loop;
// the batch kernel spreads the nodes of one sample over a wavefront's lanes.
GL_HD void snap_node(float A, float B, float C, float x0, float y0, float cs, float sn, float& ff, float& fl,
                     float& fq)
{
    float x = fmaf(A, cs, x0), y = fmaf(C, sn, fmaf(B, cs, y0));
    float dx = -A * sn, dy = fmaf(C, cs, -B * sn);
    float r2 = fmaf(x, x, y * y);
    if (r2 > 1.0f) {
        const float dl = (x * dy - y * dx) * rcp_f(r2);
        const float ir = rsqrt_f(r2);
        x *= ir;
        y *= ir;
        dx = -y * dl;
        dy = x * dl;
        r2 = 1.0f;
    }
    ff = 0.5f * (x * dy - y * dx);
    const float w = sqrt_f(fmaxf(0.0f, 1.0f - r2));
    fl = fmaf(w, w, 1.0f + w) * rcp_f(1.0f + w) * ff;
    const float x2 = x * x, y2 = y * y;
    fq = 0.5f * (x * fmaf(x2, 1.0f / 3.0f, y2) * dy - y * fmaf(y2, 1.0f / 3.0f, x2) * dx);
}

GL_HD float snap_delta(const SetConst& s, double x0d, double y0d, int n)
{
    const float x0 = (float)x0d, y0 = (float)y0d;
    const float A = (float)s.A, B = (float)s.B, C = (float)s.C;
    float sf = 0.0f, sl = 0.0f, sq = 0.0f;
    for (int i = 0; i < n; ++i) {
        // cos / sin of the node angle, from double precision (the batch kernel
        // reads the same values from a table)
        const double th = kTwoPi * (double)i / (double)n;
        float ff, fl, fq;
        snap_node(A, B, C, x0, y0, (float)cos(th), (float)sin(th), ff, fl, fq);
        const float wt = (i & 1) ? 4.0f : 2.0f;
        sf = fmaf(wt, ff, sf);
        sl = fmaf(wt, fl, sl);
        sq = fmaf(wt, fq, sq);
    }
    const float h3 = (float)(kTwoPi / 3.0) / (float)n;
    const float S_flat = sf * h3, S_lin = sl * h3 * (2.0f / 3.0f), S_quad = sq * h3;
    return ((float)s.c0 * S_flat + (float)s.c1 * S_lin + (float)s.c2 * S_quad) * (float)s.inv_phi;
}

// Relative flux of one instantaneous sub-sample by the paper's integrator.
GL_HD float flux_snap(const SetConst& s, double t, int n)
{
    double x0, y0;
    if (!centre_at(s, t, x0, y0)) return 1.0f;
    if (x0 * x0 + y0 * y0 >= (1.0 + s.k) * (1.0 + s.k)) return 1.0f;  // no overlap: nothing to integrate
    return 1.0f - snap_delta(s, x0, y0, n);
}

// Algorithmic FP64 operation counts per unit of counted work (add, sub, mul,
// divide, square root and library transcendental = 1, fused multiply-add = 2),
// read off the source of this file; the census multiplies them by what a
// launch really did.
constexpr int kFlopSample = 40;     // in-window sub-sample: phase, orbit, classify
constexpr int kFlopWhole = 30;      // whole-ellipse closed forms and singularity bound
constexpr int kFlopGuess = 97;      // closed-form first iterates (cubic 28, quartic 69)
constexpr int kFlopPartial = 160 + kFlopGuess;  // quartic set-up, frame, break points
constexpr int kFlopIter = 18;       // one safeguarded-Newton step on the quartic or cubic
constexpr int kFlopLimb = 30;       // one limb arc in closed form
constexpr int kFlopArc = 20;        // one ellipse arc set up for the tau rule
constexpr int kFlopTrapNode = 24;   // one trapezoid node (mu integrand + rotation)
constexpr int kFlopGKPiece = 21 * 64 + 10;  // one 21-node Gauss-Kronrod piece

// ---------------------------------------------------------------- surrogate helpers
// The equal-projected-area sphere: a circle of radius k sqrt(q) at the same
// centre (the oblate-minus-spherical residual of the surrogate is taken
// against it).
GL_HD SetConst sphere_of(const SetConst& s)
{
    SetConst c = s;
    const double r = sqrt_nn(s.AC);  // k^2 q = dx dy2
    c.A = r;
    c.B = 0.0;
    c.C = r;
    shape_terms(c, r);  // a circle: M2 = 2 k^2 q, K3 = K4 = 0, zA = 0
    return c;
}

// float -> BF16 bits, round to nearest even (the network's input rounding)
GL_HD unsigned short f2bf_rne(float f)
{
    unsigned int u = __builtin_bit_cast(unsigned int, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

constexpr int kSurFeat = 16;   // encoded features (zero-padded)
constexpr int kSurBinsRho = 24;
constexpr int kSurBinsQ = 8;
constexpr int kSurBins = kSurBinsRho * kSurBinsQ;

// Encodes one sample.  The instantaneous occultation depends on the nine
// inputs (k, f, theta, phi, b, a/R*, u1, u2, phase) only through k, the
// projected axis ratio q, the centre distance rho, the angle between the
// projected spin axis and the radial direction (mod pi; the flux is even in
// it) and u1, u2.  Writes the features, the residual scale k^2 (1 - q) and
// the calibration bin; returns false when the ellipse cannot touch the disk.
GL_HD bool sur_encode(const SetConst& s, double x0, double y0, float* feat, double& scale, int& bin)
{
    const double rho2 = x0 * x0 + y0 * y0, rho = sqrt_nn(rho2);
    const double k = s.k, q = s.AC / (k * k);
    if (rho >= 1.0 + k) return false;
    const double cd = rho > 0.0 ? (s.sx * x0 + s.sy * y0) / rho : 1.0;
    const double c2d = 2.0 * cd * cd - 1.0;
    const double u2 = s.c2, u1 = s.c1 - 2.0 * s.c2;
    const double z = fmin(fmax((rho - 1.0) / k, -6.0), 1.2);  // limb distance in planet radii
    const double f[kSurFeat] = {(k - 0.085) / 0.035, 2.0 * q - 1.0, z / 3.0, rho, c2d,
                                u1, u2, 1.0 - q, c2d * (1.0 - q), z * z / 9.0,
                                0, 0, 0, 0, 0, 0};
    for (int i = 0; i < kSurFeat; ++i) feat[i] = (float)f[i];
    scale = k * k * (1.0 - q) + 1e-30;
    int br = (int)((z + 6.0) / 7.2 * kSurBinsRho);
    br = br < 0 ? 0 : (br >= kSurBinsRho ? kSurBinsRho - 1 : br);
    int bq = (int)((1.0 - q) * kSurBinsQ);
    bq = bq < 0 ? 0 : (bq >= kSurBinsQ ? kSurBinsQ - 1 : bq);
    bin = br * kSurBinsQ + bq;
    return true;
}

}  // namespace gl
