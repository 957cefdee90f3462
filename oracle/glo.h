/*
 * glo.h -- CPU FP64 oracle for the oblate-planet transit light curve
 * (Price et al., "A long spin period for a sub-Neptune-mass exoplanet",
 * arXiv:2410.05408).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain, obviously
 * correct statement of what the GPU path computes.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * source, header, table or helper with the HIP library, and the HIP library
 * never calls it.
 *
 * What it computes (Section 2, "Ellipsoid Transit Model"): for a parameter set
 * and a time t, the fraction of the quadratically limb-darkened stellar flux
 * that stays visible when the sky-projected ellipse of an oblate spheroid on a
 * circular orbit covers part of the unit stellar disk:
 *
 *     F = 1 - (1/Phi) * Integral over (E intersect D) of I(r) dA,
 *     I(r) = 1 - u1 (1 - mu) - u2 (1 - mu)^2,   mu = sqrt(1 - r^2),
 *     Phi  = Integral over D of I dA.
 *
 * The area integral is evaluated as an iterated integral in the ellipse's own
 * frame (adaptive outer quadrature, clipped chords, closed-form inner
 * integral); see glo.c for the readings of the paper it rests on.
 *
 * Parameter block layout (shared with the GPU library's ABI by convention
 * only, no code): p[0..9] = k, f, theta, phi, b, a/R*, P, t0, q1, q2.
 *   k      equatorial radius / stellar radius       (0 < k < 1)
 *   f      flattening (R_eq - R_pol)/R_eq (eq. 1)   (0 <= f < 1)
 *   theta  angle between spin axis and line of sight, radians
 *   phi    sky rotation of the projected spin axis (the angle xi), radians
 *   b      impact parameter,  a/R* orbital distance (d),  P period (days),
 *   t0     mid-transit time (days),  q1, q2 Kipping (2013) LD parameters.
 */
#ifndef GLO_H
#define GLO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GLO_K, GLO_F, GLO_THETA, GLO_PHI, GLO_B, GLO_ARS, GLO_P, GLO_T0,
       GLO_Q1, GLO_Q2, GLO_NPARAM };

/* inner-integral modes for glo_occulted */
enum { GLO_INNER_CLOSED = 0, GLO_INNER_ADAPTIVE = 1 };

/* Kipping (2013) map q1,q2 -> u1,u2.  Returns 0, or -1 outside [0,1]^2. */
int glo_kipping(double q1, double q2, double *u1, double *u2);

/* Sky-plane geometry of the planet at time t.
 * out[0..1] centre (x0, y0); out[2] line-of-sight coordinate z of the centre
 * (z < 0 is the observer's side of the star); out[3..4] unit vector u_hat of
 * the semi-axis of length out[7] = k; out[5..6] unit vector s_hat (projected
 * spin axis) of the semi-axis of length out[8] = k*q.
 * Returns 1 when the planet is in front of the star, 0 otherwise. */
int glo_geometry(const double p[GLO_NPARAM], double t, double out[9]);

/* Occulted fraction delta = (1/Phi) * Integral_{E cap D} I dA for an ellipse
 * with centre (cx, cy), semi-axis k along (ux, uy) and k*q along the
 * perpendicular (uy, -ux), for limb-darkening coefficients u1, u2 given
 * directly (any real values with Phi > 0).  tol is the absolute target on
 * delta.  mode selects the inner integral (closed form or adaptive). */
double glo_occulted(double cx, double cy, double ux, double uy, double k,
                    double q, double u1, double u2, double tol, int mode);

/* Relative flux at output time t, box-averaged over an exposure t_exp with
 * n_ss midpoint sub-samples.  Returns 0 on success, -1 on a domain error
 * (then *out = NaN). */
int glo_flux(const double p[GLO_NPARAM], double t, double t_exp, int n_ss,
             double tol, double *out);

/* Batched convenience loop over the same layout as the GPU ABI:
 * params SoA [GLO_NPARAM][n_sets]; times either a shared grid of n_times
 * (offsets == NULL; out is [n_sets][n_times]) or CSR segments
 * times[offsets[s] .. offsets[s+1]) (out indexed like times).
 * n_ss / t_exp may be NULL (1 / 0).  Work is spread over nthreads OpenMP
 * threads (<= 0: all).  Returns the number of domain errors. */
int64_t glo_flux_batch(const double *params, int64_t n_sets,
                       const double *times, const int64_t *offsets,
                       int64_t n_times, const int32_t *n_ss,
                       const double *t_exp, double tol, double *out,
                       int nthreads);

/* Same loop restricted to a list of flat output indices (CSR or shared-grid
 * flat index); out_sel[i] receives the value for index sel[i]. */
int64_t glo_flux_select(const double *params, int64_t n_sets,
                        const double *times, const int64_t *offsets,
                        int64_t n_times, const int32_t *n_ss,
                        const double *t_exp, double tol, const int64_t *sel,
                        int64_t n_sel, double *out_sel, int nthreads);

/* Number of adaptive integrals, since the library was loaded, that stopped
 * with their error estimate above the target (out of panels, or a panel too
 * narrow to split).  The tests require it to stay 0. */
long glo_unconverged(void);

/* General ellipsoids: semi-axes a, b, c (stellar radii) along the body axes
 * x', y', z', orientation angles zeta, eta, xi (R = Rx(zeta) Ry(eta) Rz(xi),
 * Section 2 eq. coord-map), impact parameter, a/R*, P, t0, Kipping q1, q2,
 * and `locked` (1: the tidally-locked coordinate map of Appendix B). */
enum { GLO_E_RA, GLO_E_RB, GLO_E_RC, GLO_E_ZETA, GLO_E_ETA, GLO_E_XI, GLO_E_B, GLO_E_ARS, GLO_E_P,
       GLO_E_T0, GLO_E_Q1, GLO_E_Q2, GLO_E_LOCKED, GLO_E_NPARAM };

/* Centre (x, y, z), unit major axis u_hat, unit minor axis s_hat and the two
 * semi-axes (major, minor) of the sky shadow at time t; returns 1 when the
 * planet is on the observer's side. */
int glo_geometry_ell(const double p[GLO_E_NPARAM], double t, double out[9]);
int glo_flux_ell(const double p[GLO_E_NPARAM], double t, double t_exp, int n_ss, double tol, double *out);
int64_t glo_flux_batch_ell(const double *params, int64_t n_sets, const double *times, const int64_t *offsets,
                           int64_t n_times, const int32_t *n_ss, const double *t_exp, double tol, double *out,
                           int nthreads);

/* Number of OpenMP threads a batch call with nthreads <= 0 would use. */
int glo_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
