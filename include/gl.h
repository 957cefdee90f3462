/*
 * gl.h -- C ABI of the MI355X oblate-planet transit light-curve library.
 *
 * The library computes, for every (parameter set, time sample) pair, the
 * relative stellar flux of a star with quadratic limb darkening while the
 * sky-projected ellipse of an oblate spheroid on a circular orbit passes in
 * front of it (Price et al., arXiv:2410.05408, Section 2 "Ellipsoid Transit
 * Model": the coordinate map eq. coord-map, the projected boundary eqs. dx,
 * dy1, dy2, and the Green's-theorem integrands for quadratic limb darkening).
 * All arithmetic on the path is FP64 in hand-written HIP kernels for gfx950.
 *
 * Conventions shared by every entry point
 *  - Pointers marked "device" must point to device memory of the context's
 *    GPU (for example torch tensors on that device).  The library never frees
 *    or keeps caller pointers beyond the call; all work is only enqueued on
 *    `stream` (a hipStream_t, NULL = default stream) and runs asynchronously.
 *  - A context owns its workspace and launch plan and is used by one host
 *    thread at a time.  Calls that overlap on one context race.
 *  - Host-checkable errors (NULL pointers, sizes) return immediately and
 *    enqueue nothing.  Per-element domain errors (see gl_lightcurve_batch)
 *    write NaN to the affected outputs and set a device status word that
 *    gl_ctx_sync_status reports.
 *  - No C++ exception crosses this interface.
 */
#ifndef GL_H
#define GL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GL_OK = 0,
    GL_ERR_NULL = -1,    /* a required pointer is NULL */
    GL_ERR_SIZE = -2,    /* a size or count is out of range */
    GL_ERR_DOMAIN = -3,  /* device-side: some parameter set or grid was invalid */
    GL_ERR_DEVICE = -4,  /* a HIP runtime call failed (message in last_error) */
    GL_ERR_STATE = -5,   /* context not usable for this call */
    GL_ERR_NOMEM = -6    /* workspace allocation failed */
} gl_status;

/* Parameter block rows (SoA, double[GL_NPARAM][n_sets]):
 *  GL_K      equatorial radius / stellar radius, 0 < k < 1 (polar radius is k(1-f))
 *  GL_F      flattening (R_eq - R_pol)/R_eq, eq. 1, 0 <= f < 1
 *  GL_THETA  angle between spin axis and line of sight, rad (the paper's
 *            eta = pi/2 - theta)
 *  GL_PHI    sky rotation of the projected spin axis, rad (the paper's xi)
 *  GL_B      impact parameter, |b| < a/R*
 *  GL_ARS    orbital distance a/R* (the paper's d), > 1 + k
 *  GL_P      orbital period, days, > 0
 *  GL_T0     mid-transit time, days
 *  GL_Q1, GL_Q2  Kipping (2013) quadratic limb-darkening parameters in [0, 1]
 */
enum { GL_K, GL_F, GL_THETA, GL_PHI, GL_B, GL_ARS, GL_P, GL_T0, GL_Q1, GL_Q2, GL_NPARAM };

typedef struct gl_ctx gl_ctx;

/* Creates a context on HIP device `device` (sets it current for the call).
 * *ctx receives the context or NULL on failure. */
gl_status gl_ctx_create(gl_ctx **ctx, int device);

/* Releases the context's workspace; NULL is ignored.  Waits for the device. */
void gl_ctx_destroy(gl_ctx *ctx);

/* Light curves for a batch of parameter sets (Section 2: coordinate map,
 * projected ellipse, Green's-theorem flux with quadratic limb darkening).
 *
 *  params   device, double[GL_NPARAM][n_sets] (row GL_K first), see above.
 *  n_sets   number of parameter sets, >= 1.
 *  times    device, days.  Shared grid (offsets == NULL): double[n_times],
 *           the same times for every set.  CSR (offsets != NULL): the
 *           concatenated per-set grids, double[n_times].
 *  offsets  device, int64[n_sets + 1] or NULL.  CSR segment of set s is
 *           [offsets[s], offsets[s+1]); offsets[0] must be 0, offsets must be
 *           non-decreasing and offsets[n_sets] == n_times.
 *  n_times  shared-grid length, or total CSR length; >= 1 (shared) / >= 0 (CSR).
 *  n_ss     device int32[n_sets] supersampling factor in [1, 64], or NULL (1).
 *  t_exp    device double[n_sets] exposure time in days (>= 0), or NULL (0).
 *           Output i is the mean of the instantaneous flux at the n_ss
 *           midpoints t_i + ((j + 1/2)/n_ss - 1/2) t_exp, j = 0..n_ss-1.
 *  out      device double: shared grid [n_sets][n_times] (row-major);
 *           CSR indexed like times.  Relative flux in [0, 1].
 *  stream   hipStream_t to enqueue on (NULL: default stream).
 *
 * Domain errors (NaN/Inf parameters, k not in (0,1), f not in [0,1),
 * a/R* <= 1 + k, |b| >= a/R*, P <= 0, q outside [0,1], n_ss outside [1,64],
 * t_exp < 0, a CSR segment out of order or out of range): that set's outputs
 * are NaN (a broken segment is skipped) and the status word is set.
 * Returns GL_OK once the work is enqueued. */
gl_status gl_lightcurve_batch(gl_ctx *ctx, const double *params, int64_t n_sets,
                              const double *times, const int64_t *offsets,
                              int64_t n_times, const int32_t *n_ss,
                              const double *t_exp, double *out, void *stream);

/* General-ellipsoid parameter block rows (SoA, double[GL_E_NPARAM][n_sets]):
 *  GL_E_RA, GL_E_RB, GL_E_RC  semi-axes a, b, c (stellar radii) along the
 *            body axes x', y', z', each in (0, 1)
 *  GL_E_ZETA, GL_E_ETA, GL_E_XI  orientation, rad: R = Rx(zeta) Ry(eta) Rz(xi)
 *            (Section 2, eq. coord-map)
 *  GL_E_B, GL_E_ARS, GL_E_P, GL_E_T0, GL_E_Q1, GL_E_Q2  as GL_B ... GL_Q2
 *            (a/R* > 1 + max(a, b, c))
 *  GL_E_LOCKED  0: the body keeps its orientation (eq. coord-map); 1: tidally
 *            locked, body coordinates R Rx(-alpha) Ry(beta) (x - x_c)
 *            (Appendix B), so the shadow turns with the orbital phase.
 * The oblate block is the case b = c = k, a = k(1 - f), zeta = 0,
 * eta = pi/2 - theta, xi = phi, locked = 0. */
enum { GL_E_RA, GL_E_RB, GL_E_RC, GL_E_ZETA, GL_E_ETA, GL_E_XI, GL_E_B, GL_E_ARS, GL_E_P, GL_E_T0,
       GL_E_Q1, GL_E_Q2, GL_E_LOCKED, GL_E_NPARAM };

/* Light curves of triaxial planets (Section 2 for any a, b, c and orientation:
 * the projected ellipse of eqs. dx, dy1, dy2; Appendix B for tidally-locked
 * planets: eqs. dx-locked, dy1-locked, dy2-locked evaluated at each
 * sub-sample's orbital phase).  Arguments, layout, window, supersampling,
 * status word and errors as gl_lightcurve_batch, with params
 * double[GL_E_NPARAM][n_sets]; a set's domain error (a semi-axis outside
 * (0, 1), a/R* <= 1 + max(a, b, c), locked not 0 or 1, ...) gives NaN
 * outputs.  Free rotators run the exact path's work lists; locked sets are
 * evaluated by its fused per-chunk kernel.  Returns GL_OK once enqueued. */
gl_status gl_lightcurve_batch_ellipsoid(gl_ctx *ctx, const double *params, int64_t n_sets,
                                        const double *times, const int64_t *offsets,
                                        int64_t n_times, const int32_t *n_ss,
                                        const double *t_exp, double *out, void *stream);

/* ---------------------------------------------------------------- MCMC glue
 * Walker block rows (SoA, double[GL_W_NPARAM][n]): the fitting parameters of
 * Section 3 (Table of priors):
 *  GL_W_R    mean radius ratio r, the geometric mean of the three semi-axes
 *            (r^3 = k^3 (1 - f) with equatorial radius k)
 *  GL_W_MU, GL_W_NU  the reparameterised flattening and orientation of
 *            Appendix A: mu = (f - 1)^2 + f (f - 2) cos(2 eta) in [-1, 1],
 *            f = f_min + (1 - f_min) nu with f_min = 1 - sqrt((mu + 1) / 2),
 *            nu in [0, 1)
 *  GL_W_XI   orientation xi, rad (the oblate block's phi)
 *  GL_W_B ... GL_W_Q2  as GL_B ... GL_Q2.
 * The map to the oblate block takes eta in [0, pi/2] (mu fixes cos 2 eta
 * only; the light curve does not see the sign of eta) and theta = pi/2 - eta. */
enum { GL_W_R, GL_W_MU, GL_W_NU, GL_W_XI, GL_W_B, GL_W_ARS, GL_W_P, GL_W_T0, GL_W_Q1, GL_W_Q2,
       GL_W_NPARAM };

/* Inverse-transform draws from the (mu, nu) prior of Appendix A, whose density
 * (eq. mu-nu-joint-density) makes f uniform on [0, 1] and eta cosine-
 * distributed on [0, pi/2]: nu = u^2 / (u^2 - 2u + 2) inverts the marginal CDF
 * of nu, mu inverts the conditional CDF F(mu | nu) at w.
 *  uw     device double[2][n]: row 0 the uniforms u in [0, 1), row 1 the
 *         uniforms w in [0, 1] (the caller draws them).
 *  mu_nu  device double[2][n]: row 0 mu, row 1 nu; NaN for a pair outside
 *         the ranges.
 * Returns GL_ERR_NULL / GL_ERR_SIZE (n < 1), GL_ERR_DEVICE on a failed launch,
 * else GL_OK once enqueued on stream. */
gl_status gl_prior_mu_nu(const double *uw, int64_t n, double *mu_nu, void *stream);

/* Walker block (device double[GL_W_NPARAM][n]) to the oblate parameter block
 * (device double[GL_NPARAM][n]): k = r / cbrt(1 - f), f and eta from (mu, nu)
 * as above, theta = pi/2 - eta, phi = xi, the other rows copied.  Values that
 * leave the oblate block's domain (mu < -1, f >= 1, k >= 1, ...) are caught by
 * the light-curve call as domain errors.  Returns as gl_prior_mu_nu. */
gl_status gl_walkers_to_params(const double *walkers, int64_t n, double *params, void *stream);

/* Per-walker white-noise likelihood of model light curves (Section 3's fit
 * without its correlated-noise terms):
 *   chi2[s] = sum_i ((data_i - model_s,i) / sigma_i)^2,
 *   loglike[s] = -chi2[s] / 2 - sum_i log(sigma_i) - (N_s / 2) log(2 pi).
 *  model    device double: shared grid [n_sets][n_times]; CSR indexed by
 *           offsets (walker s owns [offsets[s], offsets[s+1])).
 *  data, sigma  device double[n_times], indexed like one walker's grid
 *           (shared) or like model (CSR); sigma > 0.
 *  chi2, loglike  device double[n_sets]; either may be NULL, not both.
 * The sums run in a fixed order (bitwise reproducible).  A walker whose model
 * holds a NaN, or whose CSR segment is out of range, gets NaN.  Returns
 * GL_ERR_NULL / GL_ERR_SIZE, GL_ERR_DEVICE on a failed launch, else GL_OK. */
gl_status gl_loglike_of_model(const double *model, int64_t n_sets, const int64_t *offsets, int64_t n_times,
                              const double *data, const double *sigma, double *chi2, double *loglike,
                              void *stream);

/* One MCMC likelihood evaluation for a batch of walkers: the walker block is
 * converted (gl_walkers_to_params, into the context's workspace), the light
 * curves are computed by the exact path into `model` (gl_lightcurve_batch's
 * grid, supersampling and layout), and the per-walker chi^2 / log-likelihood
 * against data / sigma follow (gl_loglike_of_model) -- all captured in one
 * graph with the batch.  Walkers outside the domain give NaN light curves
 * and NaN likelihoods, and set the status word (gl_ctx_sync_status).
 * Returns GL_OK once enqueued, or the errors of gl_lightcurve_batch. */
gl_status gl_loglike_batch(gl_ctx *ctx, const double *walkers, int64_t n_walkers, const double *times,
                           const int64_t *offsets, int64_t n_times, const int32_t *n_ss, const double *t_exp,
                           const double *data, const double *sigma, double *model, double *chi2,
                           double *loglike, void *stream);

/* Allocation-free variant of gl_lightcurve_batch, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, layout and results (up
 * to rounding) as gl_lightcurve_batch, without a context: the workspace and
 * work lists live in one device array of 73.6 MiB inside the library, which
 * every GPU the library runs on holds until the process ends.  The call
 * allocates nothing, launches directly on `stream` (never a graph of its
 * own), and works on the current HIP device; its first call on a device
 * looks up that device's copy of the array.
 *  Limits: n_sets <= 16384 and at most 2^18 chunks of 64 outputs (shared
 *  grid: n_sets * ceil(n_times / 64); CSR: n_times / 64 + n_sets), else
 *  GL_ERR_SIZE with nothing enqueued.  Work lists hold 2^19 in-window
 *  sub-samples; chunks beyond them are evaluated by the fused kernel.
 *  Every call on one device shares its array and clears what must start at
 *  zero: calls that overlap on one device (other streams, other threads)
 *  race.  Domain errors give NaN outputs as in gl_lightcurve_batch; there is
 *  no status word to read back.
 * Returns GL_ERR_NULL / GL_ERR_SIZE as gl_lightcurve_batch does, GL_ERR_DEVICE
 * when the array cannot be found or a launch fails, else GL_OK once the work
 * is enqueued. */
gl_status gl_lightcurve_batch_noalloc(const double *params, int64_t n_sets, const double *times,
                                      const int64_t *offsets, int64_t n_times, const int32_t *n_ss,
                                      const double *t_exp, double *out, void *stream);

/* The paper's own integrator (Section 2, "Ellipsoid Transit Model": no
 * crossing points are solved for; the ellipse boundary is sampled at n_nodes
 * equally spaced theta, every point outside the stellar disk is moved
 * radially onto the limb, lambda = atan2(y_e, x_e), with the line integral
 * reparametrised by dlambda/dtheta, and the three Green's integrands
 * f_flat, f_lin, f_quad are summed by Simpson's rule), in single precision,
 * for comparison with the exact path.  Same batch arguments, layout, window,
 * supersampling and domain errors as gl_lightcurve_batch; n_nodes even in
 * [4, 2^20].  On the moved part of the curve only the tangential part of the
 * boundary's velocity remains, so f_quad jumps at every crossing and the rule
 * converges as 1/n_nodes on partially overlapping samples (about 2e-5 at
 * 1024 nodes on walker draws, 2e-6 at 8192); samples whose ellipse lies
 * inside the disk are at single-precision noise (~1e-7).  Asynchronous;
 * launches directly (no graph). */
gl_status gl_lightcurve_batch_snap(gl_ctx *ctx, int n_nodes, const double *params, int64_t n_sets,
                                   const double *times, const int64_t *offsets, int64_t n_times,
                                   const int32_t *n_ss, const double *t_exp, double *out, void *stream);

/* Waits for the context's device, then returns GL_ERR_DOMAIN if any batch
 * since the last call met a domain error (and clears the flag), else GL_OK. */
gl_status gl_ctx_sync_status(gl_ctx *ctx);

/* Message of the last host-side error on this context ("" if none).  The
 * string is owned by the context and valid until its next call. */
const char *gl_ctx_last_error(const gl_ctx *ctx);

/* Launch-plan autotuner: times the candidate persistent-grid sizes of the
 * work-list kernels on a representative batch (same arguments as
 * gl_lightcurve_batch; `out` is overwritten), one kernel group at a time
 * (hard-sample kernel {4, 8, 16, 24, 32, 48, 64} waves per CU, trapezoid
 * kernel {4, 8, 16, 24, 32, 48, 64}, classification {8, 16, 24, 32, 48, 64},
 * arc-rule levels {8, 12, 16, 20, 32, 48, 64}; more waves than fit at once queue behind
 * the resident ones, which balances uneven per-wave work; coordinate descent
 * in two sweeps, each candidate timed as the median of seven batches after a
 * warm-up, run the way the batch call runs: as a graph where `stream` allows)
 * and keeps the fastest in the context's plan.  Synchronises `stream`.
 * Quadrature orders are not a plan setting: every sample picks its own
 * (self-checking rules). */
gl_status gl_autotune(gl_ctx *ctx, const double *params, int64_t n_sets,
                      const double *times, const int64_t *offsets, int64_t n_times,
                      const int32_t *n_ss, const double *t_exp, double *out,
                      void *stream);

/* gl_autotune on a batch of general ellipsoids (the arguments of
 * gl_lightcurve_batch_ellipsoid): the same four knobs, timed on the graph of
 * that batch (its tidally-locked sets run in the fused kernel beside the
 * hard-sample chain, which moves the best grid sizes). */
gl_status gl_autotune_ellipsoid(gl_ctx *ctx, const double *params, int64_t n_sets,
                                const double *times, const int64_t *offsets, int64_t n_times,
                                const int32_t *n_ss, const double *t_exp, double *out,
                                void *stream);

/* Current plan: persistent wavefronts per compute unit of the hard-sample
 * kernel. */
gl_status gl_ctx_get_plan(const gl_ctx *ctx, int *waves_per_cu);

/* Sets that part of the plan; waves_per_cu in [1, 64] (default 16). */
gl_status gl_ctx_set_plan(gl_ctx *ctx, int waves_per_cu);

/* The whole plan: persistent wavefronts per compute unit of the
 * classification (default 24), the hard-sample kernel (default 16, the value
 * of gl_ctx_get_plan), the trapezoid kernel (default 16) and the arc-rule
 * levels (default 20).  Any pointer may be NULL. */
gl_status gl_ctx_get_stage_plan(const gl_ctx *ctx, int *classify, int *hard, int *trap, int *gk);

/* Sets the whole plan; each value in [1, 64], else GL_ERR_SIZE. */
gl_status gl_ctx_set_stage_plan(gl_ctx *ctx, int classify, int hard, int trap, int gk);

/* Work-list capacities of the exact path, in entries: sub-sample flux slots
 * (and trapezoid entries) <= 2^27 - 1, hard samples and ellipse arcs
 * <= 2^30 - 1.  Explicit capacities hold for every batch (one pass each);
 * all three 0 selects sizing from demand (see gl_ctx_get_overflow), starting
 * again from the default (16 Mi slots, a quarter of that of hard samples,
 * twice that of arcs, about 1.5 GB of device memory, less for small
 * batches).  A chunk of 64 outputs whose samples do not fit is evaluated by
 * the fused per-lane kernel instead, with the same results up to rounding;
 * an ellipse arc that does not fit is integrated where it is found.  Waits
 * for the device and frees the current lists (reallocated by the next batch). */
gl_status gl_ctx_set_capacity(gl_ctx *ctx, int64_t sub_samples, int64_t hard_samples,
                              int64_t arcs);

/* Work lists sized from demand.  Without explicit capacities, every batch
 * records in pinned host memory how many entries each work list was asked
 * for, and the next batch on the context sizes its lists from that record
 * (growing them, and waiting for the device once when it does), and runs as
 * up to 8 passes over equal ranges of its parameter sets when its in-window
 * sub-samples exceed about 6.7e7 (2^26), or its lists a third of the device
 * memory.  Results do not depend on the number of passes or the list sizes:
 * every sub-sample and output is computed on its own.  A batch that outgrows
 * the lists planned for it is still exact (the overflowing chunks take the
 * fused kernel), and the next one is planned for it.
 *
 * gl_ctx_get_overflow waits for the device and writes into *fused_chunks the
 * number of 64-output chunks of the latest batch that did not fit its work
 * lists (0 when the lists held everything), and into *passes (may be NULL)
 * the number of passes it ran. */
gl_status gl_ctx_get_overflow(gl_ctx *ctx, int64_t *fused_chunks, int *passes);

/* When on != 0, later batches replay a captured HIP graph of the whole
 * pipeline if their arguments equal the previous batch's (default on). */
gl_status gl_ctx_set_graph(gl_ctx *ctx, int on);

/* Stages of one batch (timed separately):
 *  0 set-up (parameter preparation, chunk scan), 1 window test (fills the
 *  outputs that cannot overlap the star), 2 classification, 3 whole-ellipse
 *  trapezoid, 4 hard samples (intersection quartic, break points, limb arcs),
 *  5 ellipse arcs (Gauss-Kronrod levels 0 and 1), 6 rare paths (nested
 *  trapezoid for whole ellipses near the limb, samples integrated in place,
 *  arcs from level 2 on), 7 combination of each hard sample's sums and
 *  supersample averages, 8 fused kernel for chunks beyond the work-list
 *  capacities.  Stages 3 and 8 (on a second stream of the context, joined
 *  before the averages) run beside stages 4 to 6 and the combination (on the
 *  caller's stream): all need only the classification.  Stage 3 is timed
 *  from the second stream's start, so stage times overlap and need not add
 *  up to the batch time.  In a surrogate batch the second stream evaluates
 *  the network instead, and stages 3 and 8 follow the combination on the
 *  caller's stream. */
#define GL_NSTAGES 9

/* Instrumentation: with n_slots > 0, the next n_slots batches are launched
 * directly (no graph), with the same two-stream overlap a graph has, and
 * record a HIP event before the first stage and after every stage of every
 * pass, on the stream each stage runs on; each timed batch waits for its
 * stream and adds its stage times before returning.  n_slots = 0 turns it
 * off (and clears the sums). */
gl_status gl_ctx_set_timing(gl_ctx *ctx, int n_slots);

/* Returns the summed times (ms) from the start of stage 1 (compute) and of
 * stage 0 (pipeline) to the end of stage 7 (the last on the caller's stream,
 * after the join) over the timed batches, and how many batches were timed;
 * clears the sums.  Any output pointer may be NULL. */
gl_status gl_ctx_get_timing(gl_ctx *ctx, double *compute_ms, double *pipeline_ms, int *n);

/* Like gl_ctx_get_timing, per stage: stage_ms[GL_NSTAGES] (host memory)
 * receives the summed time of each stage over the timed batches (and the sums
 * are cleared). */
gl_status gl_ctx_get_stage_timing(gl_ctx *ctx, double *stage_ms, int *n);

/* Work census: runs the batch once (same arguments and results as
 * gl_lightcurve_batch) with counting variants of the kernels, waits, and
 * writes counts[11] (host memory): in-window sub-samples, samples with the
 * whole ellipse on the star, intersecting samples, in-window samples off the
 * star, nodes of the rigorous-order periodic trapezoid, 21-node
 * Gauss-Kronrod pieces, Newton steps of the intersection solver, limb arcs,
 * nodes of the nested periodic trapezoid, ellipse arcs listed for the
 * Gauss-Kronrod stage, ellipse arcs accepted unconverged (see
 * gl_ctx_get_unconverged). */
gl_status gl_census(gl_ctx *ctx, const double *params, int64_t n_sets, const double *times,
                    const int64_t *offsets, int64_t n_times, const int32_t *n_ss,
                    const double *t_exp, double *out, void *stream, int64_t *counts);

/* Algorithmic FP64 operations per census item (add/sub/mul/div/sqrt/
 * transcendental = 1, fused multiply-add = 2), counted from the kernel source:
 * per_item[11] (host memory) lines up with the census counts. */
gl_status gl_flop_model(int64_t *per_item);

/* Accuracy report of the arc rule (Section 2: the Green's-theorem line
 * integrals along the ellipse arcs on the star).  Each ellipse arc is
 * integrated by a clustered Gauss-Kronrod 10/21 rule, split into 1, 2, 4, 8
 * and 16 pieces until the Gauss-Kronrod difference is below its tolerance
 * (1e-6; the difference estimates the error of the 10-point Gauss sum, the
 * 21-point Kronrod sum that is kept is far more accurate); an arc still above
 * it at 16 pieces is accepted there and counted.  Waits for the context's device, writes the
 * number of such arcs over all batches since the last call into *n_arcs
 * (host memory) and clears the count.  A nonzero count does not make an
 * output invalid: it says that the error bound of those arcs was not shown. */
gl_status gl_ctx_get_unconverged(gl_ctx *ctx, int64_t *n_arcs);

/* ---------------------------------------------------------------------------
 * Residual surrogate network: x[16] -> [Linear -> GELU] x 4 (width 256) -> Linear.
 * BF16 matrix-core GEMMs with FP32 accumulation; FP32 master weights, biases,
 * output layer, loss and Adam.  Packed FP32 parameter layout:
 * W0[16][256] b0[256] W1[256][256] b1[256] W2 b2 W3 b3 w4[256] b4[1]
 * (W_l[in][out]), gl_mlp_num_params() values.  GELU is the tanh form
 * z/2 (1 + tanh(sqrt(2/pi)(z + 0.044715 z^3))); the loss is the mean squared
 * error.  A network is used by one host thread at a time.
 * ------------------------------------------------------------------------- */
#define GL_MLP_DIN 16
#define GL_MLP_WIDTH 256
typedef struct gl_mlp gl_mlp;

int gl_mlp_num_params(void);

/* Allocates a network (zero weights) for batches of up to max_batch rows
 * (a multiple of 64 in [64, 4194304]) on HIP device `device`. */
gl_status gl_mlp_create(gl_mlp **mlp, int device, int max_batch);
void gl_mlp_destroy(gl_mlp *mlp);
const char *gl_mlp_last_error(const gl_mlp *mlp);

/* Host FP32 packed parameters in/out (n must equal gl_mlp_num_params()).
 * Setting weights resets the Adam state and step count.  Synchronous. */
gl_status gl_mlp_set_weights(gl_mlp *mlp, const float *host_params, int64_t n);
gl_status gl_mlp_get_weights(const gl_mlp *mlp, float *host_params, int64_t n);

/* y[n] = network(x[n][16]); x, y device FP32; enqueued on stream. */
gl_status gl_mlp_forward(gl_mlp *mlp, const float *x, int64_t n, float *y, void *stream);

/* Gradients of the mean squared error against targets t[n] (device) for one
 * batch (n <= max_batch) into host_grads (packed layout), and the loss into
 * *host_loss (may be NULL).  Synchronises stream; weights unchanged. */
gl_status gl_mlp_grads(gl_mlp *mlp, const float *x, const float *t, int64_t n, float *host_grads,
                       float *host_loss, void *stream);

/* One Adam step (b1 0.9, b2 0.999, eps 1e-8, learning rate lr) on a batch;
 * loss_dev (device float, may be NULL) receives the batch's sum of squared
 * residuals.  Enqueued on stream. */
gl_status gl_mlp_train_step(gl_mlp *mlp, const float *x, const float *t, int64_t n, float lr,
                            float *loss_dev, void *stream);

/* ---------------------------------------------------------------------------
 * Learned surrogate with exact fallback.  The network predicts the
 * oblate-minus-equal-area-sphere residual r = F_oblate - F_sphere(k sqrt(q)),
 * scaled by k^2 (1 - q); the sphere of the same projected area is the paper's
 * comparison body for oblate transits (Section 2.1).  Inputs are the nine
 * quantities (k, f, theta, phi, b, a/R*, u1, u2, phase), encoded through the
 * symmetries of the occultation (it depends on them only through k, q, the
 * centre distance, the angle between the projected spin axis and the radial
 * direction mod pi, u1 and u2) into GL_MLP_DIN features.
 * ------------------------------------------------------------------------- */

/* Training / calibration samples, one per parameter set: params device SoA
 * double[GL_NPARAM][n], times device double[n].  Writes (device) feat
 * float[n][GL_MLP_DIN], target float[n] (scaled residual, 0 off the star),
 * and, when non-NULL, f_obl / f_sph double[n] (exact fluxes from the same
 * kernels as gl_lightcurve_batch), scale double[n] and bin int32[n] (-1 off
 * the star). */
gl_status gl_surrogate_samples(gl_ctx *ctx, const double *params, const double *times, int64_t n,
                               float *feat, float *target, double *f_obl, double *f_sph,
                               double *scale, int32_t *bin, void *stream);

/* Number of calibration bins of the error-bound table. */
int gl_surrogate_num_bins(void);

/* A trained surrogate: the network, its optimizer state, the calibrated
 * per-bin error bound and predictor choice, and the configuration it was
 * trained with.  Owned by the caller; used by one host thread at a time. */
typedef struct gl_surrogate gl_surrogate;

typedef struct {
    int64_t n_train;      /* training samples drawn (default 2e7); those on the star are used */
    int64_t n_calib;      /* calibration samples (default 1e6) */
    int epochs;           /* passes over the training samples (default 4) */
    int batch;            /* rows per Adam step, a multiple of 64 (default 8192) */
    float lr, lr_final;   /* learning rate, log-linear from lr to lr_final (2e-3 -> 1e-4) */
    double safety;        /* factor on the calibrated bound in the gate (default 4) */
    int min_bin_count;    /* calibration samples a bin needs before the gate may accept there (200) */
    double window;        /* sample times uniform in +-window * T14 (default 0.6) */
    uint64_t seed;        /* training draws use seed, calibration draws seed + 1, initial weights seed + 2 */
    int zero_predictor;   /* 1: no network, the residual is taken as 0 (the sphere alone; ablation) */
} gl_surrogate_config;

void gl_surrogate_config_default(gl_surrogate_config *cfg);

/* Trains a surrogate on the context's device (synchronises `stream`):
 *  1. draws n_train parameter sets from the walker priors (k ~ U[0.05, 0.12],
 *     f ~ U[0, 0.9], theta ~ U[0, pi], phi ~ U[0, 2 pi), b ~ U[0, 0.9],
 *     a/R* ~ U[100, 300], q1, q2 ~ U[0, 1], P = 500 d, t0 = 0) and one time
 *     each uniform in +-window * T14, with a counter-based generator from the
 *     seed; their targets come from the exact kernels (gl_surrogate_samples);
 *  2. trains the network on the samples on the star (Adam, MSE, `epochs`
 *     passes in a fresh permutation each);
 *  3. calibrates on n_calib fresh draws: per bin, the largest scaled error of
 *     the network and of the zero predictor; each bin keeps the smaller (the
 *     sphere alone where it is smaller), and bins with fewer than
 *     min_bin_count samples never accept.
 * loss_history (host float[epochs], may be NULL) receives each epoch's mean
 * squared error.  *s receives the surrogate (NULL on failure).  Errors:
 * GL_ERR_NULL, GL_ERR_SIZE (configuration out of range, or fewer samples on
 * the star than one batch), GL_ERR_NOMEM, GL_ERR_DEVICE. */
gl_status gl_surrogate_train(gl_ctx *ctx, const gl_surrogate_config *cfg, gl_surrogate **s,
                             float *loss_history, void *stream);

void gl_surrogate_destroy(gl_surrogate *s);

/* Host copies of a surrogate's packed FP32 parameters (params may be NULL;
 * n_params = gl_mlp_num_params()), calibrated bound table, per-bin predictor
 * choice (1 = sphere alone) and calibration counts (each may be NULL;
 * n_bins = gl_surrogate_num_bins()).  Waits for the device. */
gl_status gl_surrogate_get(const gl_surrogate *s, float *params, int64_t n_params, float *table,
                           uint8_t *zero_bins, int32_t *counts, int n_bins);

/* The configuration a surrogate was trained (or loaded) with. */
gl_status gl_surrogate_config_of(const gl_surrogate *s, gl_surrogate_config *cfg);

/* A surrogate on disk: header (magic, version 2, network widths, counts),
 * the configuration, the packed FP32 parameters, the Adam moments and step,
 * the bound table, the predictor choice and the calibration counts
 * (little-endian), and a 64-bit FNV-1a hash of all of it.  Load creates the
 * surrogate on the context's device.  Errors: GL_ERR_NULL; GL_ERR_SIZE when
 * the file was written for other network widths or bin counts; GL_ERR_STATE
 * when the file cannot be opened, written or read, or its magic, version,
 * length or hash is wrong. */
gl_status gl_surrogate_save(const gl_surrogate *s, const char *path);
gl_status gl_surrogate_load(gl_ctx *ctx, gl_surrogate **s, const char *path);

/* The same file from and into host arrays, with no device call (the file
 * functions also run without a GPU): cfg, params, m, v float[n_params]
 * (n_params = gl_mlp_num_params()), step, table float[n_bins], zero_bins
 * uint8[n_bins], counts int32[n_bins] (n_bins = gl_surrogate_num_bins()).
 * Errors as for gl_surrogate_save / gl_surrogate_load; on any error the
 * outputs of the read are untouched. */
gl_status gl_surrogate_file_write(const char *path, const gl_surrogate_config *cfg, const float *params,
                                  const float *m, const float *v, int64_t step, int64_t n_params,
                                  const float *table, const uint8_t *zero_bins, const int32_t *counts,
                                  int n_bins);
gl_status gl_surrogate_file_read(const char *path, gl_surrogate_config *cfg, float *params, float *m,
                                 float *v, int64_t *step, int64_t n_params, float *table,
                                 uint8_t *zero_bins, int32_t *counts, int n_bins);

/* Light curves through the surrogate: same batch arguments and output as
 * gl_lightcurve_batch.  Every in-window sub-sample whose ellipse reaches the
 * disk goes to the gate first: it is accepted when
 * safety * table[bin] * scale <= tol (its bin's calibrated scaled error, in
 * flux units through its own scale k^2 (1 - q), with the safety factor of the
 * configuration); then its flux is that of the sphere of equal projected area
 * (computed exactly, by the same kernels as the oblate flux) plus
 * scale * network(features), or the sphere alone where the bin takes it.
 * Every other sub-sample is computed exactly (the exact path's work lists).
 * Outputs are box-averaged in order.  Asynchronous unless a count is
 * requested: *n_sub_out and *n_fallback_out (host, may be NULL) then receive,
 * after waiting for `stream`, the in-window sub-samples and those of them
 * whose ellipse reaches the disk but that the gate rejected. */
gl_status gl_lightcurve_batch_surrogate(gl_ctx *ctx, const gl_surrogate *s, double tol,
                                        const double *params, int64_t n_sets, const double *times,
                                        const int64_t *offsets, int64_t n_times, const int32_t *n_ss,
                                        const double *t_exp, double *out, void *stream,
                                        int64_t *n_sub_out, int64_t *n_fallback_out);

/* Library version, e.g. "0.1.0". */
const char *gl_version(void);

#ifdef __cplusplus
}
#endif
#endif
