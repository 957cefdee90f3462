"""Seeded synthetic workloads for the oblate transit light curve.

This module only draws inputs: parameter blocks, time grids, CSR offsets and
supersampling factors.  It holds none of the flux arithmetic, so that both the
GPU path and the CPU oracle can be fed from it without sharing any of the
method.

Parameter block layout (SoA, ``float64[10][n_sets]``):
    k, f, theta, phi, b, a/R*, P (days), t0 (days), q1, q2
``k`` is the equatorial radius ratio, ``theta`` the angle between spin axis
and line of sight, ``phi`` the sky rotation of the projected spin axis, and
``q1, q2`` the Kipping (2013) limb-darkening parameters (the paper fits these,
Section 3).

The workloads stand in for the paper's data (K2 long cadence at ~30 min,
K2 short cadence at 1 min, JWST at 1-2 min; Section 3 and Section 5.3), which
are not used here: every value is drawn from a seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NPARAM = 10
K, F, THETA, PHI, B, ARS, P, T0, Q1, Q2 = range(NPARAM)
PARAM_NAMES = ("k", "f", "theta", "phi", "b", "ars", "P", "t0", "q1", "q2")

PERIOD_DAYS = 500.0
MINUTE = 1.0 / 1440.0


@dataclass
class Workload:
    """A batch in the library's layout.

    ``offsets is None``: shared grid, ``out`` has shape ``[n_sets, n_times]``.
    Otherwise CSR: set ``s`` owns ``times[offsets[s]:offsets[s+1]]``.
    """
    name: str
    params: np.ndarray                 # float64 [10, n_sets] (general ellipsoids: [13, n_sets])
    times: np.ndarray                  # float64 [n_times] or [offsets[-1]]
    offsets: np.ndarray | None         # int64 [n_sets + 1] or None
    n_ss: np.ndarray                   # int32 [n_sets]
    t_exp: np.ndarray                  # float64 [n_sets]
    meta: dict = field(default_factory=dict)

    @property
    def n_sets(self) -> int:
        return self.params.shape[1]

    @property
    def n_out(self) -> int:
        if self.offsets is None:
            return self.n_sets * self.times.shape[0]
        return int(self.offsets[-1])

    @property
    def n_sub(self) -> int:
        """Number of sub-samples (outputs times their supersampling factor)."""
        if self.offsets is None:
            return int(self.times.shape[0] * np.sum(self.n_ss, dtype=np.int64))
        seg = np.diff(self.offsets)
        return int(np.sum(seg * self.n_ss.astype(np.int64)))


def q_from_u(u1: float, u2: float) -> tuple[float, float]:
    """Kipping's (q1, q2) for given quadratic coefficients (used only to state
    a workload quoted in u1, u2 in the library's q1, q2 layout)."""
    s = u1 + u2
    return s * s, u1 / (2.0 * s)


def full_duration(k, b, ars, period):
    """First-to-fourth-contact time of a sphere of radius k (days): the
    textbook circular-orbit duration, used here only to size time grids."""
    k, b, ars = np.asarray(k), np.asarray(b), np.asarray(ars)
    sin_i = np.sqrt(1.0 - (b / ars) ** 2)
    arg = np.sqrt(np.maximum((1.0 + k) ** 2 - b ** 2, 0.0)) / (ars * sin_i)
    return period / math.pi * np.arcsin(np.minimum(arg, 1.0))


def draw_params(rng: np.random.Generator, n: int, f_max: float = 0.9) -> np.ndarray:
    """MCMC-walker priors: k~U[0.05,0.12], f~U[0,f_max], theta~U[0,pi],
    phi~U[0,2pi), b~U[0,0.9], a/R*~U[100,300], q1,q2~U[0,1]; drawn column by
    column in that order.  P = 500 d, t0 = 0."""
    p = np.empty((NPARAM, n))
    p[K] = rng.uniform(0.05, 0.12, n)
    p[F] = rng.uniform(0.0, f_max, n)
    p[THETA] = rng.uniform(0.0, math.pi, n)
    p[PHI] = rng.uniform(0.0, 2.0 * math.pi, n)
    p[B] = rng.uniform(0.0, 0.9, n)
    p[ARS] = rng.uniform(100.0, 300.0, n)
    p[Q1] = rng.uniform(0.0, 1.0, n)
    p[Q2] = rng.uniform(0.0, 1.0, n)
    p[P] = PERIOD_DAYS
    p[T0] = 0.0
    return p


def single_transit(n_times: int = 1000) -> Workload:
    """One parameter set: k=0.1, f=0.3, theta=60 deg, phi=30 deg, b=0.3,
    a/R*=200, P=500 d, u1=0.4, u2=0.25; times uniform over +-1 transit
    duration around mid-transit; no supersampling."""
    q1, q2 = q_from_u(0.4, 0.25)
    p = np.array([[0.1], [0.3], [math.pi / 3], [math.pi / 6], [0.3], [200.0],
                  [PERIOD_DAYS], [0.0], [q1], [q2]])
    t14 = float(full_duration(0.1, 0.3, 200.0, PERIOD_DAYS))
    times = np.linspace(-t14, t14, n_times)
    return Workload("single_transit", p, times, None, np.ones(1, np.int32),
                    np.zeros(1), {"t14": t14})


def walker_batch(n_sets: int = 4096, n_times: int = 3000, n_ss: int = 15,
                 seed: int = 2) -> Workload:
    """MCMC-walker batch: shared grid at 29.4-min cadence centred on the
    transit, each point box-averaged over n_ss midpoint sub-samples spanning
    the cadence (K2-long-cadence-shaped)."""
    rng = np.random.default_rng(seed)
    p = draw_params(rng, n_sets)
    dt = 29.4 * MINUTE
    times = (np.arange(n_times) - (n_times - 1) / 2.0) * dt
    return Workload("walker_batch", p, times, None,
                    np.full(n_sets, n_ss, np.int32), np.full(n_sets, dt),
                    {"cadence_days": dt, "seed": seed})


def high_cadence(n_sets: int = 512, n_times: int = 65536, seed: int = 3) -> Workload:
    """High-cadence deep-transit batch: f~U[0,0.2], 60-s cadence around the
    transit, no supersampling (JWST/K2-short-cadence-shaped)."""
    rng = np.random.default_rng(seed)
    p = draw_params(rng, n_sets, f_max=0.2)
    dt = 60.0 / 86400.0
    times = (np.arange(n_times) - (n_times - 1) / 2.0) * dt
    return Workload("high_cadence", p, times, None, np.ones(n_sets, np.int32),
                    np.zeros(n_sets), {"cadence_days": dt, "seed": seed})


def uneven_batch(n_sets: int = 16384, seed: int = 4, n_min: int = 200,
                 n_max: int = 20000) -> Workload:
    """Uneven batch: each walker has its own grid linspace(-T14, T14, n_w)
    with n_w log-uniform in [n_min, n_max] and supersampling factor in
    {1, 5, 15}; exposure = grid spacing; CSR layout."""
    rng = np.random.default_rng(seed)
    p = draw_params(rng, n_sets)
    n_w = np.floor(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_sets))).astype(np.int64)
    n_w = np.maximum(n_w, 2)
    ss = rng.choice(np.array([1, 5, 15], np.int32), n_sets)
    t14 = full_duration(p[K], p[B], p[ARS], p[P])
    offsets = np.zeros(n_sets + 1, np.int64)
    offsets[1:] = np.cumsum(n_w)
    times = np.empty(int(offsets[-1]))
    t_exp = np.empty(n_sets)
    for s in range(n_sets):
        g = np.linspace(-t14[s], t14[s], int(n_w[s]))
        times[offsets[s]:offsets[s + 1]] = g
        t_exp[s] = g[1] - g[0]
    return Workload("uneven_batch", p, times, offsets, ss.astype(np.int32), t_exp,
                    {"seed": seed})


def surrogate_samples(n: int, seed: int, window: float = 0.6):
    """Training / calibration samples for the residual surrogate: walker
    priors, one time per sample drawn uniformly in +-window*T14."""
    rng = np.random.default_rng(seed)
    p = draw_params(rng, n)
    t14 = full_duration(p[K], p[B], p[ARS], p[P])
    t = rng.uniform(-window, window, n) * t14
    return p, t


# ---------------------------------------------------------------- general ellipsoids
# Parameter block of the general model (SoA, ``float64[13][n_sets]``): semi-axes
# a, b, c along the body axes x', y', z'; orientation zeta, eta, xi; b, a/R*,
# P, t0, q1, q2; ``locked`` (1: tidally locked, Appendix B of the paper).
E_NPARAM = 13
(E_RA, E_RB, E_RC, E_ZETA, E_ETA, E_XI, E_B, E_ARS, E_P, E_T0, E_Q1, E_Q2,
 E_LOCKED) = range(E_NPARAM)


def draw_ellipsoids(rng: np.random.Generator, n: int, locked: bool) -> np.ndarray:
    """Triaxial planets.  Free rotators (locked = 0): the walker priors' orbit
    (b~U[0,0.9], a/R*~U[100,300], P = 500 d), each semi-axis U[0.03,0.15],
    angles U[-pi,pi].  Tidally locked (locked = 1): close-in orbits
    (b~U[0,0.8], a/R*~U[2.5,8], P~U[0.7,4] d) and tidal shapes, the axis
    toward the star longest: c~U[0.06,0.15], b = c U[0.7,1], a = b U[0.7,1],
    angles U[-0.3,0.3] about the equilibrium orientation.  q1, q2~U[0,1],
    t0 = 0.  Drawn column by column in that order."""
    p = np.empty((E_NPARAM, n))
    if locked:
        c = rng.uniform(0.06, 0.15, n)
        b = c * rng.uniform(0.7, 1.0, n)
        a = b * rng.uniform(0.7, 1.0, n)
        p[E_RA], p[E_RB], p[E_RC] = a, b, c
        for r in (E_ZETA, E_ETA, E_XI):
            p[r] = rng.uniform(-0.3, 0.3, n)
        p[E_B] = rng.uniform(0.0, 0.8, n)
        p[E_ARS] = rng.uniform(2.5, 8.0, n)
        p[E_P] = rng.uniform(0.7, 4.0, n)
    else:
        for r in (E_RA, E_RB, E_RC):
            p[r] = rng.uniform(0.03, 0.15, n)
        for r in (E_ZETA, E_ETA, E_XI):
            p[r] = rng.uniform(-math.pi, math.pi, n)
        p[E_B] = rng.uniform(0.0, 0.9, n)
        p[E_ARS] = rng.uniform(100.0, 300.0, n)
        p[E_P] = PERIOD_DAYS
    p[E_Q1] = rng.uniform(0.0, 1.0, n)
    p[E_Q2] = rng.uniform(0.0, 1.0, n)
    p[E_T0] = 0.0
    p[E_LOCKED] = 1.0 if locked else 0.0
    return p


def ellipsoid_batch(n_sets: int = 2048, n_w: int = 1500, seed: int = 6,
                    locked_fraction: float = 0.5) -> Workload:
    """Mixed batch of free and tidally-locked triaxial planets (the first
    ``locked_fraction`` of the sets locked), CSR layout: each set samples
    linspace(-T14, T14, n_w) of a sphere of its largest semi-axis, with
    supersampling factor in {1, 5} and exposure = grid spacing."""
    rng = np.random.default_rng(seed)
    n_lock = int(round(locked_fraction * n_sets))
    p = np.concatenate([draw_ellipsoids(rng, n_lock, True),
                        draw_ellipsoids(rng, n_sets - n_lock, False)], axis=1)
    kmax = np.max(p[E_RA:E_RC + 1], axis=0)
    t14 = full_duration(kmax, p[E_B], p[E_ARS], p[E_P])
    offsets = np.arange(n_sets + 1, dtype=np.int64) * n_w
    g = np.linspace(-1.0, 1.0, n_w)
    times = (t14[:, None] * g[None, :]).ravel()
    t_exp = t14 * (g[1] - g[0])
    ss = rng.choice(np.array([1, 5], np.int32), n_sets)
    return Workload("ellipsoid_batch", p, times, offsets, ss, t_exp,
                    {"seed": seed, "locked_sets": n_lock})


# ---------------------------------------------------------------- MCMC walkers
# Walker block (SoA, ``float64[10][n]``): the paper's fitting parameters
# (Section 3, Table of priors): mean radius ratio r (geometric mean of the
# three semi-axes), mu, nu (Appendix A), xi, b, d/R*, P, t0, q1, q2.
W_NPARAM = 10
W_R, W_MU, W_NU, W_XI, W_B, W_ARS, W_P, W_T0, W_Q1, W_Q2 = range(W_NPARAM)

# The simulated JWST/NIRISS transit of Section 5.3: 2-minute cadence, 20 ppm
# white noise, the fitted medians of the K2 fit (Table of fit results: r,
# d/R*, P, b, q1, q2) with injected f = 0.15, eta = 0, xi = 29 deg.
# f = 0.15 and eta = 0 are (mu, nu) = (0.85^2 - 0.15 * 1.85, 0) = (0.445, 0).
JWST_CADENCE = 2.0 * MINUTE
JWST_SIGMA = 20e-6
JWST_TRUTH = {"r": 0.067208, "mu": 0.445, "nu": 0.0, "xi": math.radians(29.0), "b": 0.041605,
              "ars": 231.24, "P": 542.08, "t0": 0.0, "q1": 0.26744, "q2": 0.39688}


def jwst_truth() -> np.ndarray:
    """The injected planet as a walker-block column, float64 [10, 1]."""
    t = JWST_TRUTH
    return np.array([[t["r"]], [t["mu"]], [t["nu"]], [t["xi"]], [t["b"]], [t["ars"]], [t["P"]],
                     [t["t0"]], [t["q1"]], [t["q2"]]])


def jwst_grid(half_span_days: float = 0.7):
    """Times of the simulated visit (+-0.7 d around mid-transit at 2-min
    cadence: the 0.8-d transit plus baseline), the exposure (one cadence)
    and the supersampling factor used for it (3)."""
    n = int(round(2.0 * half_span_days / JWST_CADENCE)) + 1
    times = (np.arange(n) - (n - 1) / 2.0) * JWST_CADENCE
    return times, JWST_CADENCE, 3


def walker_ball(n: int, seed: int = 8):
    """Walkers around the injected planet, a ball as an ensemble sampler is
    started with: r~N(0.067208, 7e-4), xi~U[0, pi/2], b~N(0.0416, 0.1),
    d/R*~N(231.24, 2), P~N(542.08, 2e-4), t0~N(0, 2e-3), q1~N(0.26744, 0.02),
    q2~N(0.39688, 0.03); drawn in that order.  The (mu, nu) rows are left NaN:
    they come from the prior sampler fed with the returned uniforms
    uw [2, n] (u~U[0, 0.6], w~U[0.5, 1]: the corner of the prior with
    f below about 0.5)."""
    rng = np.random.default_rng(seed)
    t = JWST_TRUTH
    walk = np.full((W_NPARAM, n), np.nan)
    walk[W_R] = rng.normal(t["r"], 7e-4, n)
    walk[W_XI] = rng.uniform(0.0, 0.5 * math.pi, n)
    walk[W_B] = rng.normal(t["b"], 0.1, n)
    walk[W_ARS] = rng.normal(t["ars"], 2.0, n)
    walk[W_P] = rng.normal(t["P"], 2e-4, n)
    walk[W_T0] = rng.normal(0.0, 2e-3, n)
    walk[W_Q1] = np.clip(rng.normal(t["q1"], 0.02, n), 0.0, 1.0)
    walk[W_Q2] = np.clip(rng.normal(t["q2"], 0.03, n), 0.0, 1.0)
    uw = np.empty((2, n))
    uw[0] = rng.uniform(0.0, 0.6, n)
    uw[1] = rng.uniform(0.5, 1.0, n)
    return walk, uw


def by_name(name: str, **kw) -> Workload:
    return {"single_transit": single_transit, "walker_batch": walker_batch,
            "high_cadence": high_cadence, "uneven_batch": uneven_batch}[name](**kw)


def adversarial_batch(n_dense: int = 3000) -> Workload:
    """Hard shapes and grazing geometries, CSR layout.

    Parameter sets: large and small k, extreme flattening with the spin axis
    in the sky plane (flat ellipses whose flat side can run along the limb and
    cross it four times), pole-on and f = 0 spheres, and impact parameters up
    to grazing (b near 1 - k, 1, 1 + k/2).  Each set gets a uniform grid over
    +-0.7 T14 plus a dense grid over the last 4% of the ingress side, so that
    contacts and near-tangent configurations are sampled finely.  Exposures
    and supersampling vary across sets.
    """
    rows = []
    for k in (0.02, 0.12, 0.3, 0.5):
        for f, theta in ((0.0, 1.0), (0.3, 0.0), (0.9, 0.5 * math.pi), (0.95, 1.3), (0.5, 2.2)):
            for phi in (0.0, 0.25 * math.pi, 0.5 * math.pi, 2.0):
                for b in (0.0, 1.0 - k, 1.0, 1.0 + 0.5 * k):
                    rows.append((k, f, theta, phi, b))
    n = len(rows)
    p = np.empty((NPARAM, n))
    rng = np.random.default_rng(99)
    for s, (k, f, theta, phi, b) in enumerate(rows):
        p[:, s] = (k, f, theta, phi, b, 20.0 + 30.0 * (s % 5), 50.0, 0.013 * (s % 3),
                   rng.uniform(), rng.uniform())
    t14 = full_duration(p[K], np.minimum(np.abs(p[B]), 1.0 + p[K] - 1e-9), p[ARS], p[P])
    grids = []
    for s in range(n):
        t0, w = p[T0, s], t14[s]
        g1 = np.linspace(t0 - 0.7 * w, t0 + 0.7 * w, n_dense)
        g2 = np.linspace(t0 - 0.52 * w, t0 - 0.44 * w, n_dense // 3)
        grids.append(np.sort(np.concatenate([g1, g2])))
    offsets = np.zeros(n + 1, np.int64)
    offsets[1:] = np.cumsum([len(g) for g in grids])
    n_ss = np.array([(1, 5, 15, 3)[s % 4] for s in range(n)], np.int32)
    t_exp = np.array([(0.0, 2e-3, 1e-2, 5e-4)[s % 4] for s in range(n)])
    return Workload("adversarial", p, np.concatenate(grids), offsets, n_ss, t_exp, {})
