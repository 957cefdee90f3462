"""Plain FP64 reference of the MCMC glue around the light curves.

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg; never by the GPU package.  It shares no code
with the HIP library.

* The (mu, nu) reparameterisation of flattening f and orientation eta and its
  inverse-transform prior sampler (Appendix A, "Model Degeneracies"): two
  independent uniforms (u, w) give nu = u^2 / (u^2 - 2u + 2) by inverting the
  marginal CDF of nu, then mu by inverting the conditional CDF F(mu | nu);
  f = f_min + (1 - f_min) nu with f_min = 1 - sqrt((mu + 1) / 2), and eta from
  mu = (f - 1)^2 + f (f - 2) cos(2 eta), taken in [0, pi/2] (mu fixes cos 2eta
  only; the flux does not see the sign of eta).
* The fitting parameters of Section 3 (Table of priors): mean radius ratio r
  (geometric mean of the three semi-axes, r^3 = R_a R_bc^2 with polar
  R_a = R_bc (1 - f)), mu, nu, xi, b, d/R*, P, t0, q1, q2; mapped to the oblate
  parameter block (k = R_bc, f, theta = pi/2 - eta, phi = xi, ...).
* White-noise log-likelihood of a model light curve against data with
  per-point errors sigma: chi^2 = sum ((d - m) / sigma)^2 and
  log L = -chi^2 / 2 - sum log sigma - (N / 2) log 2 pi, per walker.
"""
from __future__ import annotations

import math

import numpy as np

# rows of the walker block (fitting parameters)
W_R, W_MU, W_NU, W_XI, W_B, W_ARS, W_P, W_T0, W_Q1, W_Q2 = range(10)
W_NPARAM = 10


def nu_of_u(u):
    """Inverse of the marginal CDF F(nu) = (nu - sqrt(nu (2 - nu))) / (nu - 1)."""
    u = np.asarray(u, dtype=np.float64)
    return u * u / (u * u - 2.0 * u + 2.0)


def mu_of_w(w, nu):
    """Inverse of the conditional CDF F(mu | nu) at w (Appendix A)."""
    w = np.asarray(w, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    s = np.sqrt(nu * (2.0 - nu))
    g = (nu - 1.0) ** 2
    return (4.0 * w + 4.0 * (w * w - w) * s + 2.0 * (nu * (nu - 2.0) - 1.0) * w * w - g) / g


def mu_nu_from_uniforms(u, w):
    nu = nu_of_u(u)
    return mu_of_w(w, nu), nu


def f_eta_from_mu_nu(mu, nu):
    """f = f_min + (1 - f_min) nu; eta in [0, pi/2] from eq. mu (0 where f = 0:
    a sphere has no orientation)."""
    mu = np.asarray(mu, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    f_min = 1.0 - np.sqrt((mu + 1.0) / 2.0)
    f = f_min + (1.0 - f_min) * nu
    den = f * (f - 2.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        c2 = np.where(den != 0.0, (mu - (f - 1.0) ** 2) / np.where(den != 0.0, den, 1.0), 1.0)
    eta = 0.5 * np.arccos(np.clip(c2, -1.0, 1.0))
    return f, eta


def mu_of_f_eta(f, eta):
    """Eq. mu: mu(f, eta) = (f - 1)^2 + f (f - 2) cos(2 eta)."""
    return (f - 1.0) ** 2 + f * (f - 2.0) * np.cos(2.0 * eta)


def params_from_walkers(walk):
    """Walker block [W_NPARAM, n] -> oblate parameter block [10, n]
    (k, f, theta, phi, b, a/R*, P, t0, q1, q2)."""
    walk = np.asarray(walk, dtype=np.float64)
    f, eta = f_eta_from_mu_nu(walk[W_MU], walk[W_NU])
    out = np.empty((10, walk.shape[1]))
    out[0] = walk[W_R] / np.cbrt(1.0 - f)   # r^3 = R_bc^3 (1 - f)
    out[1] = f
    out[2] = 0.5 * math.pi - eta
    out[3] = walk[W_XI]
    out[4] = walk[W_B]
    out[5] = walk[W_ARS]
    out[6] = walk[W_P]
    out[7] = walk[W_T0]
    out[8] = walk[W_Q1]
    out[9] = walk[W_Q2]
    return out


def loglike(model, data, sigma, offsets=None):
    """Per-walker (chi^2, log L).  Shared grid (offsets None): model
    [n_sets, n_times] against data, sigma [n_times].  CSR: model, data and
    sigma indexed alike, walker s owning [offsets[s], offsets[s+1])."""
    model = np.asarray(model, dtype=np.float64)
    data = np.asarray(data, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    if offsets is None:
        model = model.reshape(-1, data.size)
        chi2 = np.array([math.fsum(v) for v in ((data[None, :] - model) / sigma[None, :]) ** 2])
        norm = math.fsum(np.log(sigma)) + 0.5 * data.size * math.log(2.0 * math.pi)
        return chi2, -0.5 * chi2 - norm
    chi2 = np.empty(len(offsets) - 1)
    ll = np.empty(len(offsets) - 1)
    for s in range(len(offsets) - 1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        r = (data[a:b] - model[a:b]) / sigma[a:b]
        chi2[s] = math.fsum(r * r)
        ll[s] = -0.5 * chi2[s] - math.fsum(np.log(sigma[a:b])) - 0.5 * (b - a) * math.log(2.0 * math.pi)
    return chi2, ll
