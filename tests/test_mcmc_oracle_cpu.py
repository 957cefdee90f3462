"""Pins of the oracle's MCMC glue (oracle/mcmc.py): the (mu, nu) prior
sampler of Appendix A against the CDFs and the joint density the paper states
for it, against the target prior p(f, eta) ~ cos(eta), and against the flux
degeneracy that motivates it; the white-noise likelihood against closed forms."""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import mcmc as M

HERE = os.path.dirname(os.path.abspath(__file__))


def joint_density(mu, nu):
    """Eq. mu-nu-joint-density."""
    return 2.0 ** -1.5 * (nu * (nu - 2.0) * (mu * (nu - 1.0) ** 2 + nu * (nu - 2.0) - 1.0)) ** -0.5


def test_nu_inverts_its_marginal_cdf():
    """F(nu) = (nu - sqrt(nu (2 - nu))) / (nu - 1) at nu(u) returns u, and F is
    the integral of the marginal p(nu) = 1 / (nu (2 - nu) + sqrt(nu (2 - nu)))."""
    u = np.linspace(0.001, 0.999, 999)
    nu = M.nu_of_u(u)
    F = (nu - np.sqrt(nu * (2 - nu))) / (nu - 1)
    assert np.max(np.abs(F - u)) < 1e-12
    for n in (0.05, 0.3, 0.7, 0.95):
        val = integrate.quad(lambda x: 1.0 / (x * (2 - x) + math.sqrt(x * (2 - x))), 0, n)[0]
        assert M.nu_of_u(np.array([val]))[0] == pytest.approx(n, rel=1e-9)


def test_marginal_is_the_joint_density_integrated():
    """p(nu) equals the joint density integrated over mu in [-1, 1]."""
    for n in (0.02, 0.2, 0.5, 0.8, 0.97):
        val = integrate.quad(lambda m: joint_density(m, n), -1.0, 1.0, limit=200)[0]
        ref = 1.0 / (n * (2 - n) + math.sqrt(n * (2 - n)))
        assert val == pytest.approx(ref, rel=1e-8)


def test_mu_inverts_its_conditional_cdf():
    """F(mu | nu) of Appendix A at mu(w, nu) returns w, and F(mu | nu) is the
    integral of p(mu, nu) / p(nu) from -1 (checked by quadrature)."""
    rng = np.random.default_rng(1)
    for _ in range(40):
        nu = rng.uniform(0.01, 0.99)
        w = rng.uniform(0.01, 0.99)
        mu = float(M.mu_of_w(np.array([w]), np.array([nu]))[0])
        assert -1.0 <= mu <= 1.0
        s = math.sqrt(nu * (2 - nu))
        F = (1 + s) * (2 - math.sqrt(2 - 2 * mu * (nu - 1) ** 2 - 2 * nu * (nu - 2))) / (2 * (nu - 1) ** 2)
        assert F == pytest.approx(w, abs=1e-12)
        pn = 1.0 / (nu * (2 - nu) + s)
        q = integrate.quad(lambda m: joint_density(m, nu) / pn, -1.0, mu, limit=200)[0]
        assert q == pytest.approx(w, abs=1e-8)


def test_sampled_mu_nu_histogram_matches_the_joint_density():
    rng = np.random.default_rng(2)
    n = 1_000_000
    mu, nu = M.mu_nu_from_uniforms(rng.uniform(size=n), rng.uniform(size=n))
    me = np.linspace(-1, 1, 9)
    ne = np.linspace(0, 1, 9)
    h, _, _ = np.histogram2d(mu, nu, bins=[me, ne])
    expect = np.empty_like(h)
    for i in range(8):
        for j in range(8):
            expect[i, j] = n * integrate.dblquad(lambda m, x: joint_density(m, x), ne[j], ne[j + 1],
                                                 me[i], me[i + 1], epsabs=1e-10)[0]
    assert expect.sum() == pytest.approx(n, rel=1e-6)
    chi2 = np.sum((h - expect) ** 2 / expect)
    assert chi2 < stats.chi2.ppf(0.999, 63)


def test_prior_recovers_uniform_f_and_cosine_eta():
    """p(f, eta) ~ cos(eta): f ~ U[0, 1] and sin(eta) ~ U[0, 1] (eta in [0, pi/2])."""
    rng = np.random.default_rng(3)
    n = 400_000
    mu, nu = M.mu_nu_from_uniforms(rng.uniform(size=n), rng.uniform(size=n))
    f, eta = M.f_eta_from_mu_nu(mu, nu)
    assert np.all((f >= 0) & (f <= 1)) and np.all((eta >= 0) & (eta <= 0.5 * math.pi))
    assert stats.kstest(f, "uniform").pvalue > 1e-3
    assert stats.kstest(np.sin(eta), "uniform").pvalue > 1e-3
    # independence: the correlation of f and sin(eta) vanishes
    assert abs(np.corrcoef(f, np.sin(eta))[0, 1]) < 0.01
    # round trip through eq. mu and the definition of nu
    assert np.max(np.abs(M.mu_of_f_eta(f, eta) - mu)) < 1e-9
    f_min = 1 - np.sqrt((mu + 1) / 2)
    ok = f_min < 1 - 1e-6
    assert np.max(np.abs((f - f_min)[ok] / (1 - f_min)[ok] - nu[ok])) < 1e-9


def test_equal_mu_gives_equal_light_curves(oracle):
    """The degeneracy of Appendix A (its Figure: f = 1/2, eta = 0 and
    f = 2/3, eta = 23.3 deg share mu = -1/2): with the equatorial radius held,
    as in that Figure, the two oblate planets give the same light curve
    (mu = 2 q^2 - 1 fixes the projected axis ratio q)."""
    eta2 = 0.5 * math.acos(11.0 / 16.0)
    assert M.mu_of_f_eta(0.5, 0.0) == pytest.approx(-0.5)
    assert M.mu_of_f_eta(2.0 / 3.0, eta2) == pytest.approx(-0.5)
    assert math.degrees(eta2) == pytest.approx(23.28, abs=0.01)
    walk = np.array([[0.08, 0.08], [-0.5, -0.5], [0.0, 0.0], [0.4, 0.4], [0.3, 0.3], [40.0, 40.0],
                     [10.0, 10.0], [0.0, 0.0], [0.3, 0.3], [0.4, 0.4]])
    p = M.params_from_walkers(walk)
    # the two (f, eta): the same mu, different flattenings
    p[1] = [0.5, 2.0 / 3.0]
    p[2] = [0.5 * math.pi, 0.5 * math.pi - eta2]
    p[0] = [0.08, 0.08]  # the same equatorial radius
    t = np.linspace(-0.12, 0.12, 301)
    fl = oracle.flux_batch(p, t)
    assert np.min(fl) < 0.999
    assert np.max(np.abs(fl[0] - fl[1])) < 1e-13


def test_params_from_walkers_keeps_the_mean_radius():
    rng = np.random.default_rng(4)
    walk = np.empty((10, 50))
    walk[M.W_R] = rng.uniform(0.01, 0.1, 50)
    walk[M.W_MU], walk[M.W_NU] = M.mu_nu_from_uniforms(rng.uniform(size=50), rng.uniform(size=50))
    walk[3:] = rng.uniform(size=(7, 50))
    p = M.params_from_walkers(walk)
    k, f = p[0], p[1]
    assert np.allclose((k * k * k * (1 - f)) ** (1 / 3), walk[M.W_R], rtol=1e-13)
    assert np.array_equal(p[3:], walk[3:])


def test_walker_shadow_axis_ratio_is_fixed_by_mu(oracle):
    """mu = 2 q^2 - 1 for the projected axis ratio q of the converted planet
    (eq. mu with the oblate shadow), read from the oracle's geometry."""
    rng = np.random.default_rng(6)
    n = 200
    walk = np.empty((10, n))
    walk[M.W_R] = rng.uniform(0.01, 0.1, n)
    walk[M.W_MU], walk[M.W_NU] = M.mu_nu_from_uniforms(rng.uniform(0, 0.95, n), rng.uniform(size=n))
    walk[M.W_XI] = rng.uniform(0, 0.5 * math.pi, n)
    walk[M.W_B:] = np.array([[0.2], [50.0], [10.0], [0.0], [0.3], [0.3]])
    p = M.params_from_walkers(walk)
    for s in range(n):
        g = oracle.geometry(p[:, s], 0.0)
        q = g[6] / g[5]
        assert 2 * q * q - 1 == pytest.approx(walk[M.W_MU, s], abs=1e-12)


def test_loglike_closed_forms():
    rng = np.random.default_rng(5)
    n = 777
    data = 1 + rng.normal(0, 1e-4, n)
    sigma = rng.uniform(1e-5, 3e-5, n)
    model = np.stack([data, data + 2e-5, data - sigma])
    chi2, ll = M.loglike(model, data, sigma)
    norm = np.sum(np.log(sigma)) + 0.5 * n * math.log(2 * math.pi)
    assert chi2[0] == 0.0 and ll[0] == pytest.approx(-norm, rel=1e-15)
    # (the offsets are exact up to the rounding of data + offset near 1: 1e-11 relative)
    assert chi2[1] == pytest.approx(np.sum((2e-5 / sigma) ** 2), rel=1e-9)
    assert chi2[2] == pytest.approx(n, rel=1e-9)
    # CSR: the same numbers per segment
    offs = np.array([0, n, 2 * n, 3 * n])
    c2, l2 = M.loglike(model.ravel(), np.tile(data, 3), np.tile(sigma, 3), offs)
    assert np.allclose(c2, chi2, rtol=1e-15) and np.allclose(l2, ll, rtol=1e-15)


def test_injected_curve_file():
    """The stored JWST-like visit: noise of the stated size around the model."""
    d = np.loadtxt(os.path.join(HERE, "golden", "jwst_injected.txt"))
    t, data, sigma, model = d.T
    assert np.allclose(np.diff(t), 2.0 / 1440.0)
    resid = (data - model) / sigma
    assert abs(np.std(resid) - 1.0) < 0.06 and abs(np.mean(resid)) < 0.1
    assert 0.004 < 1 - model.min() < 0.006
