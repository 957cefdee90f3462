"""Pins of the CPU oracle against results fixed by the paper and by mathematics.

Each test compares the oracle (an iterated area integral, ``oracle/glo.c``)
with something it does not share code with: textbook closed forms (Mandel &
Agol 2002, ellipse moments, lens area), a radial 1-D integral, the paper's own
parametric ellipse and Green's-theorem integrands evaluated by scipy,
Monte-Carlo area counting, and exact symmetries of the problem.  The paper
prints no light-curve values, so these are the pins.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from tests.pins import green_route as G
from tests.pins import mandel_agol as MA

TWO_PI = 2.0 * math.pi


def occ_circle(glo, z, p, u1, u2, tol=1e-14, mode=0):
    """Oracle occulted fraction for a circle of radius p at distance z."""
    return glo.occulted(0.0, z, 1.0, 0.0, p, 1.0, u1, u2, tol, mode)


def oracle_ellipse_occ(glo, k, f, theta, phi, x0, y0, u1, u2, tol=1e-14, mode=0):
    p = np.array([k, f, theta, phi, 0.3, 200.0, 500.0, 0.0, 0.5, 0.5])
    _, _, _, uh, _, kk, kq = glo.geometry(p, 0.0)
    return glo.occulted(x0, y0, uh[0], uh[1], k, kq / k, u1, u2, tol, mode)


def rand_shape(rng):
    return (rng.uniform(0.03, 0.2), rng.uniform(0.0, 0.95), rng.uniform(0.0, math.pi),
            rng.uniform(0.0, TWO_PI))


# ---------------------------------------------------------------- limb darkening
def test_kipping_map_inverse_and_corners(oracle):
    # Kipping (2013): q1 = (u1+u2)^2, q2 = u1 / (2(u1+u2)) is the inverse map
    rng = np.random.default_rng(0)
    for q1, q2 in rng.uniform(0.0, 1.0, (200, 2)):
        u1, u2 = oracle.kipping(q1, q2)
        assert (u1 + u2) ** 2 == pytest.approx(q1, abs=1e-15)
        if u1 + u2 > 1e-8:
            assert u1 / (2 * (u1 + u2)) == pytest.approx(q2, abs=1e-12)
        # physical triangle: positive intensity everywhere, monotone limb darkening
        assert u1 + u2 <= 1 + 1e-15 and u1 >= 0 and u1 + 2 * u2 >= -1e-15
    assert oracle.kipping(1.0, 0.0) == pytest.approx((0.0, 1.0))
    assert oracle.kipping(1.0, 0.5) == pytest.approx((1.0, 0.0))
    assert oracle.kipping(0.4225, 0.4 / 1.3) == pytest.approx((0.4, 0.25), abs=1e-15)
    with pytest.raises(ValueError):
        oracle.kipping(1.2, 0.5)


def test_small_planet_depth_is_central_intensity_over_mean(oracle):
    # a vanishing disk at the centre blocks pi p^2 I(0) of Phi = integral of I
    for u1, u2 in [(0.0, 0.0), (0.4, 0.25), (1.0, 0.0), (0.1, 0.6)]:
        p = 1e-3
        mean_I = 2.0 * quad(lambda r: (1 - u1 * (1 - math.sqrt(1 - r * r))
                                       - u2 * (1 - math.sqrt(1 - r * r)) ** 2) * r, 0, 1,
                            epsabs=1e-15)[0]
        d = occ_circle(oracle, 0.0, p, u1, u2)
        assert d == pytest.approx(p * p / mean_I, rel=1e-6)


# ---------------------------------------------------------------- spheres (f = 0)
@pytest.mark.parametrize("u1,u2", [(0.0, 0.0), (0.4, 0.25), (1.0, 0.0), (0.0, 1.0), (0.9, -0.3)])
def test_circle_matches_mandel_agol(oracle, u1, u2):
    rng = np.random.default_rng(11)
    zs = []
    for p in [0.02, 0.05, 0.1, 0.12, 0.2]:
        zs += [(p, z) for z in rng.uniform(0.0, 1.0 + p, 12)]
        zs += [(p, 1.0 - p + 1e-6), (p, 1.0 + p - 1e-6), (p, 1.0 - 0.5 * p), (p, 1.0)]
    for p, z in zs:
        if abs(z - p) < 1e-9 or abs(z - (1 - p)) < 1e-9:
            continue
        d_ma = MA.occulted_fraction(p, z, u1, u2)
        d_or = occ_circle(oracle, z, p, u1, u2)
        # within 1e-4 of a contact the closed form's arccos terms are
        # ill-conditioned (error ~ eps / sqrt(gap)), not the oracle
        near_contact = min(abs(z - (1 + p)), abs(z - (1 - p))) < 1e-4
        assert abs(d_ma - d_or) < (1e-12 if near_contact else 2e-13), (p, z)


def test_circle_matches_radial_integral(oracle):
    def radial(p, z, u1, u2):
        c0, c1, c2 = 1 - u1 - 2 * u2, u1 + 2 * u2, u2

        def kappa(r):  # half-angle of the radius-r circle inside the planet
            if r <= p - z:
                return math.pi
            if r <= z - p or r >= z + p:
                return 0.0
            return math.acos(max(-1.0, min(1.0, (r * r + z * z - p * p) / (2 * r * z))))

        lo, hi = max(0.0, z - p), min(1.0, z + p)
        pts = [x for x in (abs(z - p), p - z) if lo < x < hi]
        v = quad(lambda r: (c0 + c1 * math.sqrt(max(0.0, 1 - r * r)) + c2 * r * r) * 2 * r * kappa(r),
                 lo, hi, points=pts or None, epsabs=1e-15, epsrel=1e-15, limit=500)[0]
        return v / (math.pi * (1 - u1 / 3 - u2 / 6))

    for p, z in [(0.1, 0.95), (0.1, 1.05), (0.1, 0.5), (0.12, 0.99), (0.1, 0.05), (0.07, 0.9999)]:
        for u1, u2 in [(0.4, 0.25), (1.0, 0.0)]:
            assert abs(radial(p, z, u1, u2) - occ_circle(oracle, z, p, u1, u2)) < 1e-13


def test_zero_flattening_or_pole_on_is_a_circle(oracle):
    rng = np.random.default_rng(3)
    for _ in range(20):
        k = rng.uniform(0.05, 0.12)
        z = rng.uniform(0.5, 1.0 + k)
        ang = rng.uniform(0, TWO_PI)
        x0, y0 = z * math.cos(ang), z * math.sin(ang)
        u1, u2 = 0.4, 0.25
        ref = MA.occulted_fraction(k, z, u1, u2)
        # f = 0, any orientation
        d1 = oracle_ellipse_occ(oracle, k, 0.0, rng.uniform(0, math.pi), rng.uniform(0, TWO_PI),
                                x0, y0, u1, u2)
        # theta = 0 (spin axis along the line of sight), any f
        d2 = oracle_ellipse_occ(oracle, k, rng.uniform(0, 0.9), 0.0, rng.uniform(0, TWO_PI),
                                x0, y0, u1, u2)
        assert abs(d1 - ref) < 2e-13 and abs(d2 - ref) < 2e-13


# ---------------------------------------------------------------- geometry
def test_oracle_ellipse_is_the_papers_parametric_ellipse(oracle):
    """The oracle builds the silhouette from the spheroid directly; every point
    of the paper's (x0 + dx cos th, y0 + dy1 cos th + dy2 sin th) must lie on
    it, and the orbit centre must be the paper's (d cos a sin b, d sin a)."""
    rng = np.random.default_rng(5)
    th = np.linspace(0, TWO_PI, 97)
    for _ in range(50):
        k, f, theta, phi = rand_shape(rng)
        b, d, P = rng.uniform(-0.9, 0.9), rng.uniform(3, 300), rng.uniform(1, 600)
        t = rng.uniform(-0.3, 0.3) * P
        p = np.array([k, f, theta, phi, b, d, P, 0.0, 0.5, 0.5])
        front, c, z, uh, sh, kk, kq = oracle.geometry(p, t)
        x0, y0, z_ref = G.paper_centre(b, d, P, 0.0, t)
        assert c[0] == pytest.approx(x0, abs=1e-12 * d) and c[1] == pytest.approx(y0, abs=1e-12 * d)
        assert z == pytest.approx(z_ref, abs=1e-12 * d) and front == (z_ref < 0)
        A, B, C = G.paper_deltas(k, f, theta, phi)
        xs, ys = A * np.cos(th), B * np.cos(th) + C * np.sin(th)
        w = (xs * uh[0] + ys * uh[1]) / kk
        v = (xs * sh[0] + ys * sh[1]) / kq
        assert np.max(np.abs(w * w + v * v - 1.0)) < 1e-12
        assert abs(A * C - kk * kq) < 1e-15  # equal areas
        assert abs(uh[0] * sh[0] + uh[1] * sh[1]) < 1e-15


# ---------------------------------------------------------------- full overlap closed forms
def test_uniform_full_overlap_depth_is_area(oracle):
    rng = np.random.default_rng(7)
    for _ in range(40):
        k, f, theta, phi = rand_shape(rng)
        r = rng.uniform(0, 1 - k - 1e-3)
        ang = rng.uniform(0, TWO_PI)
        A, B, C = G.paper_deltas(k, f, theta, phi)
        d = oracle_ellipse_occ(oracle, k, f, theta, phi, r * math.cos(ang), r * math.sin(ang), 0.0, 0.0)
        assert abs(d - A * C) < 1e-15  # pi dx dy2 / pi


def test_full_overlap_r2_moment(oracle):
    # u1 = -2, u2 = 1 gives I = 1 + r^2 exactly (c1 = 0): delta Phi = S_flat + S_quad
    rng = np.random.default_rng(8)
    for _ in range(40):
        k, f, theta, phi = rand_shape(rng)
        r = rng.uniform(0, 1 - k - 1e-3)
        ang = rng.uniform(0, TWO_PI)
        x0, y0 = r * math.cos(ang), r * math.sin(ang)
        A, B, C = G.paper_deltas(k, f, theta, phi)
        area = math.pi * A * C
        s_quad = area * (x0 * x0 + y0 * y0 + (A * A + B * B + C * C) / 4.0)
        d = oracle_ellipse_occ(oracle, k, f, theta, phi, x0, y0, -2.0, 1.0)
        assert abs(d * 1.5 * math.pi - (area + s_quad)) < 1e-14


# ---------------------------------------------------------------- partial overlap
def test_uniform_partial_overlap_is_lens_area(oracle):
    rng = np.random.default_rng(9)
    for _ in range(40):
        k, f, theta, phi = rand_shape(rng)
        A, B, C = G.paper_deltas(k, f, theta, phi)
        rho = rng.uniform(1 - k, 1 + k)
        ang = rng.uniform(0, TWO_PI)
        x0, y0 = rho * math.cos(ang), rho * math.sin(ang)
        lens = G.lens_area(G.Ellipse(x0, y0, A, B, C)) / math.pi
        d = oracle_ellipse_occ(oracle, k, f, theta, phi, x0, y0, 0.0, 0.0)
        assert abs(d - lens) < 1e-14


def test_limb_darkened_matches_papers_green_route(oracle):
    """Partial and full overlaps with limb darkening against the paper's
    boundary integrands on its own parametric ellipse (scipy quadrature)."""
    rng = np.random.default_rng(10)
    worst = 0.0
    for i in range(50):
        k, f, theta, phi = rand_shape(rng)
        A, B, C = G.paper_deltas(k, f, theta, phi)
        rho = rng.uniform(1 - k - 0.05, 1 + k) if i % 5 else rng.uniform(0.0, 1 - k)
        ang = rng.uniform(0, TWO_PI)
        x0, y0 = rho * math.cos(ang), rho * math.sin(ang)
        u1, u2 = G.kipping(rng.uniform(), rng.uniform())
        ref = G.occulted(G.Ellipse(x0, y0, A, B, C), u1, u2)
        d = oracle_ellipse_occ(oracle, k, f, theta, phi, x0, y0, u1, u2)
        worst = max(worst, abs(d - ref))
    assert worst < 1e-12


def test_four_intersection_configuration(oracle):
    """A very flat ellipse whose flat side runs along the limb crosses it four
    times; both routes must still agree."""
    k, f, theta = 0.3, 0.9, math.pi / 2
    A, B, C = G.paper_deltas(k, f, theta, 0.0)
    found = None
    for rho in np.linspace(0.90, 1.03, 131):
        E = G.Ellipse(rho, 0.0, A, B, C)
        if len(E.roots()) == 4:
            found = rho
            break
    assert found is not None
    E = G.Ellipse(found, 0.0, A, B, C)
    for u1, u2 in [(0.0, 0.0), (0.4, 0.25)]:
        ref = G.occulted(E, u1, u2)
        d = oracle_ellipse_occ(oracle, k, f, theta, 0.0, found, 0.0, u1, u2)
        assert abs(d - ref) < 1e-12


def test_monte_carlo_area_counting(oracle):
    """Brute force: count limb-darkened random points inside the paper's
    ellipse and the disk.  Pins to the sampling error only (z-score)."""
    rng = np.random.default_rng(12)
    k, f, theta, phi = 0.1, 0.5, 1.1, 0.7
    A, B, C = G.paper_deltas(k, f, theta, phi)
    u1, u2 = 0.5, 0.2
    for x0, y0 in [(0.3, 0.92), (-0.5, 0.3), (0.99, 0.05)]:
        n = 2_000_000
        px = rng.uniform(-k, k, n) + x0
        py = rng.uniform(-k, k, n) + y0
        cth = (px - x0) / A
        sth = (py - y0 - B * cth) / C
        r2 = px * px + py * py
        inside = (cth * cth + sth * sth <= 1.0) & (r2 < 1.0)
        mu = np.sqrt(np.clip(1.0 - r2, 0.0, None))
        I = np.where(inside, 1 - u1 * (1 - mu) - u2 * (1 - mu) ** 2, 0.0)
        box = 4 * k * k
        est = I.mean() * box / (math.pi * (1 - u1 / 3 - u2 / 6))
        se = I.std() * box / math.sqrt(n) / (math.pi * (1 - u1 / 3 - u2 / 6))
        d = oracle_ellipse_occ(oracle, k, f, theta, phi, x0, y0, u1, u2)
        assert abs(d - est) < 5 * se


# ---------------------------------------------------------------- invariants
def _flux(oracle, p, t, **kw):
    return oracle.flux(np.asarray(p, float), t, **kw)


def _rand_params(rng):
    k, f, theta, phi = rand_shape(rng)
    q1, q2 = rng.uniform(size=2)
    return [min(k, 0.12), f, theta, phi, rng.uniform(0, 0.9), rng.uniform(100, 300), 500.0, 0.0, q1, q2]


def test_symmetries(oracle):
    rng = np.random.default_rng(13)
    for _ in range(25):
        p = _rand_params(rng)
        t14 = 500 / math.pi * math.asin((1 + p[0]) / p[5])
        t = rng.uniform(-0.6, 0.6) * t14
        F = _flux(oracle, p, t)
        q = list(p); q[2] = math.pi - p[2]                 # theta -> pi - theta
        assert abs(_flux(oracle, q, t) - F) < 1e-14
        q = list(p); q[3] = p[3] + math.pi                 # phi -> phi + pi
        assert abs(_flux(oracle, q, t) - F) < 1e-14
        q = list(p); q[3] = -p[3]                          # mirror y: t -> -t, phi -> -phi
        assert abs(_flux(oracle, q, -t) - F) < 1e-14
        q = list(p); q[4] = -p[4]; q[3] = math.pi - p[3]   # mirror x: b -> -b, phi -> pi - phi
        assert abs(_flux(oracle, q, t) - F) < 1e-14
        assert abs(_flux(oracle, p, t + 500.0) - F) < 1e-11  # period
        assert 0.0 <= F <= 1.0


def test_flattening_obliquity_degeneracy(oracle):
    """Appendix A: flux depends on (f, eta) only through
    mu = (f-1)^2 + f(f-2) cos(2 eta); equal mu -> identical light curves."""
    rng = np.random.default_rng(14)
    for _ in range(20):
        p = _rand_params(rng)
        f1, eta1 = rng.uniform(0.1, 0.9), rng.uniform(-math.pi / 2, math.pi / 2)
        mu = (f1 - 1) ** 2 + f1 * (f1 - 2) * math.cos(2 * eta1)
        f_min = 1 - math.sqrt((mu + 1) / 2)
        f2 = f_min + (1 - f_min) * rng.uniform(0.05, 0.95)
        c2eta = (mu - (f2 - 1) ** 2) / (f2 * (f2 - 2))
        eta2 = 0.5 * math.acos(max(-1.0, min(1.0, c2eta)))
        p1 = list(p); p1[1], p1[2] = f1, math.pi / 2 - eta1
        p2 = list(p); p2[1], p2[2] = f2, math.pi / 2 - eta2
        t14 = 500 / math.pi * math.asin((1 + p[0]) / p[5])
        for t in rng.uniform(-0.6, 0.6, 4) * t14:
            assert abs(_flux(oracle, p1, t) - _flux(oracle, p2, t)) < 1e-13


def test_out_of_transit_and_behind_the_star(oracle):
    # far from transit: exactly 1
    p = [0.1, 0.3, 1.0, 0.5, 0.3, 200.0, 500.0, 0.0, 0.4, 0.3]
    assert _flux(oracle, p, 2.0) == 1.0
    # close orbit: at alpha = pi the planet sits over the stellar centre but
    # behind the star, so nothing is occulted; at alpha = 0 it transits
    p = [0.1, 0.3, 1.0, 0.5, 0.0, 1.5, 1.0, 0.0, 0.4, 0.3]
    assert _flux(oracle, p, 0.5) == 1.0
    assert _flux(oracle, p, 0.0) < 0.995


def test_continuity_through_contact(oracle):
    p = [0.1, 0.6, 1.2, 0.4, 0.3, 200.0, 500.0, 0.0, 0.4, 0.3]
    # locate first contact by bisection on the geometry
    lo, hi = -1.0, 0.0
    for _ in range(60):
        m = 0.5 * (lo + hi)
        if _flux(oracle, p, m) < 1.0:
            hi = m
        else:
            lo = m
    assert _flux(oracle, p, lo) == 1.0
    for eps in [1e-9, 1e-7, 1e-5]:
        d = 1.0 - _flux(oracle, p, hi + eps)
        assert 0.0 < d < 1e-3 * (eps / 1e-5) ** 1.2 + 1e-12


# ---------------------------------------------------------------- the oracle itself
def test_tolerance_sweep_and_inner_modes(oracle):
    rng = np.random.default_rng(15)
    for _ in range(12):
        k, f, theta, phi = rand_shape(rng)
        rho = rng.uniform(1 - k, 1 + k)
        ang = rng.uniform(0, TWO_PI)
        x0, y0 = rho * math.cos(ang), rho * math.sin(ang)
        u1, u2 = 0.4, 0.25
        ref = oracle_ellipse_occ(oracle, k, f, theta, phi, x0, y0, u1, u2, tol=1e-14)
        for tol in (1e-8, 1e-10, 1e-12):
            assert abs(oracle_ellipse_occ(oracle, k, f, theta, phi, x0, y0, u1, u2, tol=tol) - ref) <= tol
        lit = oracle_ellipse_occ(oracle, k, f, theta, phi, x0, y0, u1, u2, tol=1e-13, mode=1)
        assert abs(lit - ref) < 1e-13


def test_supersampling_is_box_average(oracle):
    p = [0.1, 0.3, 1.0, 0.5, 0.3, 200.0, 500.0, 0.0, 0.4, 0.3]
    t_exp = 0.02
    for t in (-0.3, -0.1, 0.2):  # exposures away from contact: smooth integrand
        assert abs(_flux(oracle, p, t, t_exp=0.0, n_ss=15) - _flux(oracle, p, t)) < 1e-15
        box = quad(lambda s: _flux(oracle, p, s), t - t_exp / 2, t + t_exp / 2,
                   epsabs=1e-15, epsrel=1e-14)[0] / t_exp
        e16 = abs(_flux(oracle, p, t, t_exp=t_exp, n_ss=16) - box)
        e32 = abs(_flux(oracle, p, t, t_exp=t_exp, n_ss=32) - box)
        # midpoint rule: error ~ n^-2
        assert e32 < 0.3 * e16 + 1e-15
        assert e16 < 1e-7


def test_domain_errors_give_nan(oracle):
    good = [0.1, 0.3, 1.0, 0.5, 0.3, 200.0, 500.0, 0.0, 0.4, 0.3]
    assert math.isfinite(_flux(oracle, good, 0.0))
    for i, v in [(0, 0.0), (0, 1.2), (1, 1.0), (1, -0.1), (5, 1.05), (6, 0.0), (8, 1.5),
                 (9, -0.2), (4, 300.0), (0, float("nan")), (6, float("inf"))]:
        bad = list(good)
        bad[i] = v
        assert math.isnan(_flux(oracle, bad, 0.0))
    assert math.isnan(_flux(oracle, good, 0.0, n_ss=0))
    assert math.isnan(_flux(oracle, good, 0.0, n_ss=65))
