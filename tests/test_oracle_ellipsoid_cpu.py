"""Pins of the oracle's general-ellipsoid geometry (Section 2 for any a, b, c
and orientation; Appendix B for tidally-locked planets).

The oracle builds the sky shadow as the Schur complement of the rotated body
quadric.  These tests hold it against what does not share that route: the
paper's own parametric curve (eqs. dx, dy1, dy2 and their locked forms, typed
term by term), brute-force sampling of the ellipsoid surface, the projected
area of an ellipsoid in closed form, a locked shadow whose axes follow from
the geometry by hand, and reductions to the oblate oracle and to Mandel & Agol.
"""
import math

import numpy as np
import pytest

from tests.pins import green_route as G
from tests.pins import mandel_agol as MA

TWO_PI = 2.0 * math.pi


def pblock(a, b, c, zeta, eta, xi, imp=0.3, ars=20.0, P=3.0, t0=0.0, q1=0.36, q2=0.3, locked=0):
    return np.array([a, b, c, zeta, eta, xi, imp, ars, P, t0, q1, q2, float(locked)])


def rand_ell(rng):
    return (rng.uniform(0.03, 0.2), rng.uniform(0.03, 0.2), rng.uniform(0.03, 0.2),
            rng.uniform(-math.pi, math.pi), rng.uniform(-math.pi, math.pi), rng.uniform(-math.pi, math.pi))


def on_shadow(g, xs, ys):
    """max | (w/k1)^2 + (v/k2)^2 - 1 | of offsets (xs, ys) from the shadow centre."""
    _, _, uh, sh, k1, k2 = g
    w = (xs * uh[0] + ys * uh[1]) / k1
    v = (xs * sh[0] + ys * sh[1]) / k2
    return np.max(np.abs(w * w + v * v - 1.0))


def body_map(p, t):
    """M with body coordinates = M (x - x_c): R, or R Rx(-alpha) Ry(beta) when locked."""
    a, b, c, zeta, eta, xi, imp, ars, P, t0 = p[:10]
    R = G.rx(zeta) @ G.ry(eta) @ G.rz(xi)
    if p[12]:
        alpha = TWO_PI * (t - t0) / P
        R = R @ G.rx(-alpha) @ G.ry(math.asin(imp / ars))
    return R


def test_shadow_is_the_papers_parametric_curve(oracle):
    """Every point x0 + (dx cos th, dy1 cos th + dy2 sin th) of eqs. dx, dy1, dy2
    lies on the oracle's shadow, and the centre is the paper's."""
    rng = np.random.default_rng(21)
    th = np.linspace(0, TWO_PI, 97)
    for _ in range(60):
        a, b, c, zeta, eta, xi = rand_ell(rng)
        imp, ars, P = rng.uniform(-0.9, 0.9), rng.uniform(3, 300), rng.uniform(1, 600)
        t = rng.uniform(-0.3, 0.3) * P
        p = pblock(a, b, c, zeta, eta, xi, imp, ars, P)
        g = oracle.geometry_ell(p, t)
        x0, y0, z0 = G.paper_centre(imp, ars, P, 0.0, t)
        assert g[1] == pytest.approx([x0, y0, z0], abs=1e-12 * ars)
        assert g[0] == (z0 < 0)
        A, B, C = G.paper_deltas_ell(a, b, c, zeta, eta, xi)
        assert on_shadow(g, A * np.cos(th), B * np.cos(th) + C * np.sin(th)) < 1e-12
        assert abs(A * C - g[4] * g[5]) < 1e-15  # equal areas


def test_locked_shadow_is_the_papers_locked_curve(oracle):
    """Tidally locked: the curve of eqs. dx-locked, dy1-locked, dy2-locked at
    the orbital phase alpha = 2 pi (t - t0) / P, beta = asin(b / d)."""
    rng = np.random.default_rng(22)
    th = np.linspace(0, TWO_PI, 97)
    for _ in range(60):
        a, b, c, zeta, eta, xi = rand_ell(rng)
        imp, ars, P, t0 = rng.uniform(-0.9, 0.9), rng.uniform(2, 30), rng.uniform(0.5, 10), rng.uniform(-1, 1)
        t = t0 + rng.uniform(-0.45, 0.45) * P
        p = pblock(a, b, c, zeta, eta, xi, imp, ars, P, t0, locked=1)
        g = oracle.geometry_ell(p, t)
        alpha, beta = TWO_PI * (t - t0) / P, math.asin(imp / ars)
        A, B, C = G.paper_deltas_locked(a, b, c, zeta, eta, xi, alpha, beta)
        assert on_shadow(g, A * np.cos(th), B * np.cos(th) + C * np.sin(th)) < 1e-11
        assert abs(A * C - g[4] * g[5]) < 1e-14


def test_locked_shadow_closed_form(oracle):
    """R = I, b = 0: the axis z' (length c) points at the star; at phase alpha
    the shadow has semi-axis a along x and sqrt(b^2 cos^2 + c^2 sin^2) along y.
    Unlocked, the same body keeps its a x b shadow at every phase."""
    a, b, c = 0.05, 0.08, 0.14
    for alpha in [0.0, 0.01, 0.05, 0.3, -0.2, 1.0]:
        t = alpha / TWO_PI * 3.0
        g = oracle.geometry_ell(pblock(a, b, c, 0.0, 0.0, 0.0, 0.0, 20.0, 3.0, locked=1), t)
        axes = sorted([g[4], g[5]])
        want = sorted([a, math.sqrt(b * b * math.cos(alpha) ** 2 + c * c * math.sin(alpha) ** 2)])
        assert axes == pytest.approx(want, rel=1e-13)
        along_y = max(abs(g[2][1]), abs(g[3][1]))  # one axis is y
        assert along_y == pytest.approx(1.0, abs=1e-12)
        gu = oracle.geometry_ell(pblock(a, b, c, 0.0, 0.0, 0.0, 0.0, 20.0, 3.0), t)
        assert sorted([gu[4], gu[5]]) == pytest.approx([a, b], rel=1e-13)


def test_projected_area_closed_form(oracle):
    """An ellipsoid's orthographic shadow along the body-frame unit direction n
    has area pi a b c sqrt(n_x^2/a^2 + n_y^2/b^2 + n_z^2/c^2)."""
    rng = np.random.default_rng(23)
    for locked in (0, 1):
        for _ in range(40):
            a, b, c, zeta, eta, xi = rand_ell(rng)
            imp, ars, P = rng.uniform(-0.9, 0.9), rng.uniform(2, 30), rng.uniform(0.5, 10)
            t = rng.uniform(-0.4, 0.4) * P
            p = pblock(a, b, c, zeta, eta, xi, imp, ars, P, locked=locked)
            g = oracle.geometry_ell(p, t)
            n = body_map(p, t) @ np.array([0.0, 0.0, 1.0])
            area = math.pi * a * b * c * math.sqrt((n[0] / a) ** 2 + (n[1] / b) ** 2 + (n[2] / c) ** 2)
            assert math.pi * g[4] * g[5] == pytest.approx(area, rel=1e-12)


def test_shadow_support_by_surface_sampling(oracle):
    """Brute force: the farthest reach of sampled surface points along sky
    directions w equals the shadow's support function."""
    rng = np.random.default_rng(24)
    u = np.linspace(0.0, math.pi, 721)
    v = np.linspace(0.0, TWO_PI, 1441)
    U, V = np.meshgrid(u, v, indexing="ij")
    ws = np.stack([np.cos(np.linspace(0, TWO_PI, 24, endpoint=False)),
                   np.sin(np.linspace(0, TWO_PI, 24, endpoint=False))], axis=1)
    for locked in (0, 1):
        for _ in range(6):
            a, b, c, zeta, eta, xi = rand_ell(rng)
            p = pblock(a, b, c, zeta, eta, xi, 0.4, 8.0, 2.0, locked=locked)
            t = rng.uniform(-0.3, 0.3)
            body = np.stack([a * np.sin(U) * np.cos(V), b * np.sin(U) * np.sin(V), c * np.cos(U)]).reshape(3, -1)
            sky = (body_map(p, t).T @ body)[:2]  # M is a rotation: its inverse is M^T
            _, _, uh, sh, k1, k2 = oracle.geometry_ell(p, t)
            for w in ws:
                brute = np.max(w @ sky)
                supp = math.sqrt((k1 * (w @ uh)) ** 2 + (k2 * (w @ sh)) ** 2)
                # grid spacing pi/720: the sampled maximum is low by at most ~1e-5 k
                assert brute <= supp * (1 + 1e-12) and brute >= supp * (1 - 2e-5)


def test_spheroid_reduces_to_the_oblate_oracle(oracle):
    """b = c: the oblate model with a = k (1 - f), zeta = 0, eta = pi/2 - theta,
    xi = phi, whose oracle builds the shadow from the spheroid directly."""
    rng = np.random.default_rng(25)
    n = 24
    ob = np.empty((10, n))
    el = np.empty((13, n))
    for s in range(n):
        k, f, th, ph = rng.uniform(0.03, 0.2), rng.uniform(0, 0.9), rng.uniform(0, math.pi), rng.uniform(0, TWO_PI)
        imp, ars, P, q1, q2 = rng.uniform(-0.8, 0.8), rng.uniform(5, 300), rng.uniform(1, 600), rng.uniform(), rng.uniform()
        ob[:, s] = [k, f, th, ph, imp, ars, P, 0.0, q1, q2]
        el[:, s] = [k * (1 - f), k, k, 0.0, 0.5 * math.pi - th, ph, imp, ars, P, 0.0, q1, q2, 0.0]
    ts = np.linspace(-0.6, 0.6, 41)
    scale = np.array([ob[6, s] * (1.2 + ob[0, s]) / (math.pi * ob[5, s]) for s in range(n)])
    times = ts[None, :] * scale[:, None]
    offs = np.arange(n + 1) * ts.size
    fo = oracle.flux_batch(ob, times.ravel(), offsets=offs)
    fe = oracle.flux_batch_ell(el, times.ravel(), offsets=offs)
    assert np.max(np.abs(fo - fe)) < 1e-14
    assert np.min(fo) < 1.0 - 1e-4  # the windows hold transits


def test_sphere_is_mandel_agol(oracle):
    """a = b = c = p at any orientation, locked or not: Mandel & Agol."""
    rng = np.random.default_rng(26)
    for _ in range(30):
        pr = rng.uniform(0.03, 0.15)
        zeta, eta, xi = rng.uniform(-math.pi, math.pi, 3)
        imp, ars, P = rng.uniform(0, 0.9), rng.uniform(3, 50), rng.uniform(1, 20)
        t = rng.uniform(-1, 1) * P / (math.pi * ars)
        q1, q2 = rng.uniform(0.05, 1), rng.uniform(0, 1)
        u1, u2 = G.kipping(q1, q2)
        for locked in (0, 1):
            p = pblock(pr, pr, pr, zeta, eta, xi, imp, ars, P, 0.0, q1, q2, locked)
            f = oracle.flux_batch_ell(p[:, None], np.array([t]))[0, 0]
            x0, y0, _ = G.paper_centre(imp, ars, P, 0.0, t)
            z = math.hypot(x0, y0)
            if min(abs(z - 1 - pr), abs(z - 1 + pr)) < 1e-4:
                continue
            assert f == pytest.approx(1.0 - MA.occulted_fraction(pr, z, u1, u2), abs=3e-13)


def test_locked_follows_its_orbit(oracle):
    """Locked at phase alpha is the unlocked body turned by Rx(-alpha) Ry(beta):
    the oracle's locked shadow equals its unlocked shadow for the angles of
    R Rx(-alpha) Ry(beta) (decomposed back into Rx Ry Rz)."""
    rng = np.random.default_rng(27)
    for _ in range(40):
        a, b, c, zeta, eta, xi = rand_ell(rng)
        imp, ars, P = rng.uniform(-0.9, 0.9), rng.uniform(2, 30), rng.uniform(0.5, 10)
        t = rng.uniform(-0.4, 0.4) * P
        pl = pblock(a, b, c, zeta, eta, xi, imp, ars, P, locked=1)
        M = body_map(pl, t)
        eta2 = math.asin(max(-1.0, min(1.0, M[0, 2])))
        zeta2 = math.atan2(-M[1, 2], M[2, 2])
        xi2 = math.atan2(-M[0, 1], M[0, 0])
        assert np.allclose(G.rx(zeta2) @ G.ry(eta2) @ G.rz(xi2), M, atol=1e-12)
        gl_ = oracle.geometry_ell(pl, t)
        gu = oracle.geometry_ell(pblock(a, b, c, zeta2, eta2, xi2, imp, ars, P), t)
        assert gl_[4] == pytest.approx(gu[4], rel=1e-11) and gl_[5] == pytest.approx(gu[5], rel=1e-11)
        assert abs(abs(gl_[2] @ gu[2]) - 1.0) < 1e-9 or abs(gl_[4] - gl_[5]) < 1e-9 * gl_[4]


def test_ellipsoid_domain_errors_give_nan(oracle):
    good = pblock(0.1, 0.08, 0.06, 0.1, 0.2, 0.3)
    bad = []
    for i, v in [(0, 0.0), (1, 1.0), (2, -0.1), (7, 1.05), (6, 25.0), (8, 0.0), (10, 1.5), (11, -0.1),
                 (12, 0.5), (3, float("nan"))]:
        p = good.copy()
        p[i] = v
        bad.append(p)
    params = np.stack([good] + bad, axis=1)
    out = oracle.flux_batch_ell(params, np.array([0.0, 0.01]))
    assert np.all(np.isfinite(out[0])) and out[0, 0] < 1.0
    assert np.all(np.isnan(out[1:]))
