"""Pins of the oracle at near-tangency, where the occulted region's boundary
switches between ellipse and limb at two nearby points.

The oracle splits its outer integral at every kink of the integrand (where an
active chord limit switches between the ellipse and the disk, Section 2: the
region is the ellipse cut by the stellar disk).  Near a tangency two such
kinks can fall between neighbouring scan points, or between the last scan
point and the end of the disk chord; missing them leaves an integrand with
a kink and a square-root end inside one panel, which the adaptive rule can
accept with a wrong error estimate (it did: 1.5e-10 off at a vertex poking
out of the limb by 1e-5).  Here the uniform-source value is compared with the
closed-form lens area (exact given the intersection points), and the
limb-darkened value with the paper's Green's-theorem integrands, for an
ellipse poking out of (or just inside) the limb at its vertices and at
generic tangency points.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from tests.pins import green_route as G


def _shape(glo, k, f, theta, phi):
    p = np.array([k, f, theta, phi, 0.3, 200.0, 500.0, 0.0, 0.5, 0.5])
    _, _, _, uh, sh, _, kq = glo.geometry(p, 0.0)
    return G.paper_deltas(k, f, theta, phi), uh, sh, kq


def _occ(glo, cx, cy, uh, k, kq, u1, u2):
    return glo.occulted(cx, cy, uh[0], uh[1], k, kq / k, u1, u2)


@pytest.mark.parametrize("eps", [1e-3, 1e-5, 1e-7, 1e-9, -1e-9])
def test_vertex_just_across_the_limb_is_lens_area(oracle, eps):
    k, f, theta, phi = 0.1, 0.3, math.pi / 3, math.pi / 6
    (A, B, C), uh, sh, kq = _shape(oracle, k, f, theta, phi)
    # the centre on each semi-axis direction, the vertex eps beyond the limb
    for ax, r in ((uh, k), (-uh, k), (sh, kq), (-sh, kq)):
        cx, cy = (1.0 - r + eps) * ax[0], (1.0 - r + eps) * ax[1]
        lens = G.lens_area(G.Ellipse(cx, cy, A, B, C)) / math.pi
        assert abs(_occ(oracle, cx, cy, uh, k, kq, 0.0, 0.0) - lens) < 1e-15


def _tangent_distance(A, B, C, dx, dy):
    """Centre distance along (dx, dy) at which the ellipse touches the limb
    from inside (largest |p(theta)| = 1), by bracketing on a dense grid."""
    th = np.linspace(0.0, 2.0 * math.pi, 20001)

    def excess(rho):
        x = rho * dx + A * np.cos(th)
        y = rho * dy + B * np.cos(th) + C * np.sin(th)
        return np.max(x * x + y * y) - 1.0

    return brentq(excess, 0.0, 1.0, xtol=1e-15)


def test_generic_tangency_is_lens_area(oracle):
    rng = np.random.default_rng(5)
    for _ in range(40):
        k, f = rng.uniform(0.03, 0.3), rng.uniform(0.0, 0.95)
        theta, phi = rng.uniform(0.0, math.pi), rng.uniform(0.0, 2.0 * math.pi)
        (A, B, C), uh, _, kq = _shape(oracle, k, f, theta, phi)
        ang = rng.uniform(0.0, 2.0 * math.pi)
        dx, dy = math.cos(ang), math.sin(ang)
        rs = _tangent_distance(A, B, C, dx, dy)
        for eps in (1e-4, 1e-6, 1e-8, -1e-8):
            cx, cy = (rs + eps) * dx, (rs + eps) * dy
            lens = G.lens_area(G.Ellipse(cx, cy, A, B, C)) / math.pi
            assert abs(_occ(oracle, cx, cy, uh, k, kq, 0.0, 0.0) - lens) < 1e-15


def test_limb_darkened_tangency_matches_green_route(oracle):
    rng = np.random.default_rng(6)
    for i in range(12):
        k, f = rng.uniform(0.05, 0.2), rng.uniform(0.1, 0.9)
        theta, phi = rng.uniform(0.0, math.pi), rng.uniform(0.0, 2.0 * math.pi)
        (A, B, C), uh, _, kq = _shape(oracle, k, f, theta, phi)
        ang = rng.uniform(0.0, 2.0 * math.pi)
        dx, dy = math.cos(ang), math.sin(ang)
        rs = _tangent_distance(A, B, C, dx, dy)
        eps = 10.0 ** -(3 + i % 5)
        cx, cy = (rs + eps) * dx, (rs + eps) * dy
        u1, u2 = 0.4, 0.25
        want = G.occulted(G.Ellipse(cx, cy, A, B, C), u1, u2)
        assert abs(_occ(oracle, cx, cy, uh, k, kq, u1, u2) - want) < 1e-12


def test_no_adaptive_integral_stopped_short(oracle):
    """Every adaptive integral of the pins so far met its error target."""
    for i in range(5):
        cx, cy = 0.9 + 1e-7 * i, 0.05
        oracle.occulted(cx, cy, 1.0, 0.0, 0.1, 0.5, 0.4, 0.25)
    assert oracle.unconverged() == 0
