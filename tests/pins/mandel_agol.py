"""Quadratic limb-darkened transit of a spherical planet in closed form.

Mandel & Agol (2002, ApJ 580, L171), Section 4: the occulted flux of a disk of
radius p (stellar radii) at centre separation z from a star with
I(mu)/I(1) = 1 - g1 (1 - mu) - g2 (1 - mu)^2.  The complete elliptic integrals
are evaluated through Carlson's symmetric forms (Carlson 1995) as provided by
scipy.  Written from the published formulas; it is the textbook value the
paper's spherical validation (Section 2.1) compares against, and it pins the
oracle at f = 0.

Only the configurations a small planet (p < 1/2) can reach are covered:
no overlap, partial overlap, and full overlap off-centre (z > p) and over the
centre (z < p).  Degenerate edges (z exactly p, 1 - p, 0) are avoided by the
callers.
"""
from __future__ import annotations

import math

from scipy.special import elliprf, elliprd, elliprj


def _K(k):
    return float(elliprf(0.0, 1.0 - k * k, 1.0))


def _E(k):
    m = k * k
    return float(elliprf(0.0, 1.0 - m, 1.0) - m / 3.0 * elliprd(0.0, 1.0 - m, 1.0))


def _Pi(n, k):
    """Pi(n, k) = integral_0^{pi/2} dphi / ((1 - n sin^2) sqrt(1 - k^2 sin^2))."""
    m = k * k
    return float(elliprf(0.0, 1.0 - m, 1.0) + n / 3.0 * elliprj(0.0, 1.0 - m, 1.0, 1.0 - n))


def _lambda_e(p, z):
    """Uniform-source occulted fraction (area / pi)."""
    if z >= 1.0 + p:
        return 0.0
    if z <= 1.0 - p:
        return p * p
    k0 = math.acos((p * p + z * z - 1.0) / (2.0 * p * z))
    k1 = math.acos((1.0 - p * p + z * z) / (2.0 * z))
    return (p * p * k0 + k1 - 0.5 * math.sqrt(4.0 * z * z - (1.0 + z * z - p * p) ** 2)) / math.pi


def occulted_fraction(p: float, z: float, g1: float, g2: float) -> float:
    """1 - F for the quadratic law (Mandel & Agol 2002, eq. 8 and Table 1)."""
    if z >= 1.0 + p:
        return 0.0
    c2 = g1 + 2.0 * g2
    c4 = -g2
    c0 = 1.0 - g1 - g2  # = 1 - c2 - c4
    omega = c0 / 4.0 + c2 / 6.0 + c4 / 8.0
    a = (z - p) ** 2
    b = (z + p) ** 2
    q = p * p - z * z
    lam_e = _lambda_e(p, z)
    if z > 1.0 - p:  # partial overlap (p < 1/2)
        k = math.sqrt((1.0 - a) / (4.0 * z * p))
        lam_d = (1.0 / (9.0 * math.pi * math.sqrt(p * z))) * (
            ((1.0 - b) * (2.0 * b + a - 3.0) - 3.0 * q * (b - 2.0)) * _K(k)
            + 4.0 * p * z * (z * z + 7.0 * p * p - 4.0) * _E(k)
            - 3.0 * (q / a) * _Pi((a - 1.0) / a, k))
        k1 = math.acos((1.0 - p * p + z * z) / (2.0 * z))
        k0 = math.acos((p * p + z * z - 1.0) / (2.0 * p * z))
        eta_d = (1.0 / (2.0 * math.pi)) * (
            k1 + 2.0 * (p * p / 2.0) * (p * p + 2.0 * z * z) * k0
            - 0.25 * (1.0 + 5.0 * p * p + z * z) * math.sqrt((1.0 - a) * (b - 1.0)))
        theta = 0.0
    else:  # planet disk entirely on the star
        kinv = math.sqrt(4.0 * z * p / (1.0 - a))
        lam_d = (2.0 / (9.0 * math.pi * math.sqrt(1.0 - a))) * (
            (1.0 - 5.0 * z * z + p * p + q * q) * _K(kinv)
            + (1.0 - a) * (z * z + 7.0 * p * p - 4.0) * _E(kinv)
            - 3.0 * (q / a) * _Pi((a - b) / a, kinv))
        eta_d = (p * p / 2.0) * (p * p + 2.0 * z * z)
        theta = 1.0 if p > z else 0.0
    num = (1.0 - c2) * lam_e + c2 * (lam_d + (2.0 / 3.0) * theta) - c4 * eta_d
    return num / (4.0 * omega)
