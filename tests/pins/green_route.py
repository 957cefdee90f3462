"""A second, independent route to the occulted flux: the paper's own boundary
form, evaluated with scipy.

Geometry: the paper's parametric projected ellipse (Section 2, eqs. dx, dy1,
dy2), built from its rotation matrices R = Rx(zeta) Ry(eta) Rz(xi) with the
oblate axes a = k(1-f) (polar, body x'), b = c = k, zeta = 0, eta = pi/2 - theta,
xi = phi; orbit centre x0 = d cos(alpha) sin(beta), y0 = d sin(alpha).

Integral: Green's theorem with the three integrands the paper lists (f_flat,
f_lin, f_quad), integrated with scipy's adaptive quadrature along the ellipse
arcs that lie on the star, and in closed form along the stellar limb arcs that
close the region.  Intersections are bracketed on a dense sampling of
|p(theta)|^2 - 1 and polished with Brent's method.  Unlike the paper, no
snapping: exact arcs.  Independent of the oracle (an area integral) and of the
GPU code.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad
from scipy.optimize import brentq


def rx(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=float)


def ry(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=float)


def rz(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=float)


def paper_deltas(k, f, theta, phi):
    """(dx, dy1, dy2) of eqs. dx, dy1, dy2 for the oblate spheroid."""
    a, b, c = k * (1.0 - f), k, k
    R = rx(0.0) @ ry(0.5 * math.pi - theta) @ rz(phi)
    r1, r2, r3, r4, r5, r6, r7, r8, r9 = R.ravel()
    dx = math.sqrt(a * a * r1 * r1 + b * b * r4 * r4 + c * c * r7 * r7)
    dy1 = (a * a * r1 * r2 + b * b * r4 * r5 + c * c * r7 * r8) / dx
    dy2 = math.sqrt(a * a * b * b * r9 * r9 + a * a * c * c * r6 * r6 + b * b * c * c * r3 * r3) / dx
    return dx, dy1, dy2


def paper_deltas_ell(a, b, c, zeta, eta, xi):
    """(dx, dy1, dy2) of eqs. dx, dy1, dy2 for a triaxial ellipsoid with
    semi-axes a, b, c along x', y', z' and R = Rx(zeta) Ry(eta) Rz(xi)."""
    R = rx(zeta) @ ry(eta) @ rz(xi)
    r1, r2, r3, r4, r5, r6, r7, r8, r9 = R.ravel()
    dx = math.sqrt(a * a * r1 * r1 + b * b * r4 * r4 + c * c * r7 * r7)
    dy1 = (a * a * r1 * r2 + b * b * r4 * r5 + c * c * r7 * r8) / dx
    dy2 = math.sqrt(a * a * b * b * r9 * r9 + a * a * c * c * r6 * r6 + b * b * c * c * r3 * r3) / dx
    return dx, dy1, dy2


def paper_deltas_locked(a, b, c, zeta, eta, xi, alpha, beta):
    """(dx, dy1, dy2) of the tidally-locked eqs. dx-locked, dy1-locked and
    dy2-locked (Appendix B), term by term as printed."""
    R = rx(zeta) @ ry(eta) @ rz(xi)
    r1, r2, r3, r4, r5, r6, r7, r8, r9 = R.ravel()
    sa, ca, sb, cb = math.sin(alpha), math.cos(alpha), math.sin(beta), math.cos(beta)
    p1 = sb * (r3 * ca + r2 * sa) - r1 * cb
    p2 = sb * (r6 * ca + r5 * sa) - r4 * cb
    p3 = sb * (r9 * ca + r8 * sa) - r7 * cb
    dx = math.sqrt(a * a * p1 * p1 + b * b * p2 * p2 + c * c * p3 * p3)
    dy1 = (a * a * p1 * (r3 * sa - r2 * ca) + b * b * p2 * (r6 * sa - r5 * ca)
           + c * c * p3 * (r9 * sa - r8 * ca)) / dx
    w1 = r7 * sb + cb * (r9 * ca + r8 * sa)
    w2 = r4 * sb + cb * (r6 * ca + r5 * sa)
    w3 = r1 * sb + cb * (r3 * ca + r2 * sa)
    dy2 = math.sqrt(a * a * b * b * w1 * w1 + a * a * c * c * w2 * w2 + b * b * c * c * w3 * w3) / dx
    return dx, dy1, dy2


def paper_centre(b, d, period, t0, t):
    """(x0, y0) and the line-of-sight coordinate of the planet centre."""
    alpha = 2.0 * math.pi * (t - t0) / period
    beta = math.asin(b / d)
    return (d * math.cos(alpha) * math.sin(beta), d * math.sin(alpha),
            -d * math.cos(beta) * math.cos(alpha))


def kipping(q1, q2):
    s = math.sqrt(q1)
    return 2.0 * s * q2, s * (1.0 - 2.0 * q2)


class Ellipse:
    def __init__(self, x0, y0, A, B, C):
        self.x0, self.y0, self.A, self.B, self.C = x0, y0, A, B, C

    def point(self, th):
        return (self.x0 + self.A * np.cos(th),
                self.y0 + self.B * np.cos(th) + self.C * np.sin(th))

    def deriv(self, th):
        return -self.A * np.sin(th), -self.B * np.sin(th) + self.C * np.cos(th)

    def g(self, th):
        x, y = self.point(th)
        return x * x + y * y - 1.0

    # the paper's three integrands, per unit theta
    def f_flat(self, th):
        x, y = self.point(th)
        dx, dy = self.deriv(th)
        return 0.5 * (x * dy - y * dx)

    def f_lin(self, th):
        x, y = self.point(th)
        r2 = x * x + y * y
        m = max(0.0, 1.0 - r2)
        return (2.0 / 3.0) * (1.0 - m ** 1.5) * self.f_flat(th) / r2

    def f_quad(self, th):
        x, y = self.point(th)
        dx, dy = self.deriv(th)
        return 0.5 * (x * (x * x / 3.0 + y * y) * dy - y * (x * x + y * y / 3.0) * dx)

    def roots(self, n=20000):
        th = np.linspace(0.0, 2.0 * math.pi, n + 1)
        gv = self.g(th)
        out = []
        for i in range(n):
            if gv[i] == 0.0:
                out.append(th[i])
            elif gv[i] * gv[i + 1] < 0.0:
                out.append(brentq(self.g, th[i], th[i + 1], xtol=1e-16, rtol=8.9e-16, maxiter=200))
        return sorted(out)


def _arc(fn, a, b):
    v, _ = quad(fn, a, b, epsabs=1e-15, epsrel=1e-14, limit=400)
    return v


def limb_terms(lam_a, lam_b):
    """Closed forms of the three integrands along the unit circle, CCW from
    lam_a to lam_b: (dl/2, dl/3, dl/4 - (sin 4lb - sin 4la)/48)."""
    dl = (lam_b - lam_a) % (2.0 * math.pi)
    return (dl / 2.0, dl / 3.0,
            dl / 4.0 - (math.sin(4.0 * (lam_a + dl)) - math.sin(4.0 * lam_a)) / 48.0)


def green_integrals(E: Ellipse):
    """(S_flat, S_lin, S_quad) = integrals of 1, mu, r^2 over E cap D."""
    rts = E.roots()
    if len(rts) == 0:
        if E.g(0.0) < 0.0:  # whole ellipse on the star
            return (_arc(E.f_flat, 0.0, 2 * math.pi), _arc(E.f_lin, 0.0, 2 * math.pi),
                    _arc(E.f_quad, 0.0, 2 * math.pi))
        return 0.0, 0.0, 0.0
    S = np.zeros(3)
    n = len(rts)
    arcs = []
    for i in range(n):
        a = rts[i]
        b = rts[(i + 1) % n] + (2.0 * math.pi if i == n - 1 else 0.0)
        if E.g(0.5 * (a + b)) < 0.0:
            arcs.append((a, b))
    for (a, b) in arcs:
        S += [_arc(E.f_flat, a, b), _arc(E.f_lin, a, b), _arc(E.f_quad, a, b)]
    # limb arcs: from the end of each inside ellipse arc to the start of the next
    for i, (a, b) in enumerate(arcs):
        nxt = arcs[(i + 1) % len(arcs)][0]
        xe, ye = E.point(b)
        xs, ys = E.point(nxt)
        S += limb_terms(math.atan2(ye, xe), math.atan2(ys, xs))
    return tuple(S)


def occulted(E: Ellipse, u1, u2):
    c0, c1, c2 = 1.0 - u1 - 2.0 * u2, u1 + 2.0 * u2, u2
    sf, sl, sq = green_integrals(E)
    phi_norm = math.pi * (1.0 - u1 / 3.0 - u2 / 6.0)
    return (c0 * sf + c1 * sl + c2 * sq) / phi_norm


def lens_area(E: Ellipse):
    """Area of E cap D in closed form: Green's f_flat integrated exactly on
    each ellipse arc, (A C dth + x0 C dsin - (y0 A - x0 B) dcos)/2, plus dl/2
    on each limb arc."""
    rts = E.roots()
    A, B, C, x0, y0 = E.A, E.B, E.C, E.x0, E.y0

    def flat(a, b):
        return 0.5 * (A * C * (b - a) + x0 * C * (math.sin(b) - math.sin(a))
                      - (y0 * A - x0 * B) * (math.cos(b) - math.cos(a)))

    if not rts:
        return math.pi * A * C if E.g(0.0) < 0.0 else 0.0
    n = len(rts)
    arcs = []
    for i in range(n):
        a = rts[i]
        b = rts[(i + 1) % n] + (2.0 * math.pi if i == n - 1 else 0.0)
        if E.g(0.5 * (a + b)) < 0.0:
            arcs.append((a, b))
    area = sum(flat(a, b) for a, b in arcs)
    for i, (a, b) in enumerate(arcs):
        nxt = arcs[(i + 1) % len(arcs)][0]
        xe, ye = E.point(b)
        xs, ys = E.point(nxt)
        area += limb_terms(math.atan2(ye, xe), math.atan2(ys, xs))[0]
    return area


def flux(p, t, tol_unused=None):
    """Instantaneous relative flux for a parameter block p (library layout)."""
    k, f, theta, phi, b, d, period, t0, q1, q2 = [float(v) for v in p]
    x0, y0, z = paper_centre(b, d, period, t0, t)
    if z >= 0.0 or x0 * x0 + y0 * y0 >= (1.0 + k) ** 2:
        return 1.0
    A, B, C = paper_deltas(k, f, theta, phi)
    u1, u2 = kipping(q1, q2)
    return 1.0 - occulted(Ellipse(x0, y0, A, B, C), u1, u2)
