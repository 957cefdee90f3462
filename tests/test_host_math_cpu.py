"""CPU checks of the kernels' own per-sample arithmetic, built for the host
from the same source (tests/host/gl_host_check.cpp includes gl_device.h; the
host build takes IEEE division and square root where the device takes the
hardware estimates, everything else is shared with the kernels).

* the own sine/cosine, arctangent and angle reduction against the C library;
* instantaneous fluxes of the host build against the oracle, at the exact
  path's bar (1e-9), on hard shapes and grazing geometries and on MCMC-walker
  draws around the transit.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2410_05408_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIP_INC = "/opt/rocm/include"


@pytest.fixture(scope="session")
def host_check(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.exists(os.path.join(HIP_INC, "hip", "hip_runtime.h")):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("host") / "gl_host_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", HIP_INC,
                    "-I", os.path.join(ROOT, "paper_2410_05408_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host", "gl_host_check.cpp"), "-o", exe], check=True)
    return exe


def host_flux(exe, tmp_path, params, times, unconverged=None):
    """Instantaneous fluxes of the host build; with a list `unconverged`,
    appends the number of arcs accepted unconverged at the last level."""
    pf, tf, of = (str(tmp_path / n) for n in ("p.bin", "t.bin", "o.bin"))
    np.ascontiguousarray(params, dtype=np.float64).tofile(pf)
    np.ascontiguousarray(times, dtype=np.float64).tofile(tf)
    r = subprocess.run([exe, "flux", pf, tf, of], check=True, capture_output=True, text=True)
    if unconverged is not None:
        unconverged.append(int(r.stdout.split()[0]))
    return np.fromfile(of)


def oracle_flux(oracle, params, times):
    n = times.size
    return oracle.flux_batch(params, times, offsets=np.arange(n + 1), n_ss=np.ones(n, np.int32),
                             t_exp=np.zeros(n))


def test_own_trigonometry_against_libm(host_check):
    out = subprocess.run([host_check, "math"], check=True, capture_output=True, text=True).stdout.split()
    es, ec, ea, ew, rw = (float(v) for v in out)
    assert es <= 4.5e-16 and ec <= 4.5e-16      # sincos_pi on [-pi, pi]
    assert ea <= 9e-16                           # atan2_d, including the axes and the origin
    assert ew <= 2e-14 and rw <= math.pi + 1e-15  # angle reduction for |a| <= 40 pi


def test_host_flux_matches_oracle_on_hard_shapes(host_check, oracle, tmp_path):
    w = W.adversarial_batch(60)
    rng = np.random.default_rng(5)
    cols, ts = [], []
    for s in range(w.n_sets):
        a, b = int(w.offsets[s]), int(w.offsets[s + 1])
        pick = rng.choice(np.arange(a, b), size=min(24, b - a), replace=False)
        cols += [s] * pick.size
        ts.append(w.times[pick])
    params = w.params[:, cols]
    times = np.concatenate(ts)
    unconv = []
    got = host_flux(host_check, tmp_path, params, times, unconv)
    ref = oracle_flux(oracle, params, times)
    assert np.all(np.isfinite(got))
    assert np.sum(got < 1.0) > times.size // 3   # most samples occult something
    assert np.max(np.abs(got - ref)) <= 1e-9
    print(f"unconverged arcs on {times.size} hard-shape samples: {unconv[0]}")


def test_host_flux_matches_oracle_on_walker_draws(host_check, oracle, tmp_path):
    rng = np.random.default_rng(11)
    n = 3000
    params = W.draw_params(rng, n)
    t14 = W.full_duration(params[W.K], params[W.B], params[W.ARS], params[W.P])
    times = rng.uniform(-0.6, 0.6, n) * t14
    unconv = []
    got = host_flux(host_check, tmp_path, params, times, unconv)
    ref = oracle_flux(oracle, params, times)
    assert np.sum(got < 1.0) > n // 2
    assert np.max(np.abs(got - ref)) <= 1e-9
    assert unconv[0] == 0


def host_snap(exe, tmp_path, params, times, nodes):
    pf, tf, of = (str(tmp_path / n) for n in ("ps.bin", "ts.bin", "os.bin"))
    np.ascontiguousarray(params, dtype=np.float64).tofile(pf)
    np.ascontiguousarray(times, dtype=np.float64).tofile(tf)
    subprocess.run([exe, "snap", str(nodes), pf, tf, of], check=True)
    return np.fromfile(of)


def test_paper_integrator_against_oracle(host_check, oracle, tmp_path):
    """The paper's FP32 snap + Simpson integrator (host build of the kernel's
    routine): samples whose ellipse lies inside the disk are at
    single-precision noise at any node count; partially overlapping samples
    converge to the oracle as the node count grows (about as 1/n: the
    quadratic integrand jumps where the curve is moved onto the limb)."""
    rng = np.random.default_rng(11)
    n = 2000
    params = W.draw_params(rng, n)
    t14 = W.full_duration(params[W.K], params[W.B], params[W.ARS], params[W.P])
    times = rng.uniform(-0.6, 0.6, n) * t14
    ref = oracle_flux(oracle, params, times)
    geo = [oracle.geometry(params[:, i], times[i]) for i in range(n)]
    rho = np.array([math.hypot(g[1][0], g[1][1]) if g[0] else 9.0 for g in geo])
    k = params[W.K]
    inside, partial = rho <= 1 - k, (rho > 1 - k) & (rho < 1 + k)
    errs = {}
    for nodes in (256, 1024, 8192):
        err = np.abs(host_snap(host_check, tmp_path, params, times, nodes) - ref)
        errs[nodes] = err[partial].max()
        assert err[inside].max() <= 3e-7, nodes
        assert np.all(err[~inside & ~partial] == 0.0)  # centre beyond 1 + k: exactly 1
    assert errs[256] > errs[1024] > errs[8192]
    assert errs[8192] <= 4e-6 and errs[1024] <= 3e-5


def host_ell(exe, tmp_path, params, times):
    pf, tf, of = (str(tmp_path / n) for n in ("pe.bin", "te.bin", "oe.bin"))
    np.ascontiguousarray(params, dtype=np.float64).tofile(pf)
    np.ascontiguousarray(times, dtype=np.float64).tofile(tf)
    r = subprocess.run([exe, "ell", pf, tf, of], check=True, capture_output=True, text=True)
    return np.fromfile(of), int(r.stdout.split()[0])


@pytest.mark.parametrize("locked", [False, True])
def test_host_ellipsoid_matches_oracle(host_check, oracle, tmp_path, locked):
    """General ellipsoids, free and tidally locked: the device arithmetic (the
    paper's eqs. dx, dy1, dy2 and their locked forms, per sample when locked)
    against the oracle's quadric shadow, instantaneous flux within 1e-9."""
    rng = np.random.default_rng(31 + locked)
    n = 2000
    params = W.draw_ellipsoids(rng, n, locked)
    kmax = params[W.E_RA:W.E_RC + 1].max(axis=0)
    t14 = W.full_duration(kmax, params[W.E_B], params[W.E_ARS], params[W.E_P])
    times = rng.uniform(-0.6, 0.6, n) * t14
    got, unconv = host_ell(host_check, tmp_path, params, times)
    ref = oracle.flux_batch_ell(params, times, offsets=np.arange(n + 1))
    assert np.sum(got < 1.0) > n // 2
    assert np.max(np.abs(got - ref)) <= 1e-9
    assert unconv == 0


def host_guesses(exe, tmp_path, coeffs):
    qf, of = str(tmp_path / "q.bin"), str(tmp_path / "g.bin")
    np.ascontiguousarray(coeffs, dtype=np.float64).tofile(qf)
    subprocess.run([exe, "guesses", qf, of], check=True)
    return np.fromfile(of).reshape(-1, 5)


def _quartic(a4, b1, c1, b2, c2):
    """Coefficients a0..a4 of a4 (t^2 + b1 t + c1)(t^2 + b2 t + c2)."""
    return np.stack([a4 * c1 * c2, a4 * (b1 * c2 + b2 * c1), a4 * (c1 + c2 + b1 * b2), a4 * (b1 + b2), a4], axis=1)


def test_quartic_first_iterates(host_check, tmp_path):
    """The closed-form first iterates of the quartic solver (host build of the
    same source): Ferrari's guesses land on both real roots of a quartic with
    two real roots and a complex pair, and are all NaN when it has none or
    four; Cardano's root of q' is its real root when it has one and NaN when
    it has three.  The roots come from the construction and from numpy."""
    rng = np.random.default_rng(17)
    n = 4000
    a4 = rng.choice([-1.0, 1.0], n) * rng.uniform(0.1, 1.0, n)
    r = np.sort(rng.uniform(-1.8, 1.8, (n, 2)), axis=1)
    r[:, 1] = np.maximum(r[:, 1], r[:, 0] + 1e-2)
    p = rng.uniform(-1.0, 1.0, n)
    s = 0.25 * p * p + rng.uniform(0.05, 2.0, n)            # t^2 + p t + s has no real root
    two = _quartic(a4, -(r[:, 0] + r[:, 1]), r[:, 0] * r[:, 1], p, s)
    g = host_guesses(host_check, tmp_path, two)
    fin = np.isfinite(g[:, 1:])
    assert np.all(fin.sum(axis=1) == 2)
    for k in (0, 1):
        d = np.where(fin, np.abs(g[:, 1:] - r[:, k:k + 1]), np.inf).min(axis=1) / np.maximum(1.0, np.abs(r[:, k]))
        assert d.max() <= 1e-5, d.max()
    # no real root, and four: every guess NaN
    p2 = rng.uniform(-1.0, 1.0, n)
    s2 = 0.25 * p2 * p2 + rng.uniform(0.05, 2.0, n)
    none = _quartic(a4, p, s, p2, s2)
    r4 = np.sort(rng.uniform(-1.8, 1.8, (n, 4)), axis=1)
    r4 += np.arange(4) * 0.05                                # distinct roots
    four = _quartic(a4, -(r4[:, 0] + r4[:, 1]), r4[:, 0] * r4[:, 1], -(r4[:, 2] + r4[:, 3]), r4[:, 2] * r4[:, 3])
    for q in (none, four):
        assert np.all(np.isnan(host_guesses(host_check, tmp_path, q)[:, 1:]))
    # the real root of q' = 4 a4 t^3 + 3 a3 t^2 + 2 a2 t + a1
    for q, gq in ((two, g), (none, host_guesses(host_check, tmp_path, none))):
        for i in range(n):
            cr = np.roots([4 * q[i, 4], 3 * q[i, 3], 2 * q[i, 2], q[i, 1]])
            im = np.abs(cr.imag)
            if np.all(im < 1e-7):
                gap = np.min(np.diff(np.sort(cr.real)))
                if gap > 1e-3:
                    assert np.isnan(gq[i, 0]), (i, cr, gq[i, 0])
            elif np.sum(im < 1e-12) == 1 and np.min(im[im >= 1e-12]) > 1e-3:
                x = cr.real[np.argmin(im)]
                assert abs(gq[i, 0] - x) <= 1e-5 * max(1.0, abs(x)), (i, x, gq[i, 0])
