"""ctypes wrapper of the CPU FP64 oracle (``oracle/libglo.so``).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg; never by the GPU package.  It shares no code with
the HIP library.  See ``glo.c`` for the method and for the readings of the
paper (arXiv:2410.05408, Section 2) that it rests on.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libglo.so")

K, F, THETA, PHI, B, ARS, P, T0, Q1, Q2 = range(10)
NPARAM = 10
# general ellipsoids
E_RA, E_RB, E_RC, E_ZETA, E_ETA, E_XI, E_B, E_ARS, E_P, E_T0, E_Q1, E_Q2, E_LOCKED = range(13)
E_NPARAM = 13
INNER_CLOSED, INNER_ADAPTIVE = 0, 1
DEFAULT_TOL = 1e-14


def build(verbose: bool = False) -> str:
    """Compile ``libglo.so`` with gcc (FP contraction off, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           os.path.join(_HERE, "glo.c"), "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        d, i, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.glo_kipping.argtypes = [d, d, dp, dp]
        L.glo_kipping.restype = i
        L.glo_geometry.argtypes = [dp, d, dp]
        L.glo_geometry.restype = i
        L.glo_occulted.argtypes = [d, d, d, d, d, d, d, d, d, i]
        L.glo_occulted.restype = d
        L.glo_flux.argtypes = [dp, d, d, i, d, dp]
        L.glo_flux.restype = i
        L.glo_geometry_ell.argtypes = [dp, d, dp]
        L.glo_geometry_ell.restype = i
        L.glo_flux_batch_ell.argtypes = [dp, i64, dp, i64p, i64, i32p, dp, d, dp, i]
        L.glo_flux_batch_ell.restype = i64
        L.glo_flux_batch.argtypes = [dp, i64, dp, i64p, i64, i32p, dp, d, dp, i]
        L.glo_flux_batch.restype = i64
        L.glo_flux_select.argtypes = [dp, i64, dp, i64p, i64, i32p, dp, d,
                                      i64p, i64, dp, i]
        L.glo_flux_select.restype = i64
        L.glo_unconverged.argtypes = []
        L.glo_unconverged.restype = ctypes.c_long
        L.glo_max_threads.argtypes = []
        L.glo_max_threads.restype = i
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def kipping(q1: float, q2: float):
    u1, u2 = ctypes.c_double(), ctypes.c_double()
    rc = lib().glo_kipping(q1, q2, ctypes.byref(u1), ctypes.byref(u2))
    if rc:
        raise ValueError("q1, q2 outside [0, 1]")
    return u1.value, u2.value


def geometry(p, t: float):
    """Returns (in_front, centre(x0,y0), z, u_hat, s_hat, k, kq)."""
    pa = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(9)
    front = lib().glo_geometry(_dp(pa), float(t), _dp(out))
    return bool(front), out[0:2].copy(), out[2], out[3:5].copy(), out[5:7].copy(), out[7], out[8]


def occulted(cx, cy, ux, uy, k, q, u1, u2, tol=DEFAULT_TOL, mode=INNER_CLOSED):
    return lib().glo_occulted(float(cx), float(cy), float(ux), float(uy), float(k),
                              float(q), float(u1), float(u2), float(tol), int(mode))


def flux(p, t, t_exp=0.0, n_ss=1, tol=DEFAULT_TOL):
    pa = np.ascontiguousarray(p, dtype=np.float64)
    out = ctypes.c_double()
    rc = lib().glo_flux(_dp(pa), float(t), float(t_exp), int(n_ss), float(tol),
                        ctypes.byref(out))
    return out.value if rc == 0 else float("nan")


def _prep(params, times, offsets, n_ss, t_exp):
    params = np.ascontiguousarray(params, dtype=np.float64)
    assert params.ndim == 2 and params.shape[0] == NPARAM
    n_sets = params.shape[1]
    times = np.ascontiguousarray(times, dtype=np.float64)
    off_p = None
    if offsets is not None:
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        assert offsets.shape == (n_sets + 1,)
        off_p = offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    nss_p = None
    if n_ss is not None:
        n_ss = np.ascontiguousarray(np.broadcast_to(n_ss, (n_sets,)), dtype=np.int32)
        nss_p = n_ss.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    te_p = None
    if t_exp is not None:
        t_exp = np.ascontiguousarray(np.broadcast_to(t_exp, (n_sets,)), dtype=np.float64)
        te_p = _dp(t_exp)
    keep = (params, times, offsets, n_ss, t_exp)
    return keep, n_sets, off_p, nss_p, te_p


def flux_batch(params, times, offsets=None, n_ss=None, t_exp=None,
               tol=DEFAULT_TOL, nthreads=0):
    """Oracle over a whole batch in the GPU ABI's layout."""
    keep, n_sets, off_p, nss_p, te_p = _prep(params, times, offsets, n_ss, t_exp)
    times = keep[1]
    n_times = times.shape[0] if offsets is None else 0
    n_out = n_sets * n_times if offsets is None else int(keep[2][-1])
    out = np.empty(n_out)
    lib().glo_flux_batch(_dp(keep[0]), n_sets, _dp(times), off_p, n_times, nss_p,
                         te_p, float(tol), _dp(out), int(nthreads))
    return out if offsets is not None else out.reshape(n_sets, n_times)


def flux_select(params, times, sel, offsets=None, n_ss=None, t_exp=None,
                tol=DEFAULT_TOL, nthreads=0):
    """Oracle at selected flat output indices (shared grid: s*n_times + i)."""
    keep, n_sets, off_p, nss_p, te_p = _prep(params, times, offsets, n_ss, t_exp)
    times = keep[1]
    n_times = times.shape[0] if offsets is None else 0
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    out = np.empty(sel.shape[0])
    lib().glo_flux_select(_dp(keep[0]), n_sets, _dp(times), off_p, n_times, nss_p,
                          te_p, float(tol),
                          sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          sel.shape[0], _dp(out), int(nthreads))
    return out


def unconverged() -> int:
    """Adaptive integrals that stopped above their error target so far."""
    return int(lib().glo_unconverged())


def max_threads() -> int:
    return lib().glo_max_threads()


def geometry_ell(p, t: float):
    """(front, centre (x, y, z), u_hat (major axis), s_hat (minor), k_major, k_minor)."""
    out = np.zeros(9)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    front = lib().glo_geometry_ell(_dp(pp), float(t), _dp(out))
    return bool(front), out[0:3].copy(), out[3:5].copy(), out[5:7].copy(), out[7], out[8]


def flux_batch_ell(params, times, offsets=None, n_ss=None, t_exp=None, tol=DEFAULT_TOL, nthreads=0):
    """Oracle over a batch of general ellipsoids (params [E_NPARAM, n_sets])."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    assert params.shape[0] == E_NPARAM
    n_sets = params.shape[1]
    times = np.ascontiguousarray(times, dtype=np.float64)
    off = None if offsets is None else np.ascontiguousarray(offsets, dtype=np.int64)
    nss = None if n_ss is None else np.ascontiguousarray(n_ss, dtype=np.int32)
    te = None if t_exp is None else np.ascontiguousarray(t_exp, dtype=np.float64)
    n_out = n_sets * times.size if off is None else int(off[-1])
    out = np.empty(n_out)
    lib().glo_flux_batch_ell(_dp(params), n_sets, _dp(times),
                             None if off is None else off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             times.size if off is None else 0,
                             None if nss is None else nss.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             None if te is None else _dp(te), float(tol), _dp(out), int(nthreads))
    return out if off is not None else out.reshape(n_sets, times.size)
