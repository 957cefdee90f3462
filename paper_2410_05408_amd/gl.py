"""Python binding of the C ABI in ``include/gl.h`` (``libgl_hip.so``).

Argument marshalling only: every step of the light-curve computation runs in
the library's HIP kernels.  Tensors are PyTorch CUDA (ROCm) tensors; PyTorch
provides device memory and streams.  There is no CPU fallback: loading fails
loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GL_LIB", os.path.join(_PKG, "libgl_hip.so"))

GL_OK, GL_ERR_NULL, GL_ERR_SIZE, GL_ERR_DOMAIN = 0, -1, -2, -3
GL_ERR_DEVICE, GL_ERR_STATE, GL_ERR_NOMEM = -4, -5, -6
STATUS_NAMES = {0: "GL_OK", -1: "GL_ERR_NULL", -2: "GL_ERR_SIZE", -3: "GL_ERR_DOMAIN",
                -4: "GL_ERR_DEVICE", -5: "GL_ERR_STATE", -6: "GL_ERR_NOMEM"}
GL_K, GL_F, GL_THETA, GL_PHI, GL_B, GL_ARS, GL_P, GL_T0, GL_Q1, GL_Q2 = range(10)
GL_NPARAM = 10
(GL_E_RA, GL_E_RB, GL_E_RC, GL_E_ZETA, GL_E_ETA, GL_E_XI, GL_E_B, GL_E_ARS, GL_E_P, GL_E_T0, GL_E_Q1,
 GL_E_Q2, GL_E_LOCKED) = range(13)
GL_E_NPARAM = 13
GL_W_R, GL_W_MU, GL_W_NU, GL_W_XI, GL_W_B, GL_W_ARS, GL_W_P, GL_W_T0, GL_W_Q1, GL_W_Q2 = range(10)
GL_W_NPARAM = 10

EXPORTED = ("gl_ctx_create", "gl_ctx_destroy", "gl_lightcurve_batch", "gl_ctx_sync_status",
            "gl_ctx_last_error", "gl_autotune", "gl_ctx_get_plan", "gl_ctx_set_plan",
            "gl_ctx_set_graph", "gl_ctx_set_capacity", "gl_ctx_set_timing", "gl_ctx_get_timing",
            "gl_ctx_get_stage_timing", "gl_census", "gl_flop_model", "gl_ctx_get_unconverged",
            "gl_ctx_get_overflow", "gl_lightcurve_batch_noalloc", "gl_lightcurve_batch_snap", "gl_version",
            "gl_lightcurve_batch_ellipsoid", "gl_autotune_ellipsoid", "gl_prior_mu_nu", "gl_walkers_to_params",
            "gl_loglike_of_model", "gl_loglike_batch", "gl_ctx_get_stage_plan", "gl_ctx_set_stage_plan")
CENSUS_NAMES = ("sub_in_window", "whole_on_star", "intersecting", "off_star_in_window",
                "trapezoid_nodes", "gk21_pieces", "newton_steps", "limb_arcs",
                "nested_trapezoid_nodes", "ellipse_arcs", "unconverged_arcs")
GL_NSTAGES = 9
STAGE_NAMES = ("setup", "window", "classify", "trapezoid", "hard", "arcs", "nested", "combine", "fused")


class GLError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Loads libgl_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2410_05408_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.gl_ctx_create.argtypes = [ctypes.POINTER(vp), i]
        L.gl_ctx_create.restype = i
        L.gl_ctx_destroy.argtypes = [vp]
        L.gl_ctx_destroy.restype = None
        batch_args = [vp, vp, i64, vp, vp, i64, vp, vp, vp, vp]
        L.gl_lightcurve_batch.argtypes = batch_args
        L.gl_lightcurve_batch.restype = i
        L.gl_lightcurve_batch_ellipsoid.argtypes = batch_args
        L.gl_lightcurve_batch_ellipsoid.restype = i
        L.gl_autotune_ellipsoid.argtypes = batch_args
        L.gl_autotune_ellipsoid.restype = i
        L.gl_prior_mu_nu.argtypes = [vp, i64, vp, vp]
        L.gl_prior_mu_nu.restype = i
        L.gl_walkers_to_params.argtypes = [vp, i64, vp, vp]
        L.gl_walkers_to_params.restype = i
        L.gl_loglike_of_model.argtypes = [vp, i64, vp, i64, vp, vp, vp, vp, vp]
        L.gl_loglike_of_model.restype = i
        L.gl_loglike_batch.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.gl_loglike_batch.restype = i
        L.gl_lightcurve_batch_snap.argtypes = [vp, i] + batch_args[1:]
        L.gl_lightcurve_batch_snap.restype = i
        L.gl_lightcurve_batch_noalloc.argtypes = batch_args[1:]
        L.gl_lightcurve_batch_noalloc.restype = i
        L.gl_autotune.argtypes = batch_args
        L.gl_autotune.restype = i
        L.gl_ctx_sync_status.argtypes = [vp]
        L.gl_ctx_sync_status.restype = i
        L.gl_ctx_last_error.argtypes = [vp]
        L.gl_ctx_last_error.restype = ctypes.c_char_p
        L.gl_ctx_get_plan.argtypes = [vp, ctypes.POINTER(i)]
        L.gl_ctx_get_plan.restype = i
        L.gl_ctx_set_plan.argtypes = [vp, i]
        L.gl_ctx_set_plan.restype = i
        L.gl_ctx_get_stage_plan.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i),
                                            ctypes.POINTER(i)]
        L.gl_ctx_get_stage_plan.restype = i
        L.gl_ctx_set_stage_plan.argtypes = [vp, i, i, i, i]
        L.gl_ctx_set_stage_plan.restype = i
        L.gl_ctx_set_graph.argtypes = [vp, i]
        L.gl_ctx_set_graph.restype = i
        L.gl_ctx_set_timing.argtypes = [vp, i]
        L.gl_ctx_set_timing.restype = i
        dpp = ctypes.POINTER(ctypes.c_double)
        L.gl_ctx_get_timing.argtypes = [vp, dpp, dpp, ctypes.POINTER(i)]
        L.gl_ctx_get_timing.restype = i
        L.gl_ctx_get_stage_timing.argtypes = [vp, dpp, ctypes.POINTER(i)]
        L.gl_ctx_get_stage_timing.restype = i
        L.gl_ctx_set_capacity.argtypes = [vp, i64, i64, i64]
        L.gl_ctx_set_capacity.restype = i
        L.gl_census.argtypes = batch_args + [ctypes.POINTER(ctypes.c_int64)]
        L.gl_census.restype = i
        L.gl_flop_model.argtypes = [ctypes.POINTER(ctypes.c_int64)]
        L.gl_flop_model.restype = i
        L.gl_ctx_get_overflow.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i)]
        L.gl_ctx_get_overflow.restype = i
        L.gl_ctx_get_unconverged.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.gl_ctx_get_unconverged.restype = i
        L.gl_version.argtypes = []
        L.gl_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(ctx, st):
    if st != GL_OK:
        msg = lib().gl_ctx_last_error(ctx).decode() if ctx else ""
        raise GLError(st, msg)


# ---------------------------------------------------------------- C names
def gl_ctx_create(device: int = 0):
    h = ctypes.c_void_p()
    st = lib().gl_ctx_create(ctypes.byref(h), int(device))
    if st != GL_OK:
        raise GLError(st, "gl_ctx_create")
    return h


def gl_ctx_destroy(ctx) -> None:
    lib().gl_ctx_destroy(ctx)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _validate(params, times, offsets, n_ss, t_exp, out, rows=GL_NPARAM):
    import torch
    assert params.dtype == torch.float64 and params.is_cuda and params.is_contiguous()
    assert params.dim() == 2 and params.shape[0] == rows
    _validate_grid(params.shape[1], times, offsets, n_ss, t_exp, out)


def _validate_grid(n_sets, times, offsets, n_ss, t_exp, out):
    import torch
    assert times.dtype == torch.float64 and times.is_cuda and times.is_contiguous()
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    if offsets is None:
        assert out.numel() == n_sets * times.numel()
    else:
        assert offsets.dtype == torch.int64 and offsets.is_cuda and offsets.numel() == n_sets + 1
        assert out.numel() == times.numel()
    if n_ss is not None:
        assert n_ss.dtype == torch.int32 and n_ss.is_cuda and n_ss.numel() == n_sets
    if t_exp is not None:
        assert t_exp.dtype == torch.float64 and t_exp.is_cuda and t_exp.numel() == n_sets


def gl_lightcurve_batch(ctx, params, times, out, offsets=None, n_ss=None, t_exp=None,
                        stream=None) -> None:
    """Enqueues the light curves of ``params`` (float64 [10, n_sets]) at
    ``times`` into ``out`` on ``stream`` (default: current torch stream)."""
    _validate(params, times, offsets, n_ss, t_exp, out)
    st = lib().gl_lightcurve_batch(ctx, _ptr(params), params.shape[1], _ptr(times), _ptr(offsets),
                                   times.numel(), _ptr(n_ss), _ptr(t_exp), _ptr(out),
                                   _stream_handle(stream))
    _check(ctx, st)


def gl_lightcurve_batch_ellipsoid(ctx, params, times, out, offsets=None, n_ss=None, t_exp=None,
                                  stream=None) -> None:
    """General ellipsoids: ``params`` float64 [13, n_sets] (rows GL_E_*)."""
    _validate(params, times, offsets, n_ss, t_exp, out, rows=GL_E_NPARAM)
    st = lib().gl_lightcurve_batch_ellipsoid(ctx, _ptr(params), params.shape[1], _ptr(times), _ptr(offsets),
                                             times.numel(), _ptr(n_ss), _ptr(t_exp), _ptr(out),
                                             _stream_handle(stream))
    _check(ctx, st)


def _dev(t, dtype, rows=None, n=None):
    import torch
    assert t.dtype == dtype and t.is_cuda and t.is_contiguous()
    if rows is not None:
        assert t.dim() == 2 and t.shape[0] == rows
    if n is not None:
        assert t.numel() == n


def gl_prior_mu_nu(uw, mu_nu, stream=None) -> None:
    """(mu, nu) prior draws from the uniforms ``uw`` (float64 [2, n]) into
    ``mu_nu`` (float64 [2, n])."""
    import torch
    _dev(uw, torch.float64, rows=2)
    _dev(mu_nu, torch.float64, rows=2, n=uw.numel())
    st = lib().gl_prior_mu_nu(_ptr(uw), uw.shape[1], _ptr(mu_nu), _stream_handle(stream))
    if st != GL_OK:
        raise GLError(st, "gl_prior_mu_nu")


def gl_walkers_to_params(walkers, params, stream=None) -> None:
    """Walker block float64 [10, n] -> oblate parameter block float64 [10, n]."""
    import torch
    _dev(walkers, torch.float64, rows=GL_W_NPARAM)
    _dev(params, torch.float64, rows=GL_NPARAM, n=walkers.numel())
    st = lib().gl_walkers_to_params(_ptr(walkers), walkers.shape[1], _ptr(params), _stream_handle(stream))
    if st != GL_OK:
        raise GLError(st, "gl_walkers_to_params")


def gl_loglike_of_model(model, n_sets, data, sigma, chi2=None, loglike=None, offsets=None, stream=None) -> None:
    import torch
    _dev(model, torch.float64)
    _dev(data, torch.float64)
    _dev(sigma, torch.float64, n=data.numel())
    if offsets is None:
        assert model.numel() == n_sets * data.numel()
    else:
        _dev(offsets, torch.int64, n=n_sets + 1)
        assert model.numel() == data.numel()
    for t in (chi2, loglike):
        if t is not None:
            _dev(t, torch.float64, n=n_sets)
    st = lib().gl_loglike_of_model(_ptr(model), n_sets, _ptr(offsets), data.numel(), _ptr(data), _ptr(sigma),
                                   _ptr(chi2), _ptr(loglike), _stream_handle(stream))
    if st != GL_OK:
        raise GLError(st, "gl_loglike_of_model")


def gl_loglike_batch(ctx, walkers, times, data, sigma, model, chi2=None, loglike=None, offsets=None,
                     n_ss=None, t_exp=None, stream=None) -> None:
    """One likelihood evaluation of a batch of walkers (float64 [10, n])."""
    import torch
    _dev(walkers, torch.float64, rows=GL_W_NPARAM)
    n = walkers.shape[1]
    _validate_grid(n, times, offsets, n_ss, t_exp, model)
    _dev(data, torch.float64, n=times.numel())
    _dev(sigma, torch.float64, n=times.numel())
    for t in (chi2, loglike):
        if t is not None:
            _dev(t, torch.float64, n=n)
    st = lib().gl_loglike_batch(ctx, _ptr(walkers), n, _ptr(times), _ptr(offsets), times.numel(), _ptr(n_ss),
                                _ptr(t_exp), _ptr(data), _ptr(sigma), _ptr(model), _ptr(chi2), _ptr(loglike),
                                _stream_handle(stream))
    _check(ctx, st)


def gl_lightcurve_batch_noalloc(params, times, out, offsets=None, n_ss=None, t_exp=None,
                                stream=None) -> None:
    """The allocation-free batch (no context; the library's own device array
    holds the workspace) on the current device; raises GLError on a status."""
    _validate(params, times, offsets, n_ss, t_exp, out)
    st = lib().gl_lightcurve_batch_noalloc(_ptr(params), params.shape[1], _ptr(times), _ptr(offsets),
                                           times.numel(), _ptr(n_ss), _ptr(t_exp), _ptr(out),
                                           _stream_handle(stream))
    if st != GL_OK:
        raise GLError(st, "gl_lightcurve_batch_noalloc")


def gl_lightcurve_batch_snap(ctx, n_nodes, params, times, out, offsets=None, n_ss=None, t_exp=None,
                             stream=None) -> None:
    """The paper's FP32 snap + Simpson integrator over a batch (n_nodes nodes)."""
    _validate(params, times, offsets, n_ss, t_exp, out)
    st = lib().gl_lightcurve_batch_snap(ctx, int(n_nodes), _ptr(params), params.shape[1], _ptr(times),
                                        _ptr(offsets), times.numel(), _ptr(n_ss), _ptr(t_exp), _ptr(out),
                                        _stream_handle(stream))
    _check(ctx, st)


def gl_autotune(ctx, params, times, out, offsets=None, n_ss=None, t_exp=None, stream=None) -> None:
    _validate(params, times, offsets, n_ss, t_exp, out)
    st = lib().gl_autotune(ctx, _ptr(params), params.shape[1], _ptr(times), _ptr(offsets),
                           times.numel(), _ptr(n_ss), _ptr(t_exp), _ptr(out),
                           _stream_handle(stream))
    _check(ctx, st)


def gl_autotune_ellipsoid(ctx, params, times, out, offsets=None, n_ss=None, t_exp=None, stream=None) -> None:
    """gl_autotune on a general-ellipsoid batch (``params`` float64 [13, n_sets])."""
    _validate(params, times, offsets, n_ss, t_exp, out, rows=GL_E_NPARAM)
    st = lib().gl_autotune_ellipsoid(ctx, _ptr(params), params.shape[1], _ptr(times), _ptr(offsets),
                                     times.numel(), _ptr(n_ss), _ptr(t_exp), _ptr(out),
                                     _stream_handle(stream))
    _check(ctx, st)


def gl_ctx_sync_status(ctx) -> int:
    """Returns GL_OK or GL_ERR_DOMAIN (and clears the device flag)."""
    st = lib().gl_ctx_sync_status(ctx)
    if st not in (GL_OK, GL_ERR_DOMAIN):
        _check(ctx, st)
    return st


def gl_ctx_last_error(ctx) -> str:
    return lib().gl_ctx_last_error(ctx).decode()


def gl_ctx_get_plan(ctx) -> int:
    """Persistent wavefronts per compute unit."""
    w = ctypes.c_int()
    _check(ctx, lib().gl_ctx_get_plan(ctx, ctypes.byref(w)))
    return w.value


def gl_ctx_set_plan(ctx, waves_per_cu: int) -> None:
    _check(ctx, lib().gl_ctx_set_plan(ctx, int(waves_per_cu)))


def gl_ctx_get_stage_plan(ctx):
    """(classify, hard, trap, gk) persistent wavefronts per compute unit."""
    c, h, t, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(ctx, lib().gl_ctx_get_stage_plan(ctx, ctypes.byref(c), ctypes.byref(h), ctypes.byref(t),
                                            ctypes.byref(g)))
    return c.value, h.value, t.value, g.value


def gl_ctx_set_stage_plan(ctx, classify: int, hard: int, trap: int, gk: int) -> None:
    _check(ctx, lib().gl_ctx_set_stage_plan(ctx, int(classify), int(hard), int(trap), int(gk)))


def gl_ctx_set_graph(ctx, on: bool) -> None:
    _check(ctx, lib().gl_ctx_set_graph(ctx, 1 if on else 0))


def gl_ctx_set_timing(ctx, n_slots: int) -> None:
    _check(ctx, lib().gl_ctx_set_timing(ctx, int(n_slots)))


def gl_ctx_get_timing(ctx):
    """Returns (compute_ms_sum, pipeline_ms_sum, n_batches_timed)."""
    c, p, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    _check(ctx, lib().gl_ctx_get_timing(ctx, ctypes.byref(c), ctypes.byref(p), ctypes.byref(n)))
    return c.value, p.value, n.value


def gl_ctx_get_stage_timing(ctx):
    """Returns ({stage name: ms summed over the timed batches}, n_batches_timed)."""
    st = (ctypes.c_double * GL_NSTAGES)()
    n = ctypes.c_int()
    _check(ctx, lib().gl_ctx_get_stage_timing(ctx, st, ctypes.byref(n)))
    return dict(zip(STAGE_NAMES, list(st))), n.value


def gl_ctx_set_capacity(ctx, sub_samples: int = 0, hard_samples: int = 0, arcs: int = 0) -> None:
    """Work-list capacities of the exact path (0 = default)."""
    _check(ctx, lib().gl_ctx_set_capacity(ctx, int(sub_samples), int(hard_samples), int(arcs)))


def gl_census(ctx, params, times, out, offsets=None, n_ss=None, t_exp=None, stream=None):
    """Runs the batch with the counting kernels; returns a dict of counts."""
    _validate(params, times, offsets, n_ss, t_exp, out)
    counts = (ctypes.c_int64 * len(CENSUS_NAMES))()
    st = lib().gl_census(ctx, _ptr(params), params.shape[1], _ptr(times), _ptr(offsets),
                         times.numel(), _ptr(n_ss), _ptr(t_exp), _ptr(out),
                         _stream_handle(stream), counts)
    _check(ctx, st)
    return dict(zip(CENSUS_NAMES, list(counts)))


def gl_flop_model():
    per = (ctypes.c_int64 * len(CENSUS_NAMES))()
    st = lib().gl_flop_model(per)
    if st != GL_OK:
        raise GLError(st, "gl_flop_model")
    return dict(zip(CENSUS_NAMES, list(per)))


def gl_ctx_get_overflow(ctx):
    """Waits; returns (chunks of the latest batch evaluated by the fused kernel
    because they did not fit the work lists, passes the batch ran)."""
    n, p = ctypes.c_int64(), ctypes.c_int()
    _check(ctx, lib().gl_ctx_get_overflow(ctx, ctypes.byref(n), ctypes.byref(p)))
    return n.value, p.value


def gl_ctx_get_unconverged(ctx) -> int:
    """Waits; returns (and clears) the number of ellipse arcs accepted at the
    arc rule's last level above its tolerance since the last call."""
    n = ctypes.c_int64()
    _check(ctx, lib().gl_ctx_get_unconverged(ctx, ctypes.byref(n)))
    return n.value


def gl_version() -> str:
    return lib().gl_version().decode()


# ---------------------------------------------------------------- convenience
class Context:
    """Owns a gl_ctx handle."""

    def __init__(self, device: int = 0):
        self.handle = gl_ctx_create(device)

    def close(self):
        if self.handle is not None:
            gl_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def batch(self, params, times, out=None, offsets=None, n_ss=None, t_exp=None, stream=None):
        import torch
        if out is None:
            n = params.shape[1] * times.numel() if offsets is None else times.numel()
            out = torch.empty(n, dtype=torch.float64, device=times.device)
        gl_lightcurve_batch(self.handle, params, times, out, offsets, n_ss, t_exp, stream)
        return out

    def loglike(self, walkers, times, data, sigma, model=None, offsets=None, n_ss=None, t_exp=None, stream=None):
        """(chi2, loglike, model) of a walker batch, device tensors."""
        import torch
        n = walkers.shape[1]
        if model is None:
            m = n * times.numel() if offsets is None else times.numel()
            model = torch.empty(m, dtype=torch.float64, device=times.device)
        chi2 = torch.empty(n, dtype=torch.float64, device=times.device)
        ll = torch.empty(n, dtype=torch.float64, device=times.device)
        gl_loglike_batch(self.handle, walkers, times, data, sigma, model, chi2, ll, offsets, n_ss, t_exp, stream)
        return chi2, ll, model

    def batch_ellipsoid(self, params, times, out=None, offsets=None, n_ss=None, t_exp=None, stream=None):
        import torch
        if out is None:
            n = params.shape[1] * times.numel() if offsets is None else times.numel()
            out = torch.empty(n, dtype=torch.float64, device=times.device)
        gl_lightcurve_batch_ellipsoid(self.handle, params, times, out, offsets, n_ss, t_exp, stream)
        return out


def to_device(workload, device="cuda"):
    """Moves a ``workloads.Workload`` to device tensors in the ABI layout."""
    import torch
    d = dict(
        params=torch.from_numpy(np.ascontiguousarray(workload.params)).to(device),
        times=torch.from_numpy(np.ascontiguousarray(workload.times)).to(device),
        offsets=None if workload.offsets is None else torch.from_numpy(
            np.ascontiguousarray(workload.offsets)).to(device),
        n_ss=torch.from_numpy(np.ascontiguousarray(workload.n_ss, dtype=np.int32)).to(device),
        t_exp=torch.from_numpy(np.ascontiguousarray(workload.t_exp)).to(device),
    )
    return d


# ---------------------------------------------------------------- surrogate network
GL_MLP_DIN, GL_MLP_WIDTH = 16, 256
EXPORTED = EXPORTED + ("gl_mlp_num_params", "gl_mlp_create", "gl_mlp_destroy", "gl_mlp_last_error",
                       "gl_mlp_set_weights", "gl_mlp_get_weights", "gl_mlp_forward", "gl_mlp_grads",
                       "gl_mlp_train_step")


def _mlp_lib():
    L = lib()
    if not getattr(L, "_mlp_typed", False):
        vp, i, i64, f = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float
        fp = ctypes.POINTER(ctypes.c_float)
        L.gl_mlp_num_params.argtypes = []
        L.gl_mlp_num_params.restype = i
        L.gl_mlp_create.argtypes = [ctypes.POINTER(vp), i, i]
        L.gl_mlp_create.restype = i
        L.gl_mlp_destroy.argtypes = [vp]
        L.gl_mlp_destroy.restype = None
        L.gl_mlp_last_error.argtypes = [vp]
        L.gl_mlp_last_error.restype = ctypes.c_char_p
        L.gl_mlp_set_weights.argtypes = [vp, fp, i64]
        L.gl_mlp_set_weights.restype = i
        L.gl_mlp_get_weights.argtypes = [vp, fp, i64]
        L.gl_mlp_get_weights.restype = i
        L.gl_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.gl_mlp_forward.restype = i
        L.gl_mlp_grads.argtypes = [vp, vp, vp, i64, fp, fp, vp]
        L.gl_mlp_grads.restype = i
        L.gl_mlp_train_step.argtypes = [vp, vp, vp, i64, f, vp, vp]
        L.gl_mlp_train_step.restype = i
        L._mlp_typed = True
    return L


def gl_mlp_num_params() -> int:
    return _mlp_lib().gl_mlp_num_params()


def _mcheck(h, st):
    if st != GL_OK:
        raise GLError(st, _mlp_lib().gl_mlp_last_error(h).decode() if h else "")


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class MLP:
    """Owns a gl_mlp handle (the BF16-MFMA surrogate network)."""

    def __init__(self, device: int = 0, max_batch: int = 8192):
        L = _mlp_lib()
        self.h = ctypes.c_void_p()
        st = L.gl_mlp_create(ctypes.byref(self.h), int(device), int(max_batch))
        if st != GL_OK:
            raise GLError(st, "gl_mlp_create")
        self.max_batch = max_batch

    def close(self):
        if self.h is not None:
            _mlp_lib().gl_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, packed: np.ndarray):
        packed = np.ascontiguousarray(packed, dtype=np.float32)
        _mcheck(self.h, _mlp_lib().gl_mlp_set_weights(self.h, _fptr(packed), packed.size))

    def get_weights(self) -> np.ndarray:
        out = np.empty(gl_mlp_num_params(), np.float32)
        _mcheck(self.h, _mlp_lib().gl_mlp_get_weights(self.h, _fptr(out), out.size))
        return out

    def forward(self, x, y=None, stream=None):
        import torch
        assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous() and x.shape[1] == GL_MLP_DIN
        if y is None:
            y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _mcheck(self.h, _mlp_lib().gl_mlp_forward(self.h, _ptr(x), x.shape[0], _ptr(y),
                                                  _stream_handle(stream)))
        return y

    def grads(self, x, t, stream=None):
        out = np.empty(gl_mlp_num_params(), np.float32)
        loss = ctypes.c_float()
        _mcheck(self.h, _mlp_lib().gl_mlp_grads(self.h, _ptr(x), _ptr(t), x.shape[0], _fptr(out),
                                                ctypes.byref(loss), _stream_handle(stream)))
        return out, loss.value

    def train_step(self, x, t, lr, loss_dev=None, stream=None):
        _mcheck(self.h, _mlp_lib().gl_mlp_train_step(self.h, _ptr(x), _ptr(t), x.shape[0],
                                                     float(lr), _ptr(loss_dev),
                                                     _stream_handle(stream)))


def pack_params(params) -> np.ndarray:
    """[(W_l[in][out], b_l)] -> packed FP32 layout of the library."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unpack_params(packed, d_in=GL_MLP_DIN, width=GL_MLP_WIDTH, depth=4):
    dims = [d_in] + [width] * depth + [1]
    out, o = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        W = packed[o:o + a * b].reshape(a, b)
        o += a * b
        bb = packed[o:o + b]
        o += b
        out.append((W, bb))
    return out


# ---------------------------------------------------------------- surrogate path
EXPORTED = EXPORTED + ("gl_surrogate_samples", "gl_surrogate_num_bins", "gl_surrogate_config_default",
                       "gl_surrogate_train", "gl_surrogate_destroy", "gl_surrogate_get", "gl_surrogate_config_of",
                       "gl_surrogate_save", "gl_surrogate_load", "gl_surrogate_file_write",
                       "gl_surrogate_file_read", "gl_lightcurve_batch_surrogate")


class SurrogateConfig(ctypes.Structure):
    """gl_surrogate_config (field for field)."""
    _fields_ = [("n_train", ctypes.c_int64), ("n_calib", ctypes.c_int64), ("epochs", ctypes.c_int),
                ("batch", ctypes.c_int), ("lr", ctypes.c_float), ("lr_final", ctypes.c_float),
                ("safety", ctypes.c_double), ("min_bin_count", ctypes.c_int), ("window", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("zero_predictor", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _sur_lib():
    L = _mlp_lib()
    if not getattr(L, "_sur_typed", False):
        vp, i, i64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        fp, u8p, i32p = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32)
        cfgp = ctypes.POINTER(SurrogateConfig)
        L.gl_surrogate_samples.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.gl_surrogate_samples.restype = i
        L.gl_surrogate_num_bins.argtypes = []
        L.gl_surrogate_num_bins.restype = i
        L.gl_surrogate_config_default.argtypes = [cfgp]
        L.gl_surrogate_config_default.restype = None
        L.gl_surrogate_train.argtypes = [vp, cfgp, ctypes.POINTER(vp), fp, vp]
        L.gl_surrogate_train.restype = i
        L.gl_surrogate_destroy.argtypes = [vp]
        L.gl_surrogate_destroy.restype = None
        L.gl_surrogate_get.argtypes = [vp, fp, i64, fp, u8p, i32p, i]
        L.gl_surrogate_get.restype = i
        L.gl_surrogate_config_of.argtypes = [vp, cfgp]
        L.gl_surrogate_config_of.restype = i
        L.gl_surrogate_save.argtypes = [vp, ctypes.c_char_p]
        L.gl_surrogate_save.restype = i
        L.gl_surrogate_load.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_char_p]
        L.gl_surrogate_load.restype = i
        L.gl_surrogate_file_write.argtypes = [ctypes.c_char_p, cfgp, fp, fp, fp, i64, i64, fp, u8p, i32p, i]
        L.gl_surrogate_file_write.restype = i
        L.gl_surrogate_file_read.argtypes = [ctypes.c_char_p, cfgp, fp, fp, fp, ctypes.POINTER(i64), i64, fp,
                                             u8p, i32p, i]
        L.gl_surrogate_file_read.restype = i
        L.gl_lightcurve_batch_surrogate.argtypes = [vp, vp, d, vp, i64, vp, vp, i64, vp, vp, vp, vp,
                                                    ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.gl_lightcurve_batch_surrogate.restype = i
        L._sur_typed = True
    return L


def gl_surrogate_num_bins() -> int:
    return _sur_lib().gl_surrogate_num_bins()


def gl_surrogate_config_default() -> SurrogateConfig:
    c = SurrogateConfig()
    _sur_lib().gl_surrogate_config_default(ctypes.byref(c))
    return c


def _u8p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _i32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def gl_surrogate_train(ctx, cfg: SurrogateConfig, stream=None):
    """Returns (surrogate handle, per-epoch mean squared errors)."""
    h = ctypes.c_void_p()
    hist = np.zeros(max(1, cfg.epochs), np.float32)
    _check(ctx, _sur_lib().gl_surrogate_train(ctx, ctypes.byref(cfg), ctypes.byref(h), _fptr(hist),
                                              _stream_handle(stream)))
    return h, hist[:cfg.epochs].tolist()


def gl_surrogate_destroy(h) -> None:
    _sur_lib().gl_surrogate_destroy(h)


def gl_surrogate_get(h):
    """Host copies: (params float32, table float32, zero_bins uint8, counts int32)."""
    p = np.empty(gl_mlp_num_params(), np.float32)
    nb = gl_surrogate_num_bins()
    t, z, c = np.empty(nb, np.float32), np.empty(nb, np.uint8), np.empty(nb, np.int32)
    st = _sur_lib().gl_surrogate_get(h, _fptr(p), p.size, _fptr(t), _u8p(z), _i32p(c), nb)
    if st != GL_OK:
        raise GLError(st, "gl_surrogate_get")
    return p, t, z, c


def gl_surrogate_config_of(h) -> SurrogateConfig:
    c = SurrogateConfig()
    st = _sur_lib().gl_surrogate_config_of(h, ctypes.byref(c))
    if st != GL_OK:
        raise GLError(st, "gl_surrogate_config_of")
    return c


def gl_surrogate_save(h, path: str) -> None:
    st = _sur_lib().gl_surrogate_save(h, os.fsencode(path))
    if st != GL_OK:
        raise GLError(st, f"gl_surrogate_save({path})")


def gl_surrogate_load(ctx, path: str):
    h = ctypes.c_void_p()
    _check(ctx, _sur_lib().gl_surrogate_load(ctx, ctypes.byref(h), os.fsencode(path)))
    return h


def gl_surrogate_file_write(path, cfg, params, m, v, step, table, zero_bins, counts) -> None:
    """Writes the surrogate file from host arrays (no device call)."""
    p, mm, vv = (np.ascontiguousarray(a, dtype=np.float32) for a in (params, m, v))
    t = np.ascontiguousarray(table, dtype=np.float32)
    z = np.ascontiguousarray(zero_bins, dtype=np.uint8)
    c = np.ascontiguousarray(counts, dtype=np.int32)
    st = _sur_lib().gl_surrogate_file_write(os.fsencode(path), ctypes.byref(cfg), _fptr(p), _fptr(mm), _fptr(vv),
                                            int(step), p.size, _fptr(t), _u8p(z), _i32p(c), t.size)
    if st != GL_OK:
        raise GLError(st, f"gl_surrogate_file_write({path})")


def gl_surrogate_file_read(path):
    """Reads a surrogate file into host arrays: (cfg, params, m, v, step,
    table, zero_bins, counts)."""
    cfg = SurrogateConfig()
    n = gl_mlp_num_params()
    nb = gl_surrogate_num_bins()
    p, m, v = (np.empty(n, np.float32) for _ in range(3))
    t, z, c = np.empty(nb, np.float32), np.empty(nb, np.uint8), np.empty(nb, np.int32)
    step = ctypes.c_int64()
    st = _sur_lib().gl_surrogate_file_read(os.fsencode(path), ctypes.byref(cfg), _fptr(p), _fptr(m), _fptr(v),
                                           ctypes.byref(step), n, _fptr(t), _u8p(z), _i32p(c), nb)
    if st != GL_OK:
        raise GLError(st, f"gl_surrogate_file_read({path})")
    return cfg, p, m, v, step.value, t, z, c


def gl_surrogate_samples(ctx, params, times, feat, target, f_obl=None, f_sph=None, scale=None,
                         bin=None, stream=None):
    n = params.shape[1]
    assert times.numel() == n and feat.shape == (n, GL_MLP_DIN) and target.numel() == n
    _check(ctx, _sur_lib().gl_surrogate_samples(ctx, _ptr(params), _ptr(times), n, _ptr(feat),
                                                _ptr(target), _ptr(f_obl), _ptr(f_sph), _ptr(scale),
                                                _ptr(bin), _stream_handle(stream)))


def gl_lightcurve_batch_surrogate(ctx, sur, tol, params, times, out, offsets=None, n_ss=None, t_exp=None,
                                  stream=None, counts=True):
    """Enqueues the gated light curves; with `counts`, waits and returns
    (in-window sub-samples, of those computed exactly although reaching the disk)."""
    _validate(params, times, offsets, n_ss, t_exp, out)
    a, b = ctypes.c_int64(), ctypes.c_int64()
    st = _sur_lib().gl_lightcurve_batch_surrogate(
        ctx, sur, float(tol), _ptr(params), params.shape[1], _ptr(times), _ptr(offsets), times.numel(),
        _ptr(n_ss), _ptr(t_exp), _ptr(out), _stream_handle(stream),
        ctypes.byref(a) if counts else None, ctypes.byref(b) if counts else None)
    _check(ctx, st)
    return (a.value, b.value) if counts else None
