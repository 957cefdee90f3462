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

EXPORTED = ("gl_ctx_create", "gl_ctx_destroy", "gl_lightcurve_batch", "gl_ctx_sync_status",
            "gl_ctx_last_error", "gl_autotune", "gl_ctx_get_plan", "gl_ctx_set_plan",
            "gl_ctx_set_graph", "gl_ctx_set_timing", "gl_ctx_get_timing", "gl_census",
            "gl_flop_model", "gl_version")
CENSUS_NAMES = ("sub_in_window", "whole_on_star", "intersecting", "off_star_in_window",
                "trapezoid_nodes", "gk21_pieces", "newton_steps", "limb_arcs")


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
        L.gl_ctx_set_graph.argtypes = [vp, i]
        L.gl_ctx_set_graph.restype = i
        L.gl_ctx_set_timing.argtypes = [vp, i]
        L.gl_ctx_set_timing.restype = i
        dpp = ctypes.POINTER(ctypes.c_double)
        L.gl_ctx_get_timing.argtypes = [vp, dpp, dpp, ctypes.POINTER(i)]
        L.gl_ctx_get_timing.restype = i
        L.gl_census.argtypes = batch_args + [ctypes.POINTER(ctypes.c_int64)]
        L.gl_census.restype = i
        L.gl_flop_model.argtypes = [ctypes.POINTER(ctypes.c_int64)]
        L.gl_flop_model.restype = i
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


def _validate(params, times, offsets, n_ss, t_exp, out):
    import torch
    assert params.dtype == torch.float64 and params.is_cuda and params.is_contiguous()
    assert params.dim() == 2 and params.shape[0] == GL_NPARAM
    assert times.dtype == torch.float64 and times.is_cuda and times.is_contiguous()
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    n_sets = params.shape[1]
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


def gl_autotune(ctx, params, times, out, offsets=None, n_ss=None, t_exp=None, stream=None) -> None:
    _validate(params, times, offsets, n_ss, t_exp, out)
    st = lib().gl_autotune(ctx, _ptr(params), params.shape[1], _ptr(times), _ptr(offsets),
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


def gl_ctx_set_graph(ctx, on: bool) -> None:
    _check(ctx, lib().gl_ctx_set_graph(ctx, 1 if on else 0))


def gl_ctx_set_timing(ctx, n_slots: int) -> None:
    _check(ctx, lib().gl_ctx_set_timing(ctx, int(n_slots)))


def gl_ctx_get_timing(ctx):
    """Returns (compute_ms_sum, pipeline_ms_sum, n_batches_timed)."""
    c, p, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    _check(ctx, lib().gl_ctx_get_timing(ctx, ctypes.byref(c), ctypes.byref(p), ctypes.byref(n)))
    return c.value, p.value, n.value


def gl_census(ctx, params, times, out, offsets=None, n_ss=None, t_exp=None, stream=None):
    """Runs the batch with the counting kernel; returns a dict of counts."""
    _validate(params, times, offsets, n_ss, t_exp, out)
    counts = (ctypes.c_int64 * 8)()
    st = lib().gl_census(ctx, _ptr(params), params.shape[1], _ptr(times), _ptr(offsets),
                         times.numel(), _ptr(n_ss), _ptr(t_exp), _ptr(out),
                         _stream_handle(stream), counts)
    _check(ctx, st)
    return dict(zip(CENSUS_NAMES, list(counts)))


def gl_flop_model():
    per = (ctypes.c_int64 * 8)()
    st = lib().gl_flop_model(per)
    if st != GL_OK:
        raise GLError(st, "gl_flop_model")
    return dict(zip(CENSUS_NAMES, list(per)))


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
