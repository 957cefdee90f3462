"""Learned residual surrogate with exact fallback: orchestration only.

The library trains the network (its own BF16-MFMA kernels) on samples it
draws and evaluates with the exact kernels, calibrates the per-bin gate, and
evaluates gated light curves (gl_surrogate_train,
gl_lightcurve_batch_surrogate); this module holds the handle and the
PyTorch buffers.
"""
from __future__ import annotations

import numpy as np

from . import gl, workloads


class Samples:
    """Device-resident samples from the exact kernels (targets of the
    network), for inspection and tests."""

    def __init__(self, ctx, n: int, seed: int, window: float = 0.6, device="cuda"):
        import torch
        p, t = workloads.surrogate_samples(n, seed, window)
        self.params = torch.from_numpy(np.ascontiguousarray(p)).to(device)
        self.times = torch.from_numpy(np.ascontiguousarray(t)).to(device)
        self.feat = torch.empty((n, gl.GL_MLP_DIN), dtype=torch.float32, device=device)
        self.target = torch.empty(n, dtype=torch.float32, device=device)
        self.scale = torch.empty(n, dtype=torch.float64, device=device)
        self.bin = torch.empty(n, dtype=torch.int32, device=device)
        self.f_obl = torch.empty(n, dtype=torch.float64, device=device)
        self.f_sph = torch.empty(n, dtype=torch.float64, device=device)
        gl.gl_surrogate_samples(ctx.handle, self.params, self.times, self.feat, self.target,
                                self.f_obl, self.f_sph, self.scale, self.bin)
        self.n = n


def config(**kw) -> gl.SurrogateConfig:
    """The library's default configuration with the given fields changed."""
    c = gl.gl_surrogate_config_default()
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


class Surrogate:
    """Owns a gl_surrogate handle."""

    def __init__(self, ctx, handle, history=None):
        self.ctx = ctx
        self.h = handle
        self.history = list(history or [])

    @classmethod
    def train(cls, ctx, cfg: gl.SurrogateConfig, stream=None) -> "Surrogate":
        h, hist = gl.gl_surrogate_train(ctx.handle, cfg, stream)
        return cls(ctx, h, hist)

    @classmethod
    def load(cls, ctx, path: str) -> "Surrogate":
        return cls(ctx, gl.gl_surrogate_load(ctx.handle, path))

    def save(self, path: str) -> None:
        gl.gl_surrogate_save(self.h, path)

    def info(self):
        """(params, bound table, per-bin sphere-alone choice, calibration counts)."""
        return gl.gl_surrogate_get(self.h)

    def config(self) -> gl.SurrogateConfig:
        return gl.gl_surrogate_config_of(self.h)

    def lightcurve(self, d, out, tol=1e-6, stream=None, counts=True):
        """Gated light curves for a device workload dict (``gl.to_device``);
        with `counts`, returns (in-window sub-samples, exact fallbacks)."""
        return gl.gl_lightcurve_batch_surrogate(self.ctx.handle, self.h, tol, d["params"], d["times"], out,
                                                offsets=d["offsets"], n_ss=d["n_ss"], t_exp=d["t_exp"],
                                                stream=stream, counts=counts)

    def close(self):
        if self.h is not None:
            gl.gl_surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
