"""Learned residual surrogate with exact fallback (training and evaluation).

The network (library kernels, BF16 matrix cores) predicts the scaled residual
(F_oblate - F_sphere) / (k^2 (1 - q)) of the exact oblate flux against the
equal-projected-area sphere; the library's gate accepts F_sphere + prediction
only where the calibrated scaled-error bound of the sample's bin, times the
sample's own scale k^2 (1 - q) and a safety factor, is within the tolerance,
and computes every other sub-sample with the exact kernel.  This module only orchestrates: every number is produced by the
library (gl_surrogate_samples, gl_mlp_*, gl_surrogate_bound,
gl_lightcurve_batch_surrogate); PyTorch provides buffers, index permutations
and streams.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import gl, workloads


def init_weights(seed: int, d_in: int = gl.GL_MLP_DIN, width: int = gl.GL_MLP_WIDTH,
                 depth: int = 4) -> np.ndarray:
    """He-uniform initial weights, zero biases, packed in the library layout."""
    rng = np.random.default_rng(seed)
    dims = [d_in] + [width] * depth + [1]
    parts = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = math.sqrt(6.0 / a) if b != 1 else math.sqrt(3.0 / a)
        parts += [rng.uniform(-lim, lim, a * b), np.zeros(b)]
    return np.concatenate(parts).astype(np.float32)


class Samples:
    """Device-resident samples from the exact kernels."""

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


class Surrogate:
    def __init__(self, ctx, device: int = 0, max_batch: int = 8192, seed: int = 0, zero: bool = False):
        import torch
        self.ctx = ctx
        self.net = gl.MLP(device, max_batch)
        w = init_weights(seed)
        if zero:
            w[:] = 0.0  # the zero-residual predictor (ablation baseline)
        self.net.set_weights(w)
        self.bins = gl.gl_surrogate_num_bins()
        self.table = torch.full((self.bins,), -1.0, dtype=torch.float32, device="cuda")
        self.zero_bins = None  # bins where the sphere alone calibrated better
        self.max_batch = max_batch
        self.history = []

    def close(self):
        self.net.close()

    def train(self, data: Samples, epochs: int, batch: int = 8192, lr: float = 2e-3,
              lr_final: float = 1e-4, seed: int = 0, log=None):
        import torch
        batch = min(batch, self.max_batch)
        keep = torch.nonzero(data.bin >= 0).squeeze(1)  # samples on the star
        n = keep.numel()
        steps = max(1, epochs * (n // batch))
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        loss_dev = torch.zeros(1, dtype=torch.float32, device="cuda")
        step = 0
        t0 = time.perf_counter()
        for ep in range(epochs):
            perm = keep[torch.randperm(n, device="cuda", generator=g)]
            ep_loss = torch.zeros(1, dtype=torch.float64, device="cuda")
            for b0 in range(0, n - batch + 1, batch):
                idx = perm[b0:b0 + batch]
                x = data.feat.index_select(0, idx).contiguous()
                t = data.target.index_select(0, idx).contiguous()
                lr_s = lr * (lr_final / lr) ** (step / max(1, steps - 1))
                self.net.train_step(x, t, lr_s, loss_dev)
                ep_loss += loss_dev.double()
                step += 1
            torch.cuda.synchronize()
            mse = float(ep_loss.item()) / max(1, (n // batch) * batch)
            self.history.append(mse)
            if log:
                log(f"epoch {ep}: train mse {mse:.3e} ({time.perf_counter() - t0:.1f} s)")
        return self.history

    def predict(self, feat):
        return self.net.forward(feat)

    def calibrate(self, data: Samples, choose: bool = True):
        """Per-bin maximum scaled error on calibration samples; bins without
        samples stay negative (always computed exactly).  With `choose`, each
        bin keeps the better of the network and the zero-residual predictor
        (the equal-area sphere alone), so the gate never accepts less than the
        sphere would."""
        import torch
        pred = self.predict(data.feat)
        self.table.zero_()
        gl.gl_surrogate_bound(self.ctx.handle, pred, data.target, data.scale, data.bin, self.table)
        counts = torch.bincount(data.bin[data.bin >= 0].long(), minlength=self.bins)
        if choose:
            zero = torch.zeros_like(self.table)
            gl.gl_surrogate_bound(self.ctx.handle, torch.zeros_like(pred), data.target, data.scale,
                                  data.bin, zero)
            self.zero_bins = (zero < self.table).to(torch.uint8)
            self.table = torch.minimum(self.table, zero)
        self.table[counts == 0] = -1.0
        torch.cuda.synchronize()
        return self.table

    def save(self, path: str) -> None:
        """Writes the network, the calibrated bound table and the per-bin
        predictor choice (gl_surrogate_save)."""
        zb = None if self.zero_bins is None else self.zero_bins.cpu().numpy()
        gl.gl_surrogate_save(path, self.net.get_weights(), self.table.cpu().numpy(), zb)

    @classmethod
    def load(cls, ctx, path: str, device: int = 0, max_batch: int = 8192) -> "Surrogate":
        """A surrogate read back from gl_surrogate_save's file, ready for
        lightcurve() (no training or calibration needed)."""
        import torch
        w, table, zb = gl.gl_surrogate_load(path)
        sur = cls(ctx, device=device, max_batch=max_batch)
        sur.net.set_weights(w)
        sur.table = torch.from_numpy(table).to("cuda")
        sur.zero_bins = torch.from_numpy(zb).to("cuda")
        return sur

    def lightcurve(self, d, out, tol=1e-6, safety=4.0, stream=None):
        """Gated light curves for a device workload dict (``gl.to_device``);
        returns (n_sub, n_fallback)."""
        return gl.gl_lightcurve_batch_surrogate(self.ctx.handle, self.net, self.table, safety, tol,
                                                d["params"], d["times"], out, offsets=d["offsets"],
                                                n_ss=d["n_ss"], t_exp=d["t_exp"], stream=stream,
                                                zero_bins=self.zero_bins)
