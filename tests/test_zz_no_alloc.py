"""GPU: the allocation-free batch (gl_lightcurve_batch_noalloc) against
gl_lightcurve_batch on the same inputs, on consecutive calls that share the
library's device array, each smaller than the one before; and its size limit.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-12  # same kernels; chunks beyond the fixed lists take the fused kernel (rounding only)


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


def both(gl, ctx, w):
    import torch
    d = gl.to_device(w, "cuda:0")
    args = dict(offsets=d["offsets"], n_ss=d["n_ss"], t_exp=d["t_exp"])
    ref = ctx.batch(d["params"], d["times"], **args)
    got = torch.full_like(ref, -7.0)
    gl.gl_lightcurve_batch_noalloc(d["params"], d["times"], got, **args)
    torch.cuda.synchronize()
    assert gl.gl_ctx_sync_status(ctx.handle) == gl.GL_OK
    return got.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_matches_batch_on_consecutive_calls(gpu_lib):
    from paper_2410_05408_amd import workloads as W
    gl = gpu_lib
    ctx = gl.Context(0)
    try:
        cases = (("walker batch 4096 x 3000 x 15 (beyond the fixed lists)", W.walker_batch()),
                 ("walker batch 96 x 3000 x 15", W.walker_batch(n_sets=96)),
                 ("adversarial CSR batch, 320 sets x 266 times", W.adversarial_batch(n_dense=200)))
        for name, w in cases:
            say(f"case: allocation-free call, {name}")
            got, ref = both(gl, ctx, w)
            err = np.max(np.abs(got - ref))
            say(f"  max |noalloc - batch| {err:.2e}, identical {np.array_equal(got, ref)}, "
                f"in transit {np.sum(ref < 1.0)}")
            assert np.all(np.isfinite(got)) and err <= TOL
    finally:
        ctx.close()


def test_noalloc_rejects_sizes_beyond_its_limits(gpu_lib):
    import torch
    gl = gpu_lib
    say("case: allocation-free call beyond its limits")
    n = 16385
    params = torch.zeros((10, n), dtype=torch.float64, device="cuda")
    times = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(gl.GLError) as e:
        gl.gl_lightcurve_batch_noalloc(params, times, out)
    assert e.value.status == gl.GL_ERR_SIZE
    torch.cuda.synchronize()
    assert torch.all(out == -7.0)  # nothing was enqueued
