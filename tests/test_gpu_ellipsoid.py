"""GPU parity for general ellipsoids (free rotators and tidally-locked
planets) through gl_lightcurve_batch_ellipsoid, against the CPU FP64 oracle's
quadric-shadow route.  Bar: |gpu - oracle| <= 1e-9 on every compared point,
no arc accepted unconverged."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-9


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def run_ell(gl, ctx, w):
    import torch
    d = gl.to_device(w, "cuda:0")
    out = ctx.batch_ellipsoid(d["params"], d["times"], offsets=d["offsets"], n_ss=d["n_ss"], t_exp=d["t_exp"])
    torch.cuda.synchronize()
    st = gl.gl_ctx_sync_status(ctx.handle)
    unconv = gl.gl_ctx_get_unconverged(ctx.handle)
    assert unconv == 0, f"{unconv} arcs accepted unconverged"
    res = out.cpu().numpy()
    if w.offsets is None:
        res = res.reshape(w.n_sets, -1)
    return res, st


def test_mixed_batch_all_points(gpu_lib, ctx, oracle):
    from paper_2410_05408_amd import workloads as W
    say("case: ellipsoid batch, 96 sets (48 locked) x 400 points, n_ss in {1, 5}, all points")
    w = W.ellipsoid_batch(n_sets=96, n_w=400, seed=11)
    got, st = run_ell(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_OK
    ref = oracle.flux_batch_ell(w.params, w.times, offsets=w.offsets, n_ss=w.n_ss, t_exp=w.t_exp)
    err = np.abs(got - ref)
    lk = np.repeat(w.params[W.E_LOCKED] == 1.0, np.diff(w.offsets))
    say(f"  max err {err.max():.3e} (locked {err[lk].max():.3e}, free {err[~lk].max():.3e}), "
        f"in transit {np.sum(ref < 1)}")
    assert np.sum(ref[lk] < 1) > 1000 and np.sum(ref[~lk] < 1) > 1000
    assert err.max() <= TOL


def test_shared_grid_graph_replays(gpu_lib, ctx, oracle):
    """Shared grid (chunks of a set in one window wavefront), locked and free
    sets interleaved, replayed through the captured graph."""
    import torch
    from paper_2410_05408_amd import workloads as W
    say("case: ellipsoid shared grid, 40 sets x 1000 times, two replays")
    rng = np.random.default_rng(12)
    p = np.concatenate([W.draw_ellipsoids(rng, 20, True), W.draw_ellipsoids(rng, 20, False)], axis=1)
    p = np.ascontiguousarray(p[:, rng.permutation(40)])
    p[W.E_P] = 2.0
    p[W.E_ARS] = np.where(p[W.E_LOCKED] == 1.0, p[W.E_ARS], 5.0 + 3.0 * p[W.E_ARS] / 300.0)
    times = np.linspace(-0.25, 0.25, 1000)
    pd = torch.from_numpy(p).cuda()
    td = torch.from_numpy(times).cuda()
    ss = torch.full((40,), 3, dtype=torch.int32, device="cuda")
    te = torch.full((40,), 0.002, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    outs = []
    for _ in range(2):
        with torch.cuda.stream(s):
            o = ctx.batch_ellipsoid(pd, td, n_ss=ss, t_exp=te, stream=s)
        s.synchronize()
        outs.append(o.cpu().numpy().reshape(40, -1))
    assert gpu_lib.gl_ctx_sync_status(ctx.handle) == gpu_lib.GL_OK
    assert np.array_equal(outs[0], outs[1])
    ref = oracle.flux_batch_ell(p, times, n_ss=np.full(40, 3, np.int32), t_exp=np.full(40, 0.002))
    err = np.abs(outs[0] - ref)
    say(f"  max err {err.max():.3e}, in transit {np.sum(ref < 1)}")
    assert np.sum(ref < 1) > 5000
    assert err.max() <= TOL


def test_spheroid_block_matches_oblate_entry(gpu_lib, ctx):
    """b = c: the ellipsoid entry on the oblate model's walker draws equals the
    oblate entry (different constant set-up, same flux)."""
    import torch
    from paper_2410_05408_amd import workloads as W
    say("case: spheroids through both entry points, 64 walker sets x 3000 x 15")
    w = W.walker_batch(n_sets=64)
    p = w.params
    e = np.empty((13, w.n_sets))
    e[W.E_RA] = p[W.K] * (1.0 - p[W.F])
    e[W.E_RB] = e[W.E_RC] = p[W.K]
    e[W.E_ZETA] = 0.0
    e[W.E_ETA] = 0.5 * math.pi - p[W.THETA]
    e[W.E_XI] = p[W.PHI]
    e[W.E_B:W.E_Q2 + 1] = p[W.B:W.Q2 + 1]
    e[W.E_LOCKED] = 0.0
    d = gpu_lib.to_device(w, "cuda:0")
    a = ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"])
    b = ctx.batch_ellipsoid(torch.from_numpy(e).cuda(), d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"])
    torch.cuda.synchronize()
    diff = np.abs(a.cpu().numpy() - b.cpu().numpy())
    say(f"  max |ellipsoid - oblate| {diff.max():.3e}")
    assert diff.max() <= 1e-12


def test_full_size_sampled(gpu_lib, ctx, oracle):
    """The default mixed batch (2048 sets x 1500 points): every in-transit
    output of 24 sets and 3000 sampled outputs against the oracle."""
    from paper_2410_05408_amd import workloads as W
    say("case: ellipsoid batch full size 2048 x 1500, sampled")
    w = W.ellipsoid_batch()
    got, st = run_ell(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_OK
    assert np.all((got >= 0.0) & (got <= 1.0))
    rng = np.random.default_rng(5)
    seg = np.diff(w.offsets)
    set_of = np.repeat(np.arange(w.n_sets), seg)
    pick = np.concatenate([rng.choice(got.size, 3000, replace=False),
                           np.concatenate([np.arange(w.offsets[s], w.offsets[s + 1])
                                           for s in rng.choice(w.n_sets, 24, replace=False)])])
    sp = set_of[pick]
    ref = oracle.flux_batch_ell(np.ascontiguousarray(w.params[:, sp]), w.times[pick],
                                offsets=np.arange(pick.size + 1), n_ss=w.n_ss[sp], t_exp=w.t_exp[sp])
    err = np.abs(got[pick] - ref)
    say(f"  max err {err.max():.3e} over {pick.size} outputs, in transit {np.sum(ref < 1)}")
    assert err.max() <= TOL


def test_domain_errors(gpu_lib, ctx):
    import torch
    from paper_2410_05408_amd import workloads as W
    say("case: ellipsoid domain errors")
    rng = np.random.default_rng(13)
    p = W.draw_ellipsoids(rng, 6, True)
    p[W.E_RB, 1] = 1.2            # semi-axis outside (0, 1)
    p[W.E_ARS, 2] = 1.0 + 0.5 * p[W.E_RC, 2]  # orbit inside 1 + max axis
    p[W.E_LOCKED, 3] = 0.5        # neither free nor locked
    p[W.E_ETA, 4] = float("nan")
    times = np.linspace(-0.05, 0.05, 130)
    out = ctx.batch_ellipsoid(torch.from_numpy(p).cuda(), torch.from_numpy(times).cuda())
    torch.cuda.synchronize()
    st = gpu_lib.gl_ctx_sync_status(ctx.handle)
    o = out.cpu().numpy().reshape(6, -1)
    assert st == gpu_lib.GL_ERR_DOMAIN
    assert np.all(np.isnan(o[1:5]))
    assert np.all(np.isfinite(o[[0, 5]])) and np.min(o[[0, 5]]) < 1.0


def test_autotune_ellipsoid_keeps_results(gpu_lib, oracle):
    """gl_autotune_ellipsoid on a mixed batch picks a plan within the knobs'
    candidates, and the batch gives the same outputs bit for bit under the
    tuned plan (grid sizes only move work), still within the bar of the
    oracle on sampled points."""
    import torch
    from paper_2410_05408_amd import workloads as W
    gl = gpu_lib
    say("case: ellipsoid autotune, 64 sets (32 locked) x 300 points, CSR")
    w = W.ellipsoid_batch(n_sets=64, n_w=300, seed=21)
    c = gl.Context(0)
    try:
        before, _ = run_ell(gl, c, w)
        d = gl.to_device(w, "cuda:0")
        out = torch.empty(w.n_out, dtype=torch.float64, device="cuda")
        s = torch.cuda.Stream()
        gl.gl_autotune_ellipsoid(c.handle, d["params"], d["times"], out, offsets=d["offsets"], n_ss=d["n_ss"],
                                 t_exp=d["t_exp"], stream=s)
        s.synchronize()
        plan = gl.gl_ctx_get_stage_plan(c.handle)
        say(f"  tuned plan (classify, hard, trapezoid, arcs) {plan}")
        assert plan[0] in (8, 16, 24, 32, 48, 64) and plan[1] in (4, 8, 16, 24, 32, 48, 64)
        assert plan[2] in (4, 8, 16, 24, 32, 48, 64) and plan[3] in (8, 12, 16, 20, 32, 48, 64)
        after, st = run_ell(gl, c, w)
        assert st == gl.GL_OK
        assert np.array_equal(before, after)
        idx = np.arange(0, w.n_out, 7)
        ref = oracle.flux_batch_ell(w.params, w.times, offsets=w.offsets, n_ss=w.n_ss, t_exp=w.t_exp)
        assert np.max(np.abs(after[idx] - ref[idx])) <= TOL
    finally:
        c.close()
