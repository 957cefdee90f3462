"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Bar: |gpu - oracle| <= 1e-9 on every compared point.  The oracle shares no
code with the HIP library; both are fed from the seeded workload generator.
Every batch run through `run` also checks that the arc rule accepted no arc
unconverged at its last level (gl_ctx_get_unconverged).
"""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-9
HERE = os.path.dirname(os.path.abspath(__file__))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def run(gl, ctx, w, **kw):
    import torch
    d = gl.to_device(w, "cuda:0")
    out = ctx.batch(d["params"], d["times"], offsets=d["offsets"], n_ss=d["n_ss"],
                    t_exp=d["t_exp"], **kw)
    torch.cuda.synchronize()
    st = gl.gl_ctx_sync_status(ctx.handle)
    unconv = gl.gl_ctx_get_unconverged(ctx.handle)
    assert unconv == 0, f"{unconv} arcs accepted unconverged"
    res = out.cpu().numpy()
    if w.offsets is None:
        res = res.reshape(w.n_sets, -1)
    return res, st


def test_single_transit_all_points(gpu_lib, ctx):
    from paper_2410_05408_amd import workloads as W
    say("case: single transit, 1000 points")
    w = W.single_transit()
    got, st = run(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_OK
    ref = np.loadtxt(os.path.join(HERE, "golden", "single_transit_oracle.txt"))[:, 1]
    err = np.abs(got[0] - ref)
    say(f"  max err {err.max():.3e}")
    assert err.max() <= TOL
    assert np.all(got[0][ref == 1.0] == 1.0)


def test_walker_batch_small_all_points(gpu_lib, ctx, oracle):
    from paper_2410_05408_amd import workloads as W
    say("case: walker batch, 48 sets x 3000 times x 15 sub-samples, all points")
    w = W.walker_batch(n_sets=48)
    got, st = run(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_OK
    ref = oracle.flux_batch(w.params, w.times, n_ss=w.n_ss, t_exp=w.t_exp)
    err = np.abs(got - ref)
    say(f"  max err {err.max():.3e}, in transit {np.sum(ref < 1)}")
    assert err.max() <= TOL


def test_walker_batch_full_size_sampled(gpu_lib, ctx, oracle):
    from paper_2410_05408_amd import workloads as W
    say("case: walker batch full size 4096 x 3000 x 15, stratified sample")
    w = W.walker_batch()
    got, st = run(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_OK
    assert np.all((got >= 0.0) & (got <= 1.0))
    rng = np.random.default_rng(0)
    sets = rng.choice(w.n_sets, 24, replace=False)
    ref = oracle.flux_batch(w.params[:, sets], w.times, n_ss=w.n_ss[sets], t_exp=w.t_exp[sets])
    err = np.abs(got[sets] - ref)
    say(f"  24 full sets: max err {err.max():.3e}")
    assert err.max() <= TOL
    # every output that changes, across all sets, in a random sample
    changed = np.flatnonzero(got.ravel() < 1.0)
    sel = rng.choice(changed, min(3000, changed.size), replace=False)
    refs = oracle.flux_select(w.params, w.times, sel, n_ss=w.n_ss, t_exp=w.t_exp)
    err2 = np.abs(got.ravel()[sel] - refs)
    say(f"  3000 in-transit outputs: max err {err2.max():.3e}")
    assert err2.max() <= TOL


def test_walker_batch_bench_configuration(gpu_lib, oracle):
    """The launch configuration bench.py times, at full size: a fresh context,
    the plan from gl_autotune, the batch captured as a graph on a
    non-default stream (hard-sample chain and trapezoid on two streams) and
    replayed; every replay equals the direct launch bit for bit, and sampled
    in-transit outputs are within the bar of the oracle."""
    import torch
    from paper_2410_05408_amd import workloads as W
    gl = gpu_lib
    say("case: walker batch full size in the bench's configuration (autotuned plan, graph replays)")
    w = W.walker_batch()
    c = gl.Context(0)
    try:
        direct, st = run(gl, c, w)
        assert st == gl.GL_OK
        d = gl.to_device(w, "cuda:0")
        out = torch.empty(w.n_out, dtype=torch.float64, device="cuda")
        s = torch.cuda.Stream()
        gl.gl_autotune(c.handle, d["params"], d["times"], out, n_ss=d["n_ss"], t_exp=d["t_exp"], stream=s)
        s.synchronize()
        say(f"  plan (classify, hard, trapezoid, arcs) {gl.gl_ctx_get_stage_plan(c.handle)}")
        for rep in range(2):
            o = c.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"], stream=s)
            s.synchronize()
            assert gl.gl_ctx_sync_status(c.handle) == gl.GL_OK
            assert np.array_equal(o.cpu().numpy().reshape(w.n_sets, -1), direct), f"replay {rep}"
        rng = np.random.default_rng(5)
        changed = np.flatnonzero(direct.ravel() < 1.0)
        sel = rng.choice(changed, min(500, changed.size), replace=False)
        refs = oracle.flux_select(w.params, w.times, sel, n_ss=w.n_ss, t_exp=w.t_exp)
        err = np.abs(direct.ravel()[sel] - refs)
        say(f"  500 in-transit outputs: max err {err.max():.3e}")
        assert err.max() <= TOL
    finally:
        c.close()


def test_high_cadence_all_points(gpu_lib, ctx, oracle):
    from paper_2410_05408_amd import workloads as W
    say("case: high cadence 512 x 65536, all 33.5M points")
    w = W.high_cadence()
    got, st = run(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_OK
    ref = oracle.flux_batch(w.params, w.times, n_ss=w.n_ss, t_exp=w.t_exp)
    err = np.abs(got - ref)
    say(f"  max err {err.max():.3e}, points changed {np.sum(ref < 1)}")
    assert err.max() <= TOL


def test_uneven_batch_sampled(gpu_lib, ctx, oracle):
    from paper_2410_05408_amd import workloads as W
    say("case: uneven CSR batch 16384 walkers (71.4M outputs), sampled")
    w = W.uneven_batch()
    got, st = run(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_OK
    assert np.all((got >= 0.0) & (got <= 1.0))
    rng = np.random.default_rng(1)
    sets = rng.choice(w.n_sets, 12, replace=False)
    sel = np.concatenate([np.arange(w.offsets[s], w.offsets[s + 1]) for s in sets])
    changed = np.flatnonzero(got < 1.0)
    sel = np.concatenate([sel, rng.choice(changed, 3000, replace=False)])
    ref = oracle.flux_select(w.params, w.times, sel, offsets=w.offsets, n_ss=w.n_ss, t_exp=w.t_exp)
    err = np.abs(got[sel] - ref)
    say(f"  {sel.size} outputs: max err {err.max():.3e}")
    assert err.max() <= TOL


def test_uneven_batch_graph_replay(gpu_lib, ctx, oracle):
    """The uneven CSR batch with work lists sized from the demand of a first
    run (several passes, nothing left to the fused kernel), on a non-default
    stream, i.e. captured into a HIP graph and replayed: equal bit for bit to
    the direct launch of the same plan, equal to rounding to the first run
    (other passes, overflowing chunks in the fused kernel), and equal to the
    oracle on sampled outputs."""
    import torch
    from paper_2410_05408_amd import workloads as W
    gl = gpu_lib
    say("case: uneven CSR batch 16384 walkers, graph capture + replays vs direct launch")
    w = W.uneven_batch()
    d = gl.to_device(w, "cuda:0")
    args = dict(offsets=d["offsets"], n_ss=d["n_ss"], t_exp=d["t_exp"])
    s = torch.cuda.Stream()
    gl.gl_ctx_set_graph(ctx.handle, False)
    try:
        first = torch.empty(w.n_out, dtype=torch.float64, device="cuda")
        gl.gl_lightcurve_batch(ctx.handle, d["params"], d["times"], first, stream=s, **args)
        fused1, passes1 = gl.gl_ctx_get_overflow(ctx.handle)
        direct = torch.empty_like(first)
        for k in range(3):  # the plan settles within a run or two of the first
            gl.gl_lightcurve_batch(ctx.handle, d["params"], d["times"], direct, stream=s, **args)
            fused, passes = gl.gl_ctx_get_overflow(ctx.handle)
            say(f"  run {k + 2}: {passes} passes, {fused} fused chunks (first run: {passes1} pass(es), "
                f"{fused1} fused chunks)")
            if fused == 0:
                break
        assert fused == 0 and passes >= 2
        d_first = (first - direct).abs().max().item()
        say(f"  first run vs planned run: {d_first:.2e}")
        assert d_first <= 1e-12
        gl.gl_ctx_set_graph(ctx.handle, True)
        out = torch.empty_like(direct)
        for r in range(3):  # capture, then two replays with eager work between
            out.fill_(-1.0)
            torch.cuda.synchronize()
            gl.gl_lightcurve_batch(ctx.handle, d["params"], d["times"], out, stream=s, **args)
            with torch.cuda.stream(s):
                junk = torch.randn(4096, device="cuda").sum()  # noqa: F841
            s.synchronize()
            assert torch.equal(out, direct), f"replay {r} differs from the direct launch"
    finally:
        gl.gl_ctx_set_graph(ctx.handle, True)
    assert gl.gl_ctx_sync_status(ctx.handle) == gl.GL_OK
    assert gl.gl_ctx_get_unconverged(ctx.handle) == 0
    got = out.cpu().numpy()
    rng = np.random.default_rng(2)
    sets = rng.choice(w.n_sets, 8, replace=False)
    sel = np.concatenate([np.arange(w.offsets[s_], w.offsets[s_ + 1]) for s_ in sets])
    changed = np.flatnonzero(got < 1.0)
    sel = np.concatenate([sel, rng.choice(changed, 2000, replace=False)])
    ref = oracle.flux_select(w.params, w.times, sel, offsets=w.offsets, n_ss=w.n_ss, t_exp=w.t_exp)
    err = np.abs(got[sel] - ref)
    say(f"  {sel.size} outputs of the replayed graph: max err {err.max():.3e}")
    assert err.max() <= TOL


def test_adversarial_all_points(gpu_lib, ctx, oracle):
    from paper_2410_05408_amd import workloads as W
    say("case: adversarial shapes and grazing geometries, all points")
    w = W.adversarial_batch(600)
    got, st = run(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_OK
    ref = oracle.flux_batch(w.params, w.times, offsets=w.offsets, n_ss=w.n_ss, t_exp=w.t_exp)
    err = np.abs(got - ref)
    i = int(np.argmax(err))
    s = int(np.searchsorted(w.offsets, i, side="right") - 1)
    say(f"  max err {err.max():.3e} at set {s} params {w.params[:, s]} t {w.times[i]}")
    assert err.max() <= TOL


def _csr(params, grids, n_ss, t_exp):
    from paper_2410_05408_amd import workloads as W
    offsets = np.zeros(len(grids) + 1, np.int64)
    offsets[1:] = np.cumsum([len(g) for g in grids])
    times = np.concatenate(grids) if offsets[-1] else np.zeros(0)
    return W.Workload("csr", np.ascontiguousarray(params), times, offsets,
                      np.asarray(n_ss, np.int32), np.asarray(t_exp, float))


def test_ragged_segments_and_extremes(gpu_lib, ctx, oracle):
    from paper_2410_05408_amd import workloads as W
    say("case: ragged CSR segments (0, 1, 63, 64, 65, 127, 200), n_ss up to 64")
    base = W.walker_batch(n_sets=7).params
    base[W.B] = 0.2
    lens = [0, 1, 63, 64, 65, 127, 200]
    grids = [np.linspace(-0.3, 0.3, n) for n in lens]
    w = _csr(base, grids, [1, 64, 15, 5, 64, 2, 15], [0.0, 0.01, 0.02, 0.0, 0.03, 0.001, 0.0204])
    got, st = run(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_OK
    ref = oracle.flux_batch(w.params, w.times, offsets=w.offsets, n_ss=w.n_ss, t_exp=w.t_exp)
    err = np.abs(got - ref)
    say(f"  max err {err.max():.3e}")
    assert err.max() <= TOL


def test_several_transits_per_grid(gpu_lib, ctx, oracle):
    from paper_2410_05408_amd import workloads as W
    say("case: short period, grid spanning several transits and eclipses")
    p = W.walker_batch(n_sets=16).params
    p[W.P] = 3.0
    p[W.ARS] = 8.0
    p[W.T0] = 0.37
    w = W.Workload("multi", p, np.linspace(-7.0, 7.0, 6000), None,
                   np.full(16, 3, np.int32), np.full(16, 0.004), {})
    got, st = run(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_OK
    ref = oracle.flux_batch(w.params, w.times, n_ss=w.n_ss, t_exp=w.t_exp)
    err = np.abs(got - ref)
    say(f"  max err {err.max():.3e}, transits seen {np.sum(np.diff((ref[0] < 1).astype(int)) == 1)}")
    assert err.max() <= TOL


def test_shared_grid_of_one_time(gpu_lib, ctx, oracle):
    from paper_2410_05408_amd import workloads as W
    say("case: one time per set")
    w = W.walker_batch(n_sets=300, n_times=1, n_ss=5)
    w.times[:] = 0.01
    got, st = run(gpu_lib, ctx, w)
    ref = oracle.flux_batch(w.params, w.times, n_ss=w.n_ss, t_exp=w.t_exp)
    assert st == gpu_lib.GL_OK and np.abs(got - ref).max() <= TOL


def test_domain_errors_give_nan_and_status(gpu_lib, ctx, oracle):
    from paper_2410_05408_amd import workloads as W
    say("case: domain errors")
    w = W.walker_batch(n_sets=8, n_times=200)
    w.params[W.K, 1] = 0.0
    w.params[W.F, 3] = 1.0
    w.params[W.Q1, 5] = float("nan")
    w.n_ss[6] = 0
    got, st = run(gpu_lib, ctx, w)
    assert st == gpu_lib.GL_ERR_DOMAIN
    bad = [1, 3, 5, 6]
    assert np.all(np.isnan(got[bad]))
    good = [0, 2, 4, 7]
    ref = oracle.flux_batch(w.params[:, good], w.times, n_ss=w.n_ss[good], t_exp=w.t_exp[good])
    assert np.abs(got[good] - ref).max() <= TOL
    # the flag is cleared by the read
    w2 = W.walker_batch(n_sets=2, n_times=10)
    _, st2 = run(gpu_lib, ctx, w2)
    assert st2 == gpu_lib.GL_OK


def test_bad_csr_offsets_are_reported(gpu_lib, ctx):
    import torch
    say("case: bad CSR offsets")
    gl = gpu_lib
    params = torch.tensor(np.tile([[0.1], [0.3], [1.0], [0.5], [0.2], [200.0], [500.0], [0.0],
                                   [0.4], [0.3]], (1, 3)), device="cuda")
    times = torch.linspace(-0.3, 0.3, 30, dtype=torch.float64, device="cuda")
    out = torch.full((30,), -7.0, dtype=torch.float64, device="cuda")
    offsets = torch.tensor([0, 20, 10, 30], dtype=torch.int64, device="cuda")
    gl.gl_lightcurve_batch(ctx.handle, params, times, out, offsets=offsets)
    torch.cuda.synchronize()
    assert gl.gl_ctx_sync_status(ctx.handle) == gl.GL_ERR_DOMAIN
    # the valid first and last segments are computed, nothing outside is written
    o = out.cpu().numpy()
    assert np.all(o[:20] <= 1.0) and np.all(o[20:30] <= 1.0)


def test_host_checked_errors(gpu_lib, ctx):
    import torch
    gl = gpu_lib
    L = gl.lib()
    t = torch.zeros(4, dtype=torch.float64, device="cuda")
    assert L.gl_lightcurve_batch(ctx.handle, None, 1, gl._ptr(t), None, 4, None, None,
                                 gl._ptr(t), None) == gl.GL_ERR_NULL
    assert L.gl_lightcurve_batch(ctx.handle, gl._ptr(t), 0, gl._ptr(t), None, 4, None, None,
                                 gl._ptr(t), None) == gl.GL_ERR_SIZE
    assert L.gl_lightcurve_batch(ctx.handle, gl._ptr(t), 1, gl._ptr(t), None, 0, None, None,
                                 gl._ptr(t), None) == gl.GL_ERR_SIZE
    assert "n_times" in gl.gl_ctx_last_error(ctx.handle)


def test_deterministic_and_graph_equals_direct(gpu_lib, ctx):
    import torch
    from paper_2410_05408_amd import workloads as W
    say("case: determinism, graph replay vs direct launch")
    gl = gpu_lib
    w = W.walker_batch(n_sets=256)
    d = gl.to_device(w, "cuda:0")
    outs = []
    for graph in (True, True, True, False):
        gl.gl_ctx_set_graph(ctx.handle, graph)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            o = ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"])
        s.synchronize()
        outs.append(o.cpu().numpy())
    gl.gl_ctx_set_graph(ctx.handle, True)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_graph_replays_with_eager_work_between(gpu_lib, ctx):
    import torch
    from paper_2410_05408_amd import workloads as W
    say("case: repeated graph replays on one stream with eager work between")
    gl = gpu_lib
    w = W.walker_batch(n_sets=128)
    d = gl.to_device(w, "cuda:0")
    s = torch.cuda.Stream()
    out = torch.empty(w.n_out, dtype=torch.float64, device="cuda")
    first = None
    for r in range(5):
        with torch.cuda.stream(s):
            out.fill_(-1.0)
            gl.gl_lightcurve_batch(ctx.handle, d["params"], d["times"], out, n_ss=d["n_ss"],
                                   t_exp=d["t_exp"], stream=s)
            junk = torch.randn(1000, device="cuda").sum()  # noqa: F841
        s.synchronize()
        cur = out.cpu().numpy()
        if first is None:
            first = cur
        assert np.array_equal(cur, first), r


def test_persistent_grid_sizes_agree(gpu_lib, ctx):
    from paper_2410_05408_amd import workloads as W
    say("case: persistent grid sizes give identical results")
    gl = gpu_lib
    w = W.walker_batch(n_sets=64)
    res = []
    for wpc in (1, 4, 32, 8):
        gl.gl_ctx_set_plan(ctx.handle, wpc)
        got, st = run(gl, ctx, w)
        assert st == gl.GL_OK
        res.append(got)
    assert gl.gl_ctx_get_plan(ctx.handle) == 8
    for r in res[1:]:
        assert np.array_equal(r, res[0])


def test_autotune_keeps_results(gpu_lib, ctx):
    import torch
    from paper_2410_05408_amd import workloads as W
    say("case: autotune")
    gl = gpu_lib
    w = W.walker_batch(n_sets=512)
    d = gl.to_device(w, "cuda:0")
    before, _ = run(gl, ctx, w)
    out = torch.empty(w.n_out, dtype=torch.float64, device="cuda")
    gl.gl_autotune(ctx.handle, d["params"], d["times"], out, n_ss=d["n_ss"], t_exp=d["t_exp"])
    wpc = gl.gl_ctx_get_plan(ctx.handle)
    plan = gl.gl_ctx_get_stage_plan(ctx.handle)
    say(f"  tuned waves/CU {wpc}, stage plan (classify, hard, trapezoid, arcs) {plan}")
    assert plan[1] == wpc
    after, _ = run(gl, ctx, w)
    assert np.array_equal(before, after)
    # any plan gives the same results bit for bit (grid sizes only move work)
    gl.gl_ctx_set_stage_plan(ctx.handle, 8, 4, 6, 12)
    assert gl.gl_ctx_get_stage_plan(ctx.handle) == (8, 4, 6, 12)
    other, _ = run(gl, ctx, w)
    assert np.array_equal(before, other)
    with pytest.raises(gl.GLError):
        gl.gl_ctx_set_stage_plan(ctx.handle, 0, 16, 16, 20)
    gl.gl_ctx_set_stage_plan(ctx.handle, *plan)


def test_work_list_overflow_paths(gpu_lib, ctx, oracle):
    """Tiny work-list capacities: chunks that do not fit go to the fused
    kernel, arcs that do not fit are integrated in place; results agree with
    the oracle and (to rounding) with the default capacities."""
    from paper_2410_05408_amd import workloads as W
    gl = gpu_lib
    w = W.adversarial_batch(n_dense=40)
    ref_gpu, st = run(gl, ctx, w)
    assert st == gl.GL_OK
    ref = oracle.flux_batch(w.params, w.times, offsets=w.offsets, n_ss=w.n_ss, t_exp=w.t_exp)
    try:
        for caps in ((64, 64, 64), (4000, 200, 100), (200000, 5000, 300), (200000, 20000, 20000)):
            say(f"case: capacities sub/hard/arc = {caps}")
            gl.gl_ctx_set_capacity(ctx.handle, *caps)
            got, st = run(gl, ctx, w)
            assert st == gl.GL_OK
            d_def = np.abs(got - ref_gpu).max()
            d_orc = np.abs(got - ref).max()
            say(f"  vs default capacities {d_def:.2e}, vs oracle {d_orc:.2e}")
            assert d_orc <= TOL
            assert d_def <= 1e-12
    finally:
        gl.gl_ctx_set_capacity(ctx.handle, 0, 0, 0)


def test_census_classes_add_up(gpu_lib, ctx):
    import torch
    from paper_2410_05408_amd import workloads as W
    gl = gpu_lib
    say("case: census of a walker batch")
    w = W.walker_batch(n_sets=256)
    d = gl.to_device(w, "cuda:0")
    out = torch.empty(w.n_out, dtype=torch.float64, device="cuda")
    c = gl.gl_census(ctx.handle, d["params"], d["times"], out, n_ss=d["n_ss"], t_exp=d["t_exp"])
    say(f"  {c}")
    assert c["sub_in_window"] == c["whole_on_star"] + c["intersecting"] + c["off_star_in_window"]
    assert c["gk21_pieces"] >= c["ellipse_arcs"] >= c["intersecting"] > 0
    assert c["limb_arcs"] == c["intersecting"]
    ref = ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"])
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_stage_timing(gpu_lib, ctx):
    import torch
    from paper_2410_05408_amd import workloads as W
    gl = gpu_lib
    say("case: per-stage timing events")
    w = W.walker_batch(n_sets=128)
    d = gl.to_device(w, "cuda:0")
    ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"])  # sizes the lists
    gl.gl_ctx_set_timing(ctx.handle, 3)
    for _ in range(3):
        ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"])
    st, n = gl.gl_ctx_get_stage_timing(ctx.handle)
    gl.gl_ctx_set_timing(ctx.handle, 0)
    torch.cuda.synchronize()
    say(f"  {n} batches: {st}")
    assert n == 3 and len(st) == gl.GL_NSTAGES
    assert all(v >= 0.0 for v in st.values()) and st["trapezoid"] > 0.0
    # timed launches (trapezoid stage forked as in the graph) give the same
    # outputs as untimed ones, and the first-to-last times hold every stage
    ref = ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"]).cpu().numpy()
    gl.gl_ctx_set_timing(ctx.handle, 2)
    outs = [ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"]).cpu().numpy() for _ in range(2)]
    comp, pipe, n2 = gl.gl_ctx_get_timing(ctx.handle)
    gl.gl_ctx_set_timing(ctx.handle, 0)
    say(f"  compute {comp / n2:.4f} ms, pipeline {pipe / n2:.4f} ms per batch")
    assert n2 == 2 and 0.0 < comp <= pipe
    for o in outs:
        assert np.array_equal(o, ref)


def test_stage_timing_graph(gpu_lib, ctx):
    """Timing on a stream that takes the graph path: timed batches run
    directly with the graph's stream overlap, outputs are unchanged, every
    batch is timed, and the graph path resumes afterwards."""
    import torch
    from paper_2410_05408_amd import workloads as W
    gl = gpu_lib
    say("case: per-stage timing events on a non-default stream (graph path)")
    w = W.walker_batch(n_sets=256)
    d = gl.to_device(w, "cuda:0")
    s = torch.cuda.Stream()
    ref = ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"], stream=s)
    s.synchronize()
    ref = ref.cpu().numpy()
    gl.gl_ctx_set_timing(ctx.handle, 3)
    outs = []
    for _ in range(3):
        o = ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"], stream=s)
        s.synchronize()
        outs.append(o.cpu().numpy())
    st, n = gl.gl_ctx_get_stage_timing(ctx.handle)
    gl.gl_ctx_set_timing(ctx.handle, 2)
    for _ in range(2):
        ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"], stream=s)
    comp, pipe, n2 = gl.gl_ctx_get_timing(ctx.handle)
    gl.gl_ctx_set_timing(ctx.handle, 0)
    after = ctx.batch(d["params"], d["times"], n_ss=d["n_ss"], t_exp=d["t_exp"], stream=s)
    s.synchronize()
    say(f"  {n} batches: {st}; compute {comp / n2:.4f} ms, pipeline {pipe / n2:.4f} ms per batch")
    assert n == 3 and n2 == 2
    assert all(v >= 0.0 for v in st.values()) and st["trapezoid"] > 0.0 and st["hard"] > 0.0
    assert 0.0 < comp <= pipe
    for o in outs + [after.cpu().numpy()]:
        assert np.array_equal(o, ref)
