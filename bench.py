"""Benchmark: light-curve points per second on one MI355X, exact FP64 path.

Workload: the MCMC-walker batch -- 4096 parameter sets drawn from seed 2,
3000 times at 29.4-min cadence, each output box-averaged over 15 midpoint
sub-samples (12 288 000 outputs, 184 320 000 sub-samples per step).  One step
is one gl_lightcurve_batch call over the whole batch (parameter preparation,
window fill, intersection + quadrature, supersample average), inputs resident
in HBM.  Prints one JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (256 CU x 128 FLOP/clk x 2.4 GHz)
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(w, gpu_out, target_s=10.0):
    """The oracle on a bounded sample of the same workload, all host cores."""
    from oracle import glo
    threads = glo.max_threads()
    n_probe = 16
    t = time.perf_counter()
    glo.flux_batch(w.params[:, :n_probe], w.times, n_ss=w.n_ss[:n_probe], t_exp=w.t_exp[:n_probe],
                   nthreads=threads)
    dt = time.perf_counter() - t
    n = int(min(w.n_sets, max(n_probe, n_probe * target_s / max(dt, 1e-3))))
    sets = np.arange(n)
    t = time.perf_counter()
    ref = glo.flux_batch(w.params[:, sets], w.times, n_ss=w.n_ss[sets], t_exp=w.t_exp[sets],
                         nthreads=threads)
    dt = time.perf_counter() - t
    pts = ref.size
    err = float(np.max(np.abs(gpu_out[sets] - ref)))
    return {"value": pts / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} walkers of the batch, all {w.times.size} outputs each "
                      f"({pts} outputs, {pts * int(w.n_ss[0])} sub-samples), {dt:.1f} s wall",
            "max_abs_err_gpu_vs_oracle": err}


def surrogate_leg(ctx, d, exact_out, exact_ms, n_out, args):
    """Config-5 style: train on samples from the exact kernels, calibrate,
    evaluate the walker batch with exact fallback at 1 ppm."""
    import torch

    from paper_2410_05408_amd import surrogate as S
    t0 = time.perf_counter()
    train = S.Samples(ctx, args.sur_train, seed=5)
    cal = S.Samples(ctx, args.sur_cal, seed=6)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    sur = S.Surrogate(ctx, max_batch=8192, seed=0)
    t0 = time.perf_counter()
    hist = sur.train(train, epochs=args.sur_epochs, log=log)
    t_train = time.perf_counter() - t0
    sur.calibrate(cal)
    zero = S.Surrogate(ctx, max_batch=8192, zero=True)
    zero.calibrate(cal, choose=False)
    del train, cal
    out = torch.empty_like(exact_out)
    sur.lightcurve(d, out)  # warm-up
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        n_sub, n_fb = sur.lightcurve(d, out)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    err = float((out - exact_out).abs().max().item())
    out_z = torch.empty_like(exact_out)
    n_sub_z, n_fb_z = zero.lightcurve(d, out_z)
    torch.cuda.synchronize()
    err_z = float((out_z - exact_out).abs().max().item())
    res = {"value": n_out / (ms * 1e-3), "unit": "points/s", "ms_per_step": ms,
           "speedup_vs_exact": exact_ms / ms, "tol": 1e-6, "max_abs_err_vs_exact": err,
           "sub_samples_in_window": n_sub, "fallback_sub_samples": n_fb,
           "fallback_fraction": n_fb / max(1, n_sub),
           "zero_residual_predictor": {"fallback_fraction": n_fb_z / max(1, n_sub_z),
                                       "max_abs_err_vs_exact": err_z},
           "train_samples": args.sur_train, "calibration_samples": args.sur_cal,
           "epochs": args.sur_epochs, "train_mse_first_last": [hist[0], hist[-1]],
           "data_s": t_data, "train_s": t_train, "dtype": "bf16 mfma / f32 acc + f64"}
    sur.close()
    zero.close()
    return res


def source_digest():
    """SHA-256 over the library's kernel sources (identifies the kernels a
    stored counter measurement belongs to)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2410_05408_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs (FETCH_SIZE and WRITE_SIZE, each scaled by the reading of a plain
    copy of known size), or None when they were taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_walker_batch.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["hbm_bytes_per_launch"]


STAGE_KERNELS = {"window": "k_window_grid", "classify": "k_classify", "trapezoid": "k_trap",
                 "hard": "k_hard", "nested": "k_nested", "arcs": "k_gk<0>, k_gk<1>, k_gk_tail",
                 "combine": "k_combine + k_average"}
# stages whose work is FP64 arithmetic (the others move data)
FLOP_STAGES = ("classify", "trapezoid", "hard", "nested", "arcs")


def stage_flop_split(census, per):
    """Algorithmic FP64 operations of each compute stage (census x per-item
    counts; every census item belongs to exactly one stage)."""
    f = {k: census[k] * per[k] for k in census}
    return {
        "classify": f["sub_in_window"] + f["off_star_in_window"],
        "trapezoid": f["trapezoid_nodes"] + f["whole_on_star"],
        "hard": f["intersecting"] + f["newton_steps"] + f["limb_arcs"] + f["ellipse_arcs"],
        "nested": f["nested_trapezoid_nodes"],
        "arcs": f["gk21_pieces"],
    }


# launches that carry a stage's work: the arc stage is two level kernels of
# about equal length (and a short tail launch), every other FP64 stage is one
STAGE_LAUNCHES = {"arcs": 2}


def rooflines(stage_ms, census, per, n_out, n_in_window_out, n_times):
    """(roofline of the dominant kernel, rooflines of the other stages).  The
    dominant kernel is the FP64 kernel with the longest launch: a stage's time
    divided by the launches that carry its work."""
    flops = sum(census[k] * per[k] for k in census)
    stage_flops = stage_flop_split(census, per)
    dom = max(FLOP_STAGES, key=lambda k: stage_ms[k] / STAGE_LAUNCHES.get(k, 1))
    kern_ms = sum(v for k, v in stage_ms.items() if k != "setup")

    def alu_roof(stage):
        a = stage_flops[stage] / (stage_ms[stage] * 1e-3) / 1e12
        return {"bound": "alu", "kernel": STAGE_KERNELS[stage], "achieved": a,
                "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": a / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": measured_traffic(STAGE_KERNELS[stage]),
                "algorithmic_flop_per_launch": stage_flops[stage], "kernel_ms": stage_ms[stage]}

    # the fill and store phase against HBM: every output out of the transit
    # window is written once (8 B) by the window kernel, which also reads the
    # shared time grid once
    fill_bytes = 8 * (n_out - n_in_window_out) + 8 * n_times
    fill_gbs = fill_bytes / (stage_ms["window"] * 1e-3) / 1e9
    roof = dict(alu_roof(dom), whole_pipeline={
        "algorithmic_flop": flops, "compute_ms": kern_ms,
        "achieved": flops / (kern_ms * 1e-3) / 1e12})
    stages = {
        **{k: alu_roof(k) for k in FLOP_STAGES if k != dom},
        "window": {"bound": "hbm", "kernel": STAGE_KERNELS["window"], "achieved": fill_gbs,
                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fill_gbs / HBM_PEAK_GBS,
                   "traffic": measured_traffic(STAGE_KERNELS["window"]),
                   "algorithmic_bytes_per_launch": fill_bytes, "kernel_ms": stage_ms["window"]}}
    return roof, stages


def copy_calibration(n_bytes=1 << 30, reps=3):
    """A plain device-to-device copy of known size: the HBM byte counters read
    for it (per dispatch) give the scale applied to the compute kernel's."""
    import torch
    a = torch.ones(n_bytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": n_bytes, "bytes_written": n_bytes,
                                           "dispatches": reps}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--sur-train", type=int, default=20_000_000)
    ap.add_argument("--sur-cal", type=int, default=1_000_000)
    ap.add_argument("--sur-epochs", type=int, default=4)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the exact path "
              "shards by walker with no communication between GPUs", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        copy_calibration()
        return

    from paper_2410_05408_amd import gl, workloads

    log("building workload")
    w = workloads.walker_batch()
    dev = "cuda:0"
    d = gl.to_device(w, dev)
    out = torch.empty(w.n_out, dtype=torch.float64, device=dev)
    ctx = gl.Context(0)
    stream = torch.cuda.Stream()

    def step():
        gl.gl_lightcurve_batch(ctx.handle, d["params"], d["times"], out, n_ss=d["n_ss"],
                               t_exp=d["t_exp"], stream=stream)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    stream.synchronize()
    torch.cuda.synchronize()
    if gl.gl_ctx_sync_status(ctx.handle) != gl.GL_OK:
        raise RuntimeError(gl.gl_ctx_last_error(ctx.handle))

    log(f"timed region: {args.steps} steps (graph replay)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    log("stage timing pass (HIP events on the launch stream)")
    gl.gl_ctx_set_timing(ctx.handle, args.steps)
    for _ in range(args.steps):
        step()
    stage_sum, n_timed = gl.gl_ctx_get_stage_timing(ctx.handle)
    gl.gl_ctx_set_timing(ctx.handle, 0)
    stage_ms = {k: v / n_timed for k, v in stage_sum.items()}
    pipe_ms = sum(stage_ms.values())

    log("work census")
    census = gl.gl_census(ctx.handle, d["params"], d["times"], out, n_ss=d["n_ss"],
                          t_exp=d["t_exp"], stream=stream)
    wpc = gl.gl_ctx_get_plan(ctx.handle)
    per = gl.gl_flop_model()
    roof, roof_stages = rooflines(stage_ms, census, per, w.n_out,
                                  census["sub_in_window"] // int(w.n_ss[0]), int(w.times.size))

    got = out.cpu().numpy().reshape(w.n_sets, -1)
    in_transit = int(np.sum(got < 1.0))
    value = w.n_out / (ms_per_step * 1e-3)

    res = {
        "metric": "light-curve points/sec on 1 MI355X: exact (≤1e-9) vs surrogate+fallback (≤1 ppm)",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "walker_batch", "path": "exact", "n_sets": w.n_sets,
                   "n_times": int(w.times.size), "n_ss": int(w.n_ss[0]),
                   "cadence_min": 29.4, "seed": 2},
        "roofline": roof,
        "roofline_stages": roof_stages,
        "stage_ms": stage_ms,
        "sub_samples_per_s": w.n_sub / (ms_per_step * 1e-3),
        "in_transit_points_per_s": in_transit / (ms_per_step * 1e-3),
        "in_transit_points": in_transit,
        "pipeline_ms_direct_launch": pipe_ms,
        "plan": {"waves_per_cu": wpc},
        "census": census,
    }
    if not args.no_surrogate:
        log("surrogate leg: data, training, calibration, gated evaluation")
        res["surrogate"] = surrogate_leg(ctx, d, out, ms_per_step, w.n_out, args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on the host cores)")
        res["cpu_baseline"] = cpu_baseline(w, got)
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
