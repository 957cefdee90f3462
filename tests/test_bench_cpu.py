"""CPU: the host arithmetic of bench.py (FLOP split, roofline fields) and
its one-GPU guard.  No GPU and no library calls."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2410_05408_amd import gl  # noqa: E402


def _census_and_per():
    # distinct counts and distinct per-item costs (powers of two apart), so a
    # census item dropped from the split or counted twice changes the sum
    census = {k: 3 + 7 * i for i, k in enumerate(gl.CENSUS_NAMES)}
    per = {k: 1 << (2 * i) for i, k in enumerate(gl.CENSUS_NAMES)}
    per["unconverged_arcs"] = 0  # their pieces are already counted as pieces
    return census, per


def test_stage_flop_split_counts_every_item_once():
    census, per = _census_and_per()
    split = bench.stage_flop_split(census, per)
    assert set(split) == set(bench.FLOP_STAGES)
    assert sum(split.values()) == sum(census[k] * per[k] for k in census)


def test_rooflines_pick_the_longest_launch_and_rate_it():
    census, per = _census_and_per()
    stage_ms = {"setup": 0.01, "window": 0.03, "classify": 0.04, "trapezoid": 0.09, "hard": 0.05,
                "arcs": 0.16, "nested": 0.01, "combine": 0.03, "fused": 0.006}
    roof, stages = bench.rooflines(stage_ms, census, per, n_out=1000, n_in_window_out=100, n_times=10,
                                   step_ms=0.25)
    split = bench.stage_flop_split(census, per)
    # the arc stage is two launches (0.08 ms each), so the trapezoid's 0.09 ms is the longest
    assert roof["kernel"] == bench.STAGE_KERNELS["trapezoid"]
    a = split["trapezoid"] / (0.09e-3) / 1e12
    assert roof["achieved"] == pytest.approx(a)
    assert roof["frac"] == pytest.approx(a / bench.FP64_VECTOR_PEAK_TFLOPS)
    assert roof["bound"] == "alu" and roof["unit"] == "TFLOP/s" and roof["peak"] == 78.6
    assert roof["whole_pipeline"]["step_ms"] == 0.25
    assert roof["whole_pipeline"]["achieved"] == pytest.approx(
        sum(census[k] * per[k] for k in census) / 0.25e-3 / 1e12)
    arcs = stages["arcs"]
    assert arcs["launches_per_step"] == 2 and arcs["kernel_ms"] == pytest.approx(0.08)
    assert arcs["algorithmic_flop_per_launch"] == pytest.approx(split["arcs"] / 2)
    # the window stage against HBM: the out-of-window outputs (8 B each) and
    # the shared grid's times once
    win = stages["window"]
    assert win["bound"] == "hbm" and win["algorithmic_bytes_per_launch"] == 8 * 900 + 8 * 10
    assert "trapezoid" not in stages and set(stages) == set(bench.FLOP_STAGES) - {"trapezoid"} | {"window"}


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
