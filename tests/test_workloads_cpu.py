"""Host-side checks of the seeded workload generator and the stored fixture."""
import math
import os

import numpy as np

from paper_2410_05408_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_workload_sizes():
    w = W.walker_batch()
    assert (w.n_sets, w.times.shape[0], w.n_out, w.n_sub) == (4096, 3000, 12_288_000, 184_320_000)
    w = W.high_cadence()
    assert (w.n_sets, w.n_out) == (512, 33_554_432)
    assert np.all(w.params[W.F] <= 0.2)
    w = W.uneven_batch()
    assert w.n_sets == 16384 and w.offsets[-1] == w.times.shape[0]
    seg = np.diff(w.offsets)
    assert seg.min() >= 200 and seg.max() <= 20000
    assert set(np.unique(w.n_ss)) <= {1, 5, 15}
    assert np.all(np.diff(w.times[w.offsets[0]:w.offsets[1]]) > 0)


def test_seeded_and_in_prior():
    a, b = W.walker_batch(n_sets=64), W.walker_batch(n_sets=64)
    assert np.array_equal(a.params, b.params)
    p = a.params
    assert np.all((p[W.K] >= 0.05) & (p[W.K] <= 0.12))
    assert np.all((p[W.THETA] >= 0) & (p[W.THETA] <= math.pi))
    assert np.all((p[W.Q1] >= 0) & (p[W.Q1] <= 1))


def test_single_transit_fixture_matches_oracle(oracle):
    w = W.single_transit()
    data = np.loadtxt(os.path.join(HERE, "golden", "single_transit_oracle.txt"))
    assert np.array_equal(data[:, 0], w.times)
    out = oracle.flux_batch(w.params, w.times, n_ss=w.n_ss, t_exp=w.t_exp, tol=1e-14)[0]
    assert np.max(np.abs(out - data[:, 1])) < 1e-15
