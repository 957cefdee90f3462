"""Pins of the oracle's batch layout against its per-point definition.

``glo_flux_batch`` and ``glo_flux_select`` walk the library's batch layout
(SoA parameter block, shared grid or CSR segments, per-set supersampling
factor and exposure) and call the per-point flux for each output.  Every GPU
parity test compares against them, so a layout mistake here (a wrong segment
lookup, a shared-grid index taken modulo the wrong length, one set's n_ss or
t_exp applied to another) would hide the same mistake in the kernels.  These
tests rebuild every output from the per-point flux in a plain Python loop that
reads the layout independently (segment bounds straight from the offsets,
parameters column by column) and require bit-for-bit equality: both sides call
the same per-point function, so any difference is a layout difference.

The per-point flux itself (Section 2: the occulted fraction of the
limb-darkened disk, box-averaged over midpoint sub-samples) is pinned in
test_oracle_pins.py.
"""
import math

import numpy as np

from paper_2410_05408_amd import workloads as W


def _ragged_batch():
    """Six parameter sets around their transits with ragged CSR segments,
    two of them empty, and per-set supersampling and exposure."""
    rng = np.random.default_rng(123)
    p = W.draw_params(rng, 6)
    p[W.B] = [0.1, 0.5, 0.2, 0.7, 0.0, 0.3]
    p[W.T0] = [0.0, 0.01, -0.02, 0.0, 0.03, 0.0]
    lengths = [0, 1, 7, 0, 9, 5]
    n_ss = np.array([3, 1, 5, 2, 4, 1], np.int32)
    t_exp = np.array([0.02, 0.0, 0.03, 0.01, 0.015, 0.0])
    t14 = W.full_duration(p[W.K], p[W.B], p[W.ARS], p[W.P])
    segs = []
    for s, n in enumerate(lengths):
        # times spread over ingress, the middle and egress of set s
        segs.append(np.sort(rng.uniform(-0.6, 0.6, n)) * t14[s] + p[W.T0, s])
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    return p, np.concatenate(segs), offsets, n_ss, t_exp


def _per_point(oracle, p, s, t, n_ss, t_exp):
    return oracle.flux(np.ascontiguousarray(p[:, s]), float(t), float(t_exp[s]), int(n_ss[s]))


def test_flux_batch_csr_is_the_per_point_flux(oracle):
    p, times, offsets, n_ss, t_exp = _ragged_batch()
    got = oracle.flux_batch(p, times, offsets=offsets, n_ss=n_ss, t_exp=t_exp)
    assert got.shape == (times.shape[0],)
    want = np.empty_like(got)
    for s in range(p.shape[1]):
        for i in range(int(offsets[s]), int(offsets[s + 1])):
            want[i] = _per_point(oracle, p, s, times[i], n_ss, t_exp)
    assert np.array_equal(got, want)
    # the batch is not trivial: most outputs are in transit and they differ
    assert np.sum(want < 1.0) >= 15 and np.unique(want).size >= 15


def test_flux_select_csr_is_the_per_point_flux(oracle):
    p, times, offsets, n_ss, t_exp = _ragged_batch()
    n = times.shape[0]
    # every segment's first and last output, in scrambled order, with repeats
    sel = []
    for s in range(p.shape[1]):
        if offsets[s + 1] > offsets[s]:
            sel += [int(offsets[s]), int(offsets[s + 1]) - 1]
    sel = np.array(sel + [n - 1, 0, 3, 3], np.int64)[::-1].copy()
    got = oracle.flux_select(p, times, sel, offsets=offsets, n_ss=n_ss, t_exp=t_exp)
    for v, idx in zip(got, sel):
        # the owning set read straight from the offsets: the last s whose
        # segment starts at or before idx and is not empty
        s = max(j for j in range(p.shape[1]) if offsets[j] <= idx < offsets[j + 1])
        assert v == _per_point(oracle, p, s, times[idx], n_ss, t_exp)


def test_flux_batch_and_select_shared_grid(oracle):
    rng = np.random.default_rng(7)
    p = W.draw_params(rng, 3)
    p[W.B] = [0.2, 0.4, 0.6]
    n_ss = np.array([1, 3, 5], np.int32)
    t_exp = np.array([0.0, 0.01, 0.02])
    t14 = float(np.max(W.full_duration(p[W.K], p[W.B], p[W.ARS], p[W.P])))
    times = np.linspace(-0.7 * t14, 0.7 * t14, 11)
    got = oracle.flux_batch(p, times, n_ss=n_ss, t_exp=t_exp)
    assert got.shape == (3, 11)
    for s in range(3):
        for i in range(11):
            assert got[s, i] == _per_point(oracle, p, s, times[i], n_ss, t_exp)
    sel = np.array([32, 0, 11, 10, 21, 22, 5], np.int64)  # flat index s * n_times + i
    got_sel = oracle.flux_select(p, times, sel, n_ss=n_ss, t_exp=t_exp)
    for v, idx in zip(got_sel, sel):
        assert v == got[idx // 11, idx % 11]
    # sets differ, so a set taken from the wrong row would show
    assert len({tuple(np.round(got[s], 12)) for s in range(3)}) == 3


def test_defaults_are_one_subsample_and_no_exposure(oracle):
    rng = np.random.default_rng(9)
    p = W.draw_params(rng, 2)
    times = np.array([-0.05, 0.0, 0.07])
    got = oracle.flux_batch(p, times)
    for s in range(2):
        for i in range(3):
            assert got[s, i] == oracle.flux(np.ascontiguousarray(p[:, s]), times[i], 0.0, 1)


def test_domain_error_stays_in_its_own_set(oracle):
    p, times, offsets, n_ss, t_exp = _ragged_batch()
    p = p.copy()
    p[W.K, 2] = 1.5  # set 2 invalid
    got = oracle.flux_batch(p, times, offsets=offsets, n_ss=n_ss, t_exp=t_exp)
    bad = np.zeros(times.shape[0], bool)
    bad[offsets[2]:offsets[3]] = True
    assert np.all(np.isnan(got[bad])) and not np.any(np.isnan(got[~bad]))
    assert not math.isnan(got[-1])
