"""Pins of the oracle's open-loop source draws and of its target sampling
(CPU only).

The brain-scale share is checked on the GPU against an oracle that holds a
sample of the targets and is fed the open-loop virtual sources.  Both helpers
are pinned here against something other than themselves:

* the open-loop spikes against an independent numpy-Philox drawing of the
  same definition (word and half selection, counter, threshold, order);
* an oracle holding targets [lo, hi) against the full oracle restricted to
  those targets: table rows, ring buffers and counts after a replay, and
  state, spikes and rings after an open-loop run (in open loop the sample's
  dynamics do not depend on the other targets).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2109_12855_amd import workloads as W


# --------------------------------------------------------------------------
# open-loop virtual sources
# --------------------------------------------------------------------------
@pytest.mark.parametrize("t0,n_steps,rate,seed", [
    (0, 32, 200.0, 77), (5, 32, 200.0, 3), (1003, 32, 120.0, 11), (8, 19, 8.0, 5),
])
def test_open_loop_spikes_match_numpy_philox(t0, n_steps, rate, seed):
    cfg = dict(W.ALPHA_BRAIN_SHARE, n_src_exc=4000, n_src_inh=1000, src_rate_hz=rate, seed=seed)
    s_ref, l_ref = brute.open_loop_spikes(cfg, t0, n_steps)
    s, l = oracle.open_loop_spikes(cfg, t0, n_steps)
    assert len(s_ref) > 0
    assert np.array_equal(s, s_ref) and np.array_equal(l, l_ref)


def test_open_loop_threshold_is_the_bernoulli_probability():
    """At a rate where p * 2^32 is far from an integer, the count over many
    draws matches p = 1 - exp(-rate h) within 5 sd, and a source never fires
    at rate 0."""
    cfg = dict(W.ALPHA_BRAIN_SHARE, n_src_exc=40000, n_src_inh=10000, src_rate_hz=500.0, seed=9)
    s, l = oracle.open_loop_spikes(cfg, 0, 20)
    p = -math.expm1(-500.0 * 1e-4)
    n = 50000 * 20
    assert abs(len(s) - n * p) < 5 * math.sqrt(n * p * (1 - p))
    s0, _ = oracle.open_loop_spikes(dict(cfg, src_rate_hz=0.0), 0, 20)
    assert len(s0) == 0


# --------------------------------------------------------------------------
# target sampling
# --------------------------------------------------------------------------
def _open_cfg(seed=21):
    cfg = W.tiny(model=1, n=400, k=50, seed=seed, d_lo=4, d_hi=9)
    cfg.update(n_src_exc=4000, n_src_inh=1000, src_rate_hz=60.0, w_exc=45.6 * 40.0)
    return cfg


def _restrict(row, tgt, dly, w, lo, hi):
    keep = (tgt >= lo) & (tgt < hi)
    src_of = np.repeat(np.arange(len(row) - 1), np.diff(row))
    counts = np.bincount(src_of[keep], minlength=len(row) - 1)
    return np.concatenate([[0], np.cumsum(counts)]), tgt[keep], dly[keep], w[keep]


@pytest.mark.parametrize("lo,hi", [(0, 1), (100, 220), (397, 400), (0, 400)])
def test_sampled_table_is_the_restricted_table(lo, hi):
    cfg = _open_cfg()
    full = oracle.Net(cfg)
    part = oracle.Net(dict(cfg, tgt_lo=lo, tgt_hi=hi))
    assert part.n_local == hi - lo and part.n_src == full.n_src
    want = _restrict(*full.source_major(), lo, hi)
    got = part.source_major()
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    # the sampled targets' draws are the full net's draws of those targets
    K = cfg["k_exc"] + cfg["k_inh"]
    fs, fd, fw = full.target_major()
    ps, pd, pw = part.target_major()
    assert np.array_equal(ps, fs[lo * K:hi * K]) and np.array_equal(pd, fd[lo * K:hi * K])
    assert np.array_equal(pw, fw[lo * K:hi * K])


def test_sampled_replay_rings_and_counts():
    cfg = _open_cfg(seed=4)
    lo, hi = 150, 260
    full = oracle.Net(cfg)
    part = oracle.Net(dict(cfg, tgt_lo=lo, tgt_hi=hi))
    src, lag = W.replay_spikes(5000, 900, cfg["d_min"], seed=8)
    wf, nf = full.deliver(src, lag, 0)
    wp, np_ = part.deliver(src, lag, 0)
    assert 0 < np_ < nf
    assert np.array_equal(part.counts(), full.counts()[:, lo:hi])
    # the same additions in the same order per cell: bitwise equal
    assert np.array_equal(part.ring(), full.ring()[:, lo:hi])


def test_sampled_open_loop_run():
    cfg = _open_cfg(seed=13)
    lo, hi = 37, 301
    full = oracle.Net(cfg)
    part = oracle.Net(dict(cfg, tgt_lo=lo, tgt_hi=hi))
    fst, fid = full.simulate(230)
    pst, pid = part.simulate(230)
    assert len(fst) > 20, "test net should be active"
    keep = (fid >= lo) & (fid < hi)
    assert np.array_equal(pst, fst[keep]) and np.array_equal(pid, fid[keep])
    fs, ps = full.state(), part.state()
    for k in ("V", "y1", "y2", "r"):
        assert np.array_equal(ps[k], fs[k][lo:hi])
    assert np.array_equal(part.ring(), full.ring()[:, lo:hi])
    assert np.array_equal(part.counts(), full.counts()[:, lo:hi])


def test_sampling_uses_global_target_ids():
    """A sample's draws depend on the global id: two disjoint samples of the
    same size hold different tables, and a sample is not the full net of its
    own size."""
    cfg = _open_cfg(seed=2)
    a = oracle.Net(dict(cfg, tgt_lo=0, tgt_hi=50)).target_major()[0]
    b = oracle.Net(dict(cfg, tgt_lo=50, tgt_hi=100)).target_major()[0]
    assert not np.array_equal(a, b)
