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


# --------------------------------------------------------------------------
# source ranges of the open-loop draws, and the partitioned driver
# --------------------------------------------------------------------------
def test_open_loop_source_ranges_cover_the_full_draw():
    cfg = dict(W.ALPHA_BRAIN_SHARE, n_src_exc=40000, n_src_inh=10000, src_rate_hz=80.0, seed=4)
    full = oracle.open_loop_spikes(cfg, 13, 10)
    cuts = [0, 1, 17000, 17001, 33333, 50000]
    parts = [oracle.open_loop_spikes(cfg, 13, 10, s_lo=a, s_hi=b) for a, b in zip(cuts, cuts[1:])]
    for (s, l), a, b in zip(parts, cuts, cuts[1:]):
        assert np.all((s >= a) & (s < b))
    src, lag = oracle._merge_lag_src(parts)
    assert np.array_equal(src, full[0]) and np.array_equal(lag, full[1])


@pytest.mark.parametrize("model,n,k,parts", [(0, 60, 12, 1), (0, 60, 12, 4), (1, 90, 20, 7)])
def test_partitioned_closed_loop_equals_single_oracle(model, n, k, parts):
    cfg = W.tiny(model=model, n=n, k=k, seed=31, d_lo=4, d_hi=9)
    one = oracle.Net(cfg)
    st, idx = one.simulate(347)
    assert len(st) > 20
    part = oracle.Partitioned(cfg, parts, threads=3)
    pst, pid = part.simulate(100)
    pst2, pid2 = part.simulate(247)
    assert np.array_equal(np.concatenate([pst, pst2]), st)
    assert np.array_equal(np.concatenate([pid, pid2]), idx)
    ps, os_ = part.state(), one.state()
    for key in ("V", "y1", "y2", "r"):
        assert np.array_equal(ps[key], os_[key])
    assert np.array_equal(part.ring(), one.ring())
    part.close()


def test_partitioned_open_loop_target_subset():
    cfg = _open_cfg(seed=17)
    one = oracle.Net(dict(cfg, tgt_hi=250))
    st, idx = one.simulate(123)
    assert len(st) > 10
    part = oracle.Partitioned(cfg, 3, threads=3, targets=250)
    pst, pid = part.simulate(123)
    assert np.array_equal(pst, st) and np.array_equal(pid, idx)
    assert np.array_equal(part.ring(), one.ring())
    part.close()
    with pytest.raises(ValueError):
        oracle.Partitioned(W.tiny(model=0, n=40, k=8), 2, targets=20)


def test_partitioned_set_state_and_kicked_realizations():
    """The partitioned oracle's set_state splits the arrays over its ranges
    (a kicked start gives the single oracle's kicked run), and a kicked
    start is a different realization of the same net."""
    from helpers import kicked

    cfg = W.tiny(model=0, n=200, k=40, seed=12, d_lo=4, d_hi=9)
    one = oracle.Net(cfg)
    V = kicked(one.state()["V"], 3)
    assert (V != one.state()["V"]).sum() == 20
    one.set_state(V=V)
    st, idx = one.simulate(400)
    part = oracle.Partitioned(cfg, 4, threads=2)
    part.set_state(V=V)
    pst, pid = part.simulate(400)
    part.close()
    assert np.array_equal(pst, st) and np.array_equal(pid, idx)
    st0, idx0 = oracle.Net(cfg).simulate(400)
    assert len(st0) > 100
    assert not (np.array_equal(st0, st) and np.array_equal(idx0, idx))
