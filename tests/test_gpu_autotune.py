"""Block-size autotuning on the GPU.

The block size only partitions the targets among workgroups: window sums
are exact integers per delivery and the Poisson drive is keyed by neuron
and step, so a network's spikes and state do not depend on it.  The tuned
sizes must therefore reproduce the default-size run bit for bit, and the
JSON cache must return what the timing chose.
"""
import json

import numpy as np
import pytest

from paper_2109_12855_amd import sdeliver
from paper_2109_12855_amd import workloads as W

from test_gpu_batch import _same_members, _small_sweep

pytestmark = pytest.mark.gpu


def test_autotune_batch_and_cache(tmp_path):
    cfgs = _small_sweep(4, seed=17)
    cache = str(tmp_path / "tune.json")
    bn, us = sdeliver.autotune(cfgs, targets=(4, 32, 256), warmup=4, slices=8, cache=cache)
    assert len(bn) == len(cfgs) and us > 0
    assert all(b >= 64 and b % 64 == 0 for b in bn)
    entries = json.load(open(cache))
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.count(":") == 2 and val["block_neurons"] == bn
    # a cache hit returns the stored result
    bn2, us2 = sdeliver.autotune(cfgs, targets=(4, 32, 256), warmup=4, slices=8, cache=cache)
    assert bn2 == bn and abs(us2 - us) <= 1e-3
    assert len(json.load(open(cache))) == 1
    # another problem adds a second entry
    sdeliver.autotune(cfgs[:2], targets=(8, 256), warmup=2, slices=4, cache=cache)
    assert len(json.load(open(cache))) == 2
    # tuned sizes give the default run's results exactly
    tuned = sdeliver.Batch([dict(c, block_neurons=b) for c, b in zip(cfgs, bn)]).build()
    plain = sdeliver.Batch(cfgs).build()
    tuned.simulate_steps(400)
    plain.simulate_steps(400)
    _same_members(tuned, plain, len(cfgs))


def test_autotune_single_network():
    cfg = dict(W.DELTA_SMALL, record_spikes=1)
    (b,), us = sdeliver.autotune([cfg], targets=(2, 8, 32), warmup=4, slices=8)
    assert b % 64 == 0 and us > 0
    runs = []
    for bb in (b, 0):
        net = sdeliver.Net(dict(cfg, block_neurons=bb)).build()
        net.simulate_steps(500)
        runs.append((net.spikes(), net.state()))
        net.close()
    (sa, ia), xa = runs[0]
    (sb, ib), xb = runs[1]
    assert len(sa) > 0 and np.array_equal(sa, sb) and np.array_equal(ia, ib)
    assert np.array_equal(xa["V"], xb["V"])


def _block_for(cfg, T):
    """The block size sd_autotune derives from a target of T blocks."""
    n = cfg["n_exc"] + cfg["n_inh"]
    b = -(-n // T)
    b = max(64, -(-b // 64) * 64)
    while b >= 64:
        try:
            sdeliver.query_sizes(cfg, block_neurons=b)
            return b
        except sdeliver.SdError:
            b -= 64
    return 0


def test_autotune_bins_source_major(tmp_path):
    """Block size and region capacity of a source-major open-loop network:
    the result is one of the candidate pairs, the cache returns it, and the
    tuned network's run equals the default one bit for bit (block size and
    region capacity only partition the work: window sums are exact
    integers, and events past a small region take the exact spill path)."""
    cfg = dict(W.tiny(model=1, n=20000, k=500, seed=5, d_lo=10, d_hi=20), n_src_exc=160000,
               n_src_inh=40000, src_rate_hz=8.0, drive_rate_hz=0.0, w_exc=45.6 * 10,
               layout=sdeliver.SD_LAYOUT_SOURCE, record_spikes=1)
    targets, scales = (20, 40), (0.25, 1.0)
    cache = str(tmp_path / "bins.json")
    bn, cap, us = sdeliver.autotune_bins(cfg, targets=targets, cap_scales=scales, warmup=3,
                                         slices=6, cache=cache)
    assert us > 0
    cands = set()
    for T in targets:
        b = _block_for(cfg, T)
        c0 = sdeliver.query_sizes(cfg, block_neurons=b)["bin_cap"]
        for f in scales:
            c = min(1024, max(64, -(-int(np.ceil(f * c0)) // 64) * 64))
            cands.add((b, c))
    assert (bn, cap) in cands, (bn, cap, cands)
    entries = json.load(open(cache))
    (key, val), = entries.items()
    assert ":bins:" in key and val["bin_cap"] == cap and val["block_neurons"] == [bn]
    assert sdeliver.autotune_bins(cfg, targets=targets, cap_scales=scales, warmup=3, slices=6,
                                  cache=cache)[:2] == (bn, cap)
    runs = []
    for over in (dict(block_neurons=bn, bin_cap=cap), dict(block_neurons=_block_for(cfg, 40),
                                                           bin_cap=64), {}):
        net = sdeliver.Net(dict(cfg, **over)).build()
        net.prepare_input(400)
        net.simulate_steps(400)
        runs.append((net.spikes(), net.state()["V"]))
        net.close()
    for (s, i), v in runs[1:]:
        assert len(runs[0][0][0]) > 20
        assert np.array_equal(s, runs[0][0][0]) and np.array_equal(i, runs[0][0][1])
        assert np.array_equal(v, runs[0][1])
