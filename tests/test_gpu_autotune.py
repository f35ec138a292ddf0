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
