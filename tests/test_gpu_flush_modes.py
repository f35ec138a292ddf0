"""Blocks of more than half a workgroup (576 and 1024 neurons here) flush
their window rows through the dynamic variant of the slice kernel: neurons
are handed out one at a time from an LDS counter and the updating threads
join after their update.  Smaller blocks give one neuron to each free
thread.

The block size only partitions the targets: window sums are exact integers
per delivery and the Poisson drive is keyed by neuron and step.  So a run
with large blocks must reproduce a run with 256-neuron blocks bit for bit,
in both layouts, and a replay delivery must match the oracle (counts exactly,
the ring within the FP32 accumulation bound).  Both test networks have a
ragged last block.
"""
import numpy as np
import pytest

import oracle
from paper_2109_12855_amd import sdeliver
from paper_2109_12855_amd import workloads as W

from helpers import spike_exact
from test_gpu_parity import _replay_check

pytestmark = pytest.mark.gpu

LAYOUTS = [sdeliver.SD_LAYOUT_BLOCK, sdeliver.SD_LAYOUT_SOURCE]


def _run(cfg, steps):
    net = sdeliver.Net(cfg).build()
    sizes = dict(net.sizes)
    net.simulate_steps(steps)
    st, idx = net.spikes()
    state = net.state()
    stats = net.stats()
    net.close()
    return sizes, st, idx, state, stats


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("bn", [576, 1024])
def test_large_blocks_match_small_blocks(layout, bn):
    cfg = dict(W.tiny(model=1, n=2111, k=300, seed=41, d_lo=3, d_hi=12), record_spikes=1,
               layout=layout)
    zb, sb, ib, xb, tb = _run(dict(cfg, block_neurons=bn), 600)
    zd, sd, idd, xd, td = _run(dict(cfg, block_neurons=256), 600)  # one neuron per free thread
    assert zb["block_neurons"] == bn and zd["block_neurons"] == 256
    assert zb["n_blocks"] * bn > 2111 > (zb["n_blocks"] - 1) * bn  # ragged last block
    assert len(sb) > 50
    assert np.array_equal(sb, sd) and np.array_equal(ib, idd)
    for key in ("V", "r"):
        assert np.array_equal(xb[key], xd[key]), key
    assert tb["events_delivered"] == td["events_delivered"] > 0
    ref_cfg = dict(cfg, block_neurons=bn)
    net = sdeliver.Net(ref_cfg).build()
    eps, t_bad, n_cmp, _ = spike_exact(ref_cfg, net, lambda: oracle.Net(ref_cfg), horizon=600,
                                       min_exact=60)
    net.close()
    assert n_cmp > 50, n_cmp


@pytest.mark.parametrize("wform", [0, 3])
@pytest.mark.parametrize("bn", [576, 1024])
def test_large_blocks_replay(bn, wform):
    cfg = dict(W.tiny(model=1, n=2111, k=300, seed=31, d_lo=2, d_hi=9), wform=wform,
               block_neurons=bn)
    n = cfg["n_exc"] + cfg["n_inh"]
    src, lag = W.replay_spikes(n, 500, cfg["d_min"], seed=5)
    net = _replay_check(cfg, src, lag)
    assert net.sizes["block_neurons"] == bn
    _replay_check(cfg, src, lag, t0=9)
