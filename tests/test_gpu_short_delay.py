"""The short-minimum-delay workload on the GPU: delays of 1..20 steps, so a
slice is one 0.1 ms step (d_min = 1) and every step ends with a delivery.

Against the oracle on small nets (replay delivery and closed-loop rasters,
both layouts, FP32 and packed records), and at full size (112,500 neurons,
1.27e9 synapses) the block-major and source-major layouts must give the
same spikes: their delivery paths share no table or walk, and both round a
delivery's exact window sums once.
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


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("wform", [0, 3])
def test_replay_one_step_slices(layout, wform):
    cfg = dict(W.tiny(model=1, n=2111, k=300, seed=31, d_lo=1, d_hi=20), wform=wform,
               layout=layout)
    assert cfg["d_min"] == 1
    n = cfg["n_exc"] + cfg["n_inh"]
    src, lag = W.replay_spikes(n, 500, cfg["d_min"], seed=3)
    assert np.all(lag == 0)
    _replay_check(cfg, src, lag)
    _replay_check(cfg, src, lag, t0=9)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_closed_loop_one_step_slices(layout):
    cfg = dict(W.tiny(model=1, n=400, k=80, seed=12, d_lo=1, d_hi=20), record_spikes=1,
               layout=layout)
    net = sdeliver.Net(cfg).build()
    ras = []
    spike_exact(cfg, net, lambda: oracle.Net(cfg), horizon=500, min_exact=50, raster=ras)
    assert len(ras[0][0]) > 10


def test_full_size_layouts_agree():
    """The full short-delay net, 400 one-step slices in each layout."""
    runs = []
    for layout in LAYOUTS:
        net = sdeliver.Net(dict(W.ALPHA_112K_SHORT_DELAY, record_spikes=1,
                                layout=layout)).build()
        net.simulate_steps(400)
        st, idx = net.spikes()
        runs.append((st, idx, net.state()["V"], net.stats()))
        net.close()
    (sa, ia, va, ta), (sb, ib, vb, tb) = runs
    assert len(sa) > 1000
    assert np.array_equal(sa, sb) and np.array_equal(ia, ib)
    assert np.array_equal(va, vb)
    assert ta["events_delivered"] == tb["events_delivered"] > 0
    assert ta["slices"] == 400
