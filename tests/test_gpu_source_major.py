"""The source-major layout on the GPU: tables, delivery and dynamics against
the oracle, identity with the block-major layout, the spill path of the
binning pass, and the one-GPU share of the brain-scale network (1.27e10
synapses) on a target sample.

Both layouts add every weight of a delivery into a 64-bit fixed-point LDS
window with the same quantum (exact integer sums, in any order) and round
each window cell to FP32 once, so rings, spikes and state are identical
between the layouts, and between binning regions of any size.
"""
import numpy as np
import pytest

import oracle
from paper_2109_12855_amd import sdeliver
from paper_2109_12855_amd import workloads as W

from helpers import spike_exact
from test_gpu_parity import _dev, _replay_check, _tiny_cases

pytestmark = pytest.mark.gpu

SM = sdeliver.SD_LAYOUT_SOURCE


def _sorted_segments(row, tgt, dly, w):
    out = []
    for s in range(len(row) - 1):
        a, b = row[s], row[s + 1]
        out.append(sorted(zip(tgt[a:b].tolist(), dly[a:b].tolist(),
                              np.float32(w[a:b]).tolist())))
    return out


@pytest.mark.parametrize("case", [0, 2, 4])
@pytest.mark.parametrize("wform", [0, 2, 3])
def test_connections_match_oracle(case, wform):
    cfg = dict(_tiny_cases()[case], wform=wform, layout=SM)
    net = sdeliver.Net(cfg).build()
    assert net.sizes["layout"] == SM
    row, tgt, dly, w = net.connections()
    ref = oracle.Net(dict(cfg, wform=W.ORACLE_WFORM[wform]))
    orow, otgt, odly, ow = ref.source_major()
    assert np.array_equal(row, orow)
    assert _sorted_segments(row, tgt, dly, w) == _sorted_segments(orow, otgt, odly, ow)


@pytest.mark.parametrize("case", range(5))
def test_replay_delivery(case):
    cfg = dict(_tiny_cases()[case], layout=SM)
    n = cfg["n_exc"] + cfg["n_inh"]
    src, lag = W.replay_spikes(n, max(1, n // 3), cfg["d_min"], seed=case)
    _replay_check(cfg, src, lag)


# 300,000 targets: more than one target part (parts hold at most 2^18
# targets), a block straddling the parts' boundary, and at in-degree 10 most
# (spike, part) segments hold zero or one synapse.
TWO_PARTS = W.tiny(model=1, n=300_000, k=10, seed=12, d_lo=10, d_hi=20)


def test_two_target_parts_replay():
    """Counts exact, weights within 1e-6 sum|w| per cell and every event
    delivered, for 30,000 replayed spikes, against the full oracle."""
    cfg = dict(TWO_PARTS, layout=SM)
    n = cfg["n_exc"] + cfg["n_inh"]
    src, lag = W.replay_spikes(n, 30_000, cfg["d_min"], seed=13)
    _replay_check(cfg, src, lag)


def test_two_target_parts_closed_loop():
    cfg = dict(TWO_PARTS, record_spikes=1, layout=SM)
    net = sdeliver.Net(cfg).build()
    ras = []
    eps, t_bad, n_cmp, _ = spike_exact(cfg, net, lambda: oracle.Net(cfg), horizon=300,
                                       min_exact=30, raster=ras)
    assert n_cmp > 1000, n_cmp
    # spikes on both sides of the parts' boundary
    idx = ras[0][1]
    assert (idx < (1 << 18)).any() and (idx >= (1 << 18)).any()
    assert net.stats()["overflow"] == 0


@pytest.mark.parametrize("case", [0, 1, 3])
def test_closed_loop_tiny(case):
    cfg = dict(_tiny_cases()[case], record_spikes=1, layout=SM)
    net = sdeliver.Net(cfg).build()
    ras = []
    spike_exact(cfg, net, lambda: oracle.Net(cfg), horizon=400, min_exact=40, raster=ras)
    assert len(ras[0][0]) > 10


def _run(cfg, steps):
    net = sdeliver.Net(dict(cfg, record_spikes=1)).build()
    net.simulate_steps(steps)
    st, idx = net.spikes()
    out = (st, idx, net.state(), net.stats())
    net.close()
    return out


def _same_run(ra, rb):
    (sa, ia, xa, ta), (sb, ib, xb, tb) = ra, rb
    assert len(sa) > 0
    assert np.array_equal(sa, sb) and np.array_equal(ia, ib)
    for k in ("V", "y1", "y2", "r"):
        if k in xa:
            assert np.array_equal(xa[k], xb[k]), k
    for k in ("events_delivered", "spikes_delivered", "spikes_emitted"):
        assert ta[k] == tb[k], k


@pytest.mark.parametrize("cfg,steps", [
    (W.DELTA_SMALL, 1000),
    (W.tiny(model=1, n=2111, k=300, seed=8, d_lo=10, d_hi=20), 600),
])
def test_layouts_identical_dynamics(cfg, steps):
    """Block-major and source-major runs are identical in spikes and state
    (one delay, and delays spread over 10-20 steps)."""
    _same_run(_run(dict(cfg, layout=sdeliver.SD_LAYOUT_BLOCK), steps),
              _run(dict(cfg, layout=SM), steps))


@pytest.mark.parametrize("wform", [0, 2])
def test_spill_path_identical(wform):
    """Regions of 4 records: nearly every event of a delivery takes the
    fixed-point spill path, and the ring equals the one from ample regions
    and the block-major layout's, cell by cell."""
    cfg = dict(W.tiny(model=1, n=2111, k=300, seed=8, d_lo=10, d_hi=20), wform=wform)
    n = cfg["n_exc"] + cfg["n_inh"]
    src, lag = W.replay_spikes(n, 700, cfg["d_min"], seed=5)
    rings, evs = [], []
    for over in (dict(layout=SM, bin_cap=4), dict(layout=SM), dict(layout=sdeliver.SD_LAYOUT_BLOCK)):
        for count in (False, True):
            net = sdeliver.Net(dict(cfg, **over)).build()
            net.set_count_mode(count)
            net.deliver(*_dev(src, lag), 0)
            rings.append(net.ring())
            evs.append(net.stats()["events_delivered"])
            net.close()
    for i in (2, 4):
        assert np.array_equal(rings[0], rings[i]) and np.array_equal(rings[1], rings[i + 1]), i
    assert len(set(evs)) == 1


def test_spill_path_closed_loop():
    """A closed-loop run with regions of 4 records equals the default run."""
    cfg = dict(W.tiny(model=1, n=2111, k=300, seed=8, d_lo=10, d_hi=20), layout=SM)
    _same_run(_run(dict(cfg, bin_cap=4), 300), _run(cfg, 300))


@pytest.mark.parametrize("cfg,n_spikes", [
    (W.tiny(model=1, n=2111, k=300, seed=8, d_lo=10, d_hi=20), 700),
    (dict(W.ALPHA_112K, wform=3), 900),
    (dict(W.ALPHA_112K, wform=0), 900),
])
def test_layouts_identical_rings(cfg, n_spikes):
    """One delivery (weights and counts) into a fresh ring: both layouts
    hold the same exact fixed-point sums, rounded once, so every cell is
    identical."""
    n = cfg["n_exc"] + cfg["n_inh"]
    src, lag = W.replay_spikes(n, n_spikes, cfg["d_min"], seed=n_spikes)
    rings = {}
    for layout in (sdeliver.SD_LAYOUT_BLOCK, SM):
        for count in (False, True):
            net = sdeliver.Net(dict(cfg, layout=layout)).build()
            net.set_count_mode(count)
            net.deliver(*_dev(src, lag), 0)
            rings[(layout, count)] = net.ring()
            ev = net.stats()["events_delivered"]
            net.close()
            rings[(layout, count, "ev")] = ev
    for count in (False, True):
        a, b = rings[(sdeliver.SD_LAYOUT_BLOCK, count)], rings[(SM, count)]
        assert np.array_equal(a, b), count
        assert rings[(sdeliver.SD_LAYOUT_BLOCK, count, "ev")] == rings[(SM, count, "ev")]


def _open_loop_small():
    return dict(W.tiny(model=1, n=500, k=100, seed=21, d_lo=10, d_hi=20), n_src_exc=20000,
                n_src_inh=5000, src_rate_hz=8.0, drive_rate_hz=0.0, w_exc=45.6 * 30,
                record_spikes=1)


@pytest.mark.parametrize("layout", [sdeliver.SD_LAYOUT_BLOCK, SM])
def test_open_loop_against_oracle(layout):
    cfg = dict(_open_loop_small(), layout=layout)
    net = sdeliver.Net(cfg).build()
    assert net.sizes["layout"] == layout
    net.prepare_input(300)
    ras = []
    spike_exact(cfg, net, lambda: oracle.Net(cfg), horizon=300, min_exact=30, raster=ras)
    assert len(ras[0][0]) > 5


@pytest.mark.parametrize("layout", [sdeliver.SD_LAYOUT_BLOCK, SM])
def test_open_loop_counts_exact(layout):
    """Count mode: the first input slice's arrivals per cell equal the
    oracle's for the same virtual spikes."""
    cfg = dict(_open_loop_small(), layout=layout)
    net = sdeliver.Net(cfg).build()
    net.set_count_mode(True)
    net.prepare_input(20)
    net.simulate_steps(10)   # slice 0 updated; its input is pending
    net.deliver()            # ... delivered into the window [10, 30)
    got = net.ring(20)
    ref = oracle.Net(dict(cfg, wform=W.ORACLE_WFORM[cfg["wform"]]))
    src, lag = oracle.open_loop_spikes(cfg, 0, 10)
    ref.deliver(src, lag, 0)
    L = cfg["ring_len"]
    exp = ref.counts()[[(10 + s) % L for s in range(20)]]
    assert np.array_equal(got.astype(np.int64), exp.astype(np.int64))
    assert net.stats()["spikes_delivered"] == len(src)


# Target samples of the brain-scale share: across the boundary of the first
# two target parts of 2^18 (its block gets records of both parts), inside a
# part, and the last, ragged block (1,125,000 = 1,255 * 896 + 520).
SHARE_SAMPLES = [(262_144 - 224, 262_144 + 224), (517_000, 517_448), (1_125_000 - 448, 1_125_000)]


def test_brain_share_full_size_sample():
    """The one-GPU share of the brain-scale net at full size (1,125,000
    targets, 10M virtual sources, 1.27e10 synapses): one input slice in
    count mode, compared cell by cell with the oracle on three samples of
    448 targets."""
    cfg = dict(W.ALPHA_BRAIN_SHARE)
    net = sdeliver.Net(cfg).build()
    assert net.n_syn == 1125000 * 11250
    assert net.sizes["layout"] == SM
    net.set_count_mode(True)
    net.prepare_input(20)
    net.simulate_steps(10)
    net.deliver()
    got = net.ring(20)
    src, lag = oracle.open_loop_spikes(cfg, 0, 10, cap=1 << 20)
    assert 60_000 < len(src) < 100_000
    L = cfg["ring_len"]
    for lo, hi in SHARE_SAMPLES:
        ref = oracle.Net(dict(cfg, wform=W.ORACLE_WFORM[cfg["wform"]], tgt_lo=lo, tgt_hi=hi))
        ref.deliver(src, lag, 0)
        exp = ref.counts()[[(10 + s) % L for s in range(20)]]
        assert np.array_equal(got[:, lo:hi].astype(np.int64), exp.astype(np.int64)), (lo, hi)
        del ref
    # every input spike was delivered
    st = net.stats()
    assert st["spikes_delivered"] == len(src)
    assert st["overflow"] == 0


def test_long_open_loop_schedule_is_complete():
    """An input schedule of 523 slices of 10M virtual sources has 6.5e9
    (source, 8-step chunk) draws, more than one dispatch's 2^32 work-items:
    the spikes delivered in the last slices equal the oracle's draws for
    them exactly."""
    cfg = dict(W.ALPHA_BRAIN_SHARE, n_exc=800, n_inh=200, k_exc=80, k_inh=20)
    net = sdeliver.Net(cfg).build()
    net.prepare_input(5230)
    net.simulate_steps(5000)
    s0 = net.stats()["spikes_delivered"]
    net.simulate_steps(30)           # delivers the slices starting at 4990, 5000, 5010
    got = net.stats()["spikes_delivered"] - s0
    net.close()
    src, lag = oracle.open_loop_spikes(cfg, 4990, 30, cap=1 << 21)
    assert len(src) > 200_000
    assert got == len(src)
