"""Persistent slices: several whole slices per cooperative launch, each
block's ring window kept in LDS across them, grid barriers between slices
(Alg. REF, Sec. 3.2; neuron update, Sec. 2.1).

* Count mode makes every ring sum an exact integer, so a persistent run and
  the one-launch-per-slice run must agree bit for bit: rasters, neuron
  state, the ring rows still due and the statistics, also when the two
  modes alternate within one run.
* With weights, a persistent run is compared with the FP64 oracle
  spike-exactly up to a rounding-level tie (tolerance from the measured
  drift), for several nets, weight forms and minimum delays, with
  persistent launches of various lengths and at full size.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from helpers import spike_exact
from paper_2109_12855_amd import sdeliver
from paper_2109_12855_amd import workloads as W

pytestmark = pytest.mark.gpu

NETS = {
    "delta_1000": W.tiny(model=0, n=1000, k=100, seed=6, d_lo=10, d_hi=20),
    "alpha_2111_ragged": W.tiny(model=1, n=2111, k=300, seed=8, d_lo=10, d_hi=20),
    "alpha_300_dmin4": W.tiny(model=1, n=300, k=60, seed=5, d_lo=4, d_hi=9),
    "alpha_2000_dmin1": W.tiny(model=1, n=2000, k=200, seed=9, d_lo=1, d_hi=20),
}


class _Modes:
    """A net whose simulate_steps alternates persistent launches (of up to
    ``per`` slices) and one-launch-per-slice runs, ``chunk`` steps each."""

    def __init__(self, net, per: int, chunk: int):
        self.net, self.per, self.chunk, self.on = net, per, chunk, True

    def simulate_steps(self, n: int):
        while n > 0:
            m = min(n, self.chunk)
            self.net.set_persistent(self.per if self.on else 0)
            self.net.simulate_steps(m)
            self.on = not self.on
            n -= m

    def __getattr__(self, k):
        return getattr(self.net, k)


def _run(cfg, steps, per, chunk=None):
    net = sdeliver.Net(dict(cfg, record_spikes=1)).build()
    net.set_count_mode(True)
    if per:
        if chunk:
            _Modes(net, per, chunk).simulate_steps(steps)
        else:
            net.set_persistent(per)
            net.simulate_steps(steps)
    else:
        net.simulate_steps(steps)
    return net


@pytest.mark.parametrize("name", list(NETS))
@pytest.mark.parametrize("per,chunk", [(64, None), (3, None), (7, 37)])
def test_count_mode_bit_identical(name, per, chunk):
    cfg = NETS[name]
    steps = 300
    a = _run(cfg, steps, 0)
    b = _run(cfg, steps, per, chunk)
    sa, sb = a.spikes(), b.spikes()
    assert len(sa[0]) > 20
    oa, ob = np.lexsort((sa[1], sa[0])), np.lexsort((sb[1], sb[0]))
    assert np.array_equal(sa[0][oa], sb[0][ob]) and np.array_equal(sa[1][oa], sb[1][ob])
    for k, v in a.state().items():
        assert np.array_equal(v, b.state()[k]), k
    rows = cfg["d_max"]
    assert np.array_equal(a.ring(rows), b.ring(rows))
    ta, tb = a.stats(), b.stats()
    for k in ("events_delivered", "spikes_delivered", "spikes_emitted", "overflow"):
        assert ta[k] == tb[k], (k, ta[k], tb[k])
    assert tb["overflow"] == 0
    assert a.t_now == b.t_now == steps
    pa, pb = a.pending(), b.pending()
    ka = np.sort(pa[0].astype(np.int64) * 32 + pa[1])
    kb = np.sort(pb[0].astype(np.int64) * 32 + pb[1])
    assert pa[2] == pb[2] and np.array_equal(ka, kb)


@pytest.mark.parametrize("name", list(NETS))
@pytest.mark.parametrize("wform", [0, 3])
def test_against_oracle(name, wform):
    cfg = dict(NETS[name], wform=wform)
    net = sdeliver.Net(dict(cfg, record_spikes=1)).build()
    net.set_persistent(16)
    eps, t_bad, n_cmp, _ = spike_exact(cfg, net, lambda: oracle.Net(cfg), horizon=400,
                                       min_exact=40)
    assert n_cmp > 20, n_cmp
    assert net.stats()["overflow"] == 0


def test_mixed_modes_against_oracle():
    cfg = dict(W.DELTA_SMALL)
    net = sdeliver.Net(dict(cfg, record_spikes=1)).build()
    eps, t_bad, n_cmp, _ = spike_exact(cfg, _Modes(net, 5, 45), lambda: oracle.Net(cfg),
                                       horizon=500, min_exact=45)
    assert n_cmp > 100, n_cmp
    assert net.stats()["overflow"] == 0


def test_mixed_modes_event_counts():
    """Every delivered slice's events equal the spiking sources'
    out-degrees, across persistent and one-launch-per-slice runs."""
    cfg = dict(W.DELTA_SMALL, record_spikes=1)
    net = sdeliver.Net(cfg).build()
    _Modes(net, 4, 30).simulate_steps(600)
    stats = net.stats()
    st, idx = net.spikes()
    row, _, _, _ = net.connections()
    deg = np.diff(row)
    delivered = st < net.pending()[2]
    assert delivered.sum() > 100
    assert stats["events_delivered"] == int(deg[idx[delivered]].sum())
    assert stats["spikes_delivered"] == int(delivered.sum())
    assert stats["spikes_emitted"] == len(st)


def test_full_size_fp32_against_oracle():
    """The 112,500-neuron net (252 blocks of 448, all resident), FP32 form:
    50 ms spike-exact against the partitioned FP64 oracle."""
    cfg = dict(W.ALPHA_112K, wform=0)
    net = sdeliver.Net(dict(cfg, record_spikes=1)).build()
    net.set_persistent(50)
    eps, t_bad, n_cmp, part = spike_exact(
        cfg, net, lambda: oracle.Partitioned(cfg, 16, threads=16), horizon=500, min_exact=5)
    part.close()
    assert n_cmp > 200, n_cmp
    assert eps < 1e-3
    assert net.stats()["overflow"] == 0


def test_rejects_ineligible_nets():
    tiny = W.tiny(model=0, n=1000, k=100, seed=6, d_lo=10, d_hi=20)
    net = sdeliver.Net(tiny)
    with pytest.raises(sdeliver.SdError) as e:
        net.set_persistent(8)  # before build_connections
    assert e.value.status == sdeliver.SD_ESTATE
    net.close()
    wide = dict(W.tiny(model=0, n=4000, k=100, seed=6, d_lo=2, d_hi=5), block_neurons=2048)
    for cfg in (dict(tiny, layout=sdeliver.SD_LAYOUT_SOURCE), wide, W.plastic(tiny)):
        net = sdeliver.Net(cfg).build()
        with pytest.raises(sdeliver.SdError) as e:
            net.set_persistent(8)
        assert e.value.status == sdeliver.SD_EUNSUPPORTED, cfg.get("name")
        net.set_persistent(0)  # always accepted
        net.close()


def test_barrier_timeout_ends_launch():
    """The timeout path of the grid barrier, forced from the host: with no
    polls allowed, the first workgroup to reach a barrier gives up, every
    workgroup leaves the launch (none waits), and bit 4 of the overflow
    flags reports it; the default limit then runs clean again."""
    cfg = NETS["delta_1000"]
    net = sdeliver.Net(cfg).build()
    net.set_persistent(8)
    net.set_barrier_spin(0)
    net.simulate_steps(8 * cfg["d_min"])
    assert net.stats()["overflow"] & 16
    net.close()
    net = sdeliver.Net(cfg).build()
    net.set_persistent(8)
    net.set_barrier_spin(0)
    net.set_barrier_spin(-1)
    net.simulate_steps(8 * cfg["d_min"])
    assert net.stats()["overflow"] == 0
    net.close()
