"""Batched networks (parameter sweep) on the GPU.

A batch advances independent networks together, one fused launch per slice
over the union of their blocks.  Every member runs the same per-block code
as a single context and the delivery sums are exact integers, so a member's
spikes and state must equal those of the same network run alone, bit for
bit; the single-network path itself is checked against the oracle in
test_gpu_parity.py.
"""
import numpy as np
import pytest

from paper_2109_12855_amd import sdeliver
from paper_2109_12855_amd import workloads as W

pytestmark = pytest.mark.gpu


def _small_sweep(n_nets, seed, wform=0):
    """sweep_nets parameters with sizes cut down for quick runs."""
    out = []
    rng = np.random.default_rng(seed)
    for i, c in enumerate(W.sweep_nets(n_nets, seed=seed, wform=wform)):
        n = int(rng.integers(1000, 6001))
        k = int(rng.integers(100, 801))
        n_e, k_e = int(round(0.8 * n)), int(round(0.8 * k))
        j = 0.8 * np.sqrt(100.0 / k_e)
        eta = float(rng.choice([1.5, 2.0, 3.0]))
        out.append(dict(c, name=f"small_{i}", n_exc=n_e, n_inh=n - n_e, k_exc=k_e, k_inh=k - k_e,
                        w_exc=j, drive_w=j,
                        drive_rate_hz=W._delta_drive(eta, 20.0, j, k_e, 20.0), record_spikes=1))
    return out


def _alone(cfg, splits):
    net = sdeliver.Net(cfg).build()
    for m in splits:
        net.simulate_steps(m)
    st, idx = net.spikes()
    return st, idx, net.state(), net.stats()


def _check_members(bt, cfgs, splits, which=None):
    for i in (which if which is not None else range(len(cfgs))):
        st, idx = bt.members[i].spikes()
        s = bt.members[i].state()
        st1, idx1, s1, stats1 = _alone(cfgs[i], splits)
        assert len(st) > 0, i
        assert np.array_equal(st, st1) and np.array_equal(idx, idx1), i
        for k in ("V", "r"):
            assert np.array_equal(s[k], s1[k]), (i, k)
        stats = bt.members[i].stats()
        for k in ("events_delivered", "spikes_delivered", "spikes_emitted", "slices"):
            assert stats[k] == stats1[k], (i, k)


@pytest.mark.parametrize("wform", [0, 2])
def test_batch_equals_members_alone(wform):
    cfgs = _small_sweep(6, seed=3, wform=wform)
    bt = sdeliver.Batch(cfgs).build()
    bt.simulate_steps(300)
    _check_members(bt, cfgs, [300])


def test_batch_split_calls():
    cfgs = _small_sweep(4, seed=5)
    bt = sdeliver.Batch(cfgs).build()
    for m in (7, 8, 15, 270):
        bt.simulate_steps(m)
    assert all(m.t_now == 300 for m in bt.members)
    _check_members(bt, cfgs, [300])


def test_batch_rejects_mismatched_members():
    a = _small_sweep(2, seed=9)
    b = dict(a[1], d_lo=10, d_hi=10, d_min=10, d_max=10)
    with pytest.raises(sdeliver.SdError) as e:
        sdeliver.Batch([a[0], b])
    assert e.value.status == sdeliver.SD_EINVAL
    with pytest.raises(sdeliver.SdError):
        sdeliver.Batch([a[0], dict(a[1], wform=2)])


def test_batch_single_member():
    cfgs = _small_sweep(1, seed=13)
    bt = sdeliver.Batch(cfgs).build()
    bt.simulate_steps(150)
    _check_members(bt, cfgs, [150])


def _same_members(ga, eb, n):
    for i in range(n):
        sa, ia = ga.members[i].spikes()
        sb, ib = eb.members[i].spikes()
        assert np.array_equal(sa, sb) and np.array_equal(ia, ib), i
        xa, xb = ga.members[i].state(), eb.members[i].state()
        for k in ("V", "y1", "y2", "r"):
            assert np.array_equal(xa[k], xb[k]), (i, k)
        ta, tb = ga.members[i].stats(), eb.members[i].stats()
        for k in ("events_delivered", "spikes_delivered", "spikes_emitted", "slices", "t_now"):
            assert ta[k] == tb[k], (i, k)


def test_batch_graph_equals_eager():
    """Steady-state stretches replayed from the captured graph give the same
    spikes, state and counters as eager launches after every call: partial
    slices, the first delivery, replays of several periods and eager
    remainders alternate, with host read-backs between the calls."""
    cfgs = _small_sweep(4, seed=11)
    ga = sdeliver.Batch(cfgs).build().set_graph(True)
    eb = sdeliver.Batch(cfgs).build()
    d_min = cfgs[0]["d_min"]
    replays = []
    for m in (7, 3, 13 * d_min, 14 * d_min - 2, 5, 4 * d_min, 27 * d_min + 3):
        ga.simulate_steps(m)
        eb.simulate_steps(m)
        _same_members(ga, eb, len(cfgs))
        replays.append(ga.graph_launches)
    assert ga.members[0].stats()["spikes_emitted"] > 0
    # replays happened in several calls, none in the eager batch
    assert len(set(replays)) >= 3 and replays[-1] >= 6, replays
    assert eb.graph_launches == 0


def test_sweep_64_full_size():
    """The 64-network sweep at its full sizes (N up to 40,000, K up to
    5,000), 0.5 s through the captured graph: three members compared with
    their single runs."""
    # raster room for the refractory-limited maximum rate (one spike per
    # 2 ms refractory period + 0.1 ms step) over the run
    cfgs = [dict(c, record_spikes=1, record_cap=(c["n_exc"] + c["n_inh"]) * 260)
            for c in W.sweep_nets(64)]
    bt = sdeliver.Batch(cfgs).build().set_graph(True)
    bt.simulate_steps(5000)
    assert bt.graph_launches >= 50
    n_syn = sum(m.n_syn for m in bt.members)
    assert n_syn > 3e9
    sizes = [c["n_exc"] + c["n_inh"] for c in cfgs]
    which = [int(np.argmin(sizes)), int(np.argmax(sizes)), 17]
    _check_members(bt, cfgs, [5000], which=which)
    for m in bt.members:
        assert m.stats()["overflow"] == 0
