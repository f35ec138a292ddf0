"""Pins of the oracle's plastic synapses (CPU only).

Reading of the paper's plasticity discussion (Sec. 6): an excitatory weight is
updated when a presynaptic spike is delivered, from the time of the target's
last spike visible at the synapse (the delay lies on the target side) and the
source's previous spike -- nearest-spike pairs with exponential windows,
potentiation capped at w_max, depression floored at 0; the updated weight is
the one delivered.

Pinned against: an independent dense, target-major, time-stepped brute force
(spikes and every weight); the exponential pair window of scripted pre/post
pairs; invariants (zero amplitudes reproduce the static network exactly,
inhibitory and unpaired weights never change, bounds hold).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2109_12855_amd import workloads as W


def _plastic_tiny(model, n, k, seed, **amp):
    cfg = W.tiny(model=model, n=n, k=k, seed=seed, d_lo=3, d_hi=8)
    return W.plastic(cfg, **amp)


def _source_major_from_target_major(res, n_src):
    src = res["src"].reshape(-1)
    order = np.argsort(src, kind="stable")
    return res["w"].reshape(-1)[order]


@pytest.mark.parametrize("model,n,k,seed,steps", [
    (0, 30, 8, 3, 400), (1, 40, 10, 11, 300), (0, 50, 12, 5, 300),
])
def test_plastic_brute_force(model, n, k, seed, steps):
    cfg = _plastic_tiny(model, n, k, seed, a_plus=0.1, a_minus=0.1, w_max=3.0)
    res = brute.simulate_plastic(cfg, steps)
    net = oracle.Net(cfg)
    st, idx = net.simulate(steps)
    assert len(res["spikes"]) > 20
    assert list(zip(st.tolist(), idx.tolist())) == res["spikes"]
    # every weight: the oracle has delivered every spike of complete slices;
    # spikes of the open slice are pending, and brute force updated their
    # synapses already -- compare after delivering those too
    ps, pl, t0 = net.pending()
    net.deliver(ps, pl, t0)
    w_ref = _source_major_from_target_major(res, n)
    w = net.weights()
    assert np.allclose(w, w_ref, rtol=0, atol=1e-12 * max(1.0, cfg["w_exc"]))
    # something changed, in both directions
    w0 = oracle.Net(dict(cfg, plastic=0)).weights()
    d = w - w0
    assert (d > 0).any() and (d < 0).any()


def test_stdp_window_closed_form():
    """The pair window: a source spike after a target spike (visible at the
    synapse Dt steps earlier) depresses by A- exp(-Dt h / tau-); a target
    spike seen Dt steps after the source's previous spike potentiates by
    A+ exp(-Dt h / tau+) at the next source spike."""
    cfg = W.plastic(W.tiny(model=1, n=10, k=2, seed=2), a_plus=0.3, a_minus=0.2)
    A_p, A_m = cfg["stdp_a_plus"], cfg["stdp_a_minus"]
    tp, tm, h = cfg["stdp_tau_plus"], cfg["stdp_tau_minus"], cfg["h"]
    w0 = cfg["w_exc"]
    for dt in (0, 1, 7, 50, 200, 1000):
        d = 5
        # depression: target spike at 100, visible at 105, source spike at 105 + dt
        got = oracle.stdp_update(cfg, w0, 105 + dt, -1, 100, d)
        assert math.isclose(w0 - got, A_m * math.exp(-dt * h / tm), rel_tol=1e-12)
        # potentiation: previous source spike at 300, target spike at 300 - d + dt
        # (visible at 300 + dt), next source spike long after (no depression left)
        t_last = 300 - d + dt
        if dt > 0:
            got = oracle.stdp_update(cfg, w0, 10**7, 300, t_last, d)
            dep = A_m * math.exp(-(10**7 - t_last - d) * h / tm)
            assert math.isclose(got - w0 + dep, A_p * math.exp(-dt * h / tp), rel_tol=1e-12)
    # a target spike seen exactly at the previous source spike is not a
    # post-after-pre pair (it was depression at that spike)
    assert oracle.stdp_update(cfg, w0, 10**7, 300, 295, 5) <= w0
    # no visible target spike: no change
    assert oracle.stdp_update(cfg, w0, 500, 300, -1, 5) == w0
    # bounds
    assert oracle.stdp_update(dict(cfg, stdp_a_minus=10 * w0), w0, 106, -1, 100, 5) == 0.0
    assert oracle.stdp_update(dict(cfg, stdp_a_plus=10 * w0), w0, 10**7, 300, 296, 5) == \
        cfg["stdp_w_max"]


def test_scripted_pairs_through_delivery():
    """A silent net (no drive, V0 = 0): the target of one synapse is made to
    spike at chosen steps, and its source's spikes are delivered at chosen
    steps; the synapse's weight follows the pair window, every other weight
    of other targets stays put."""
    cfg = W.plastic(W.tiny(model=1, n=20, k=4, seed=9, d_lo=3, d_hi=8, drive_rate_hz=0.0,
                           v0_lo=0.0, v0_hi=0.0), a_plus=0.1, a_minus=0.12)
    net = oracle.Net(cfg)
    row, tgt, dly, w_init = net.source_major()
    # an excitatory source with at least one synapse
    s = next(s for s in range(cfg["n_exc"]) if row[s + 1] > row[s])
    e = int(row[s])
    j, d = int(tgt[e]), int(dly[e])
    A_p, A_m = cfg["stdp_a_plus"], cfg["stdp_a_minus"]
    h, tp, tm = cfg["h"], cfg["stdp_tau_plus"], cfg["stdp_tau_minus"]
    Dmin = cfg["d_min"]

    def fire_target_at(t):
        # advance to step t, then make j cross threshold in step t
        while net.t_now < t:
            net.update(1)
        st = net.state()
        V = st["V"].copy()
        V[j] = 200.0
        net.set_state(V=V)
        spk_t, spk_i = net.update(1)
        assert (t, j) in set(zip(spk_t.tolist(), spk_i.tolist()))

    def deliver_at(t_pre):
        t0 = (t_pre // Dmin) * Dmin
        while net.t_now < t0 + Dmin:
            net.update(1)
        net.deliver(np.array([s], np.uint32), np.array([t_pre - t0], np.uint8), t0)

    fire_target_at(12)                       # visible at the synapse at 12 + d
    deliver_at(12 + d + 4)                   # 4 steps later: depression
    w1 = net.weights()[e]
    assert math.isclose(w_init[e] - w1, A_m * math.exp(-4 * h / tm), rel_tol=1e-12)
    fire_target_at(net.t_now + 3)            # a target spike after that source spike
    t_post = net.t_now - 1
    t_pre1 = 12 + d + 4
    t_pre2 = ((t_post + d) // Dmin + 2) * Dmin + 1
    deliver_at(t_pre2)
    w2 = net.weights()[e]
    pot = A_p * math.exp(-(t_post + d - t_pre1) * h / tp)
    dep = A_m * math.exp(-(t_pre2 - t_post - d) * h / tm)
    assert math.isclose(w2, w1 + pot - dep, rel_tol=1e-12)
    # synapses onto other targets did not change
    others = tgt != j
    assert np.array_equal(net.weights()[others], w_init[others])


def test_zero_amplitudes_reproduce_the_static_net():
    cfg = _plastic_tiny(1, 60, 12, 7, a_plus=0.0, a_minus=0.0)
    a = oracle.Net(cfg)
    b = oracle.Net(dict(cfg, plastic=0))
    sa, sb = a.simulate(300), b.simulate(300)
    assert len(sa[0]) > 20
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
    assert np.array_equal(a.ring(), b.ring())
    assert np.array_equal(a.weights(), b.weights())


def test_inhibitory_static_and_bounds():
    cfg = _plastic_tiny(0, 50, 12, 8, a_plus=0.5, a_minus=0.6, w_max=1.5)
    net = oracle.Net(cfg)
    row, tgt, dly, w0 = net.source_major()
    net.simulate(400)
    w = net.weights()
    src_of = np.repeat(np.arange(len(row) - 1), np.diff(row))
    inh = src_of >= cfg["n_exc"]
    assert np.array_equal(w[inh], w0[inh])
    assert np.all(w[~inh] >= 0) and np.all(w[~inh] <= cfg["stdp_w_max"])
    assert (w[~inh] != w0[~inh]).any()
