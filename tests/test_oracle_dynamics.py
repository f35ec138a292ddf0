"""Pins of the oracle's generation, delivery and update against brute force,
closed forms and invariants (CPU only)."""
import math

import numpy as np
import pytest
import scipy.stats

import oracle
from oracle import brute
from paper_2109_12855_amd import workloads as W


# --------------------------------------------------------------------------
# connection generation
# --------------------------------------------------------------------------
@pytest.mark.parametrize("model,n,k,seed", [(0, 20, 6, 3), (1, 30, 10, 11), (0, 50, 15, 5)])
def test_generation_matches_numpy_philox(model, n, k, seed):
    cfg = W.tiny(model=model, n=n, k=k, seed=seed)
    net = oracle.Net(cfg)
    src, dly, widx = net.target_major()
    bs, bd, bw, _ = brute.connections(cfg)
    assert np.array_equal(src.reshape(n, k), bs)
    assert np.array_equal(dly.reshape(n, k), bd)
    assert np.array_equal(widx.reshape(n, k), bw)


def test_source_major_is_stable_sort():
    cfg = W.tiny(model=1, n=50, k=12, seed=4)
    net = oracle.Net(cfg)
    src, dly, widx = net.target_major()
    row, tgt, sdly, sw = net.source_major()
    order = np.argsort(src, kind="stable")
    K = 12
    assert np.array_equal(tgt, (order // K).astype(np.int32))
    assert np.array_equal(sdly, dly[order])
    assert np.array_equal(row, np.concatenate([[0], np.cumsum(np.bincount(src, minlength=50))]))
    _, _, _, bw = brute.connections(cfg)
    assert np.array_equal(sw, bw.reshape(-1)[order])


def test_fixed_indegree_and_uniformity():
    cfg = dict(W.ALPHA_112K, tgt_lo=1000, tgt_hi=1040)  # 40 targets x 11,250 draws
    net = oracle.Net(cfg)
    src, dly, widx = net.target_major()
    src = src.reshape(40, 11250)
    assert np.all(src[:, :9000] < 90000)
    assert np.all(src[:, 9000:] >= 90000) and np.all(src < 112500)
    # delays uniform over {10..20}
    obs = np.bincount(dly, minlength=21)[10:21]
    assert scipy.stats.chisquare(obs).pvalue > 1e-4
    assert dly.min() == 10 and dly.max() == 20
    # sources uniform over 100 bins of the E population
    h = np.bincount(src[:, :9000].reshape(-1) * 100 // 90000, minlength=100)
    assert scipy.stats.chisquare(h).pvalue > 1e-4
    # weight indices uniform over 64 bins
    hw = np.bincount(widx.astype(np.int64) >> 10, minlength=64)
    assert scipy.stats.chisquare(hw).pvalue > 1e-4


# --------------------------------------------------------------------------
# brute force on tiny networks
# --------------------------------------------------------------------------
@pytest.mark.parametrize("model,n,k,seed,steps", [
    (0, 20, 6, 3, 400), (0, 40, 10, 8, 400), (1, 30, 10, 11, 300), (1, 50, 12, 2, 300),
])
def test_brute_force_spikes_and_ring(model, n, k, seed, steps):
    cfg = W.tiny(model=model, n=n, k=k, seed=seed)
    res = brute.simulate(cfg, steps)
    net = oracle.Net(cfg)
    st, idx = net.simulate(steps)
    got = list(zip(st.tolist(), idx.tolist()))
    assert len(res["spikes"]) > 5, "test net should be active"
    assert got == res["spikes"]
    # ring contents: spikes of complete slices are delivered, the open slice
    # is pending
    d_min = cfg["d_min"]
    t_now = net.t_now
    t_deliv = (t_now // d_min) * d_min
    if t_now % d_min == 0:
        t_deliv = t_now - d_min  # last complete slice is delivered at the next call
    rb_ref, cnt_ref = brute.pending_ring(res, cfg, t_now, t_deliv, cfg["ring_len"])
    assert np.allclose(net.ring(), rb_ref, rtol=0, atol=1e-11)
    assert np.array_equal(net.counts().astype(np.int64), cnt_ref)
    st_o = net.state()
    assert np.allclose(st_o["V"], res["V"], rtol=0, atol=1e-10)
    assert np.array_equal(st_o["r"], res["r"])


@pytest.mark.parametrize("split", [[400], [7, 393], [15, 15, 370], [1, 2, 3, 394], [399, 1]])
def test_slice_boundaries_do_not_matter(split):
    cfg = W.tiny(model=1, n=40, k=10, seed=9, d_lo=4, d_hi=9)
    a = oracle.Net(cfg)
    sa = a.simulate(400)
    b = oracle.Net(cfg)
    parts = [b.simulate(m) for m in split]
    sb = (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]))
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
    assert np.array_equal(a.ring(), b.ring())
    assert np.array_equal(a.state()["V"], b.state()["V"])


# --------------------------------------------------------------------------
# delivery invariants
# --------------------------------------------------------------------------
@pytest.mark.parametrize("wform", [0, 1, 2])
def test_delivered_weight_invariant(wform):
    cfg = W.tiny(model=1, n=200, k=40, seed=21, d_lo=10, d_hi=20, wform=wform)
    net = oracle.Net(cfg)
    out_w, out_deg = net.out_weight()
    src, lag = W.replay_spikes(200, 60, 10, seed=5)
    net.simulate(0)
    wsum, nev = net.deliver(src, lag, 0)
    assert nev == int(out_deg[src].sum())
    assert abs(wsum - out_w[src].sum()) <= 1e-12 * np.abs(out_w[src]).sum()
    rb = net.ring()
    cnt = net.counts()
    assert int(cnt.sum()) == nev
    assert abs(rb.sum() - wsum) <= 1e-12 * np.abs(out_w[src]).sum() + 1e-9


def test_deliver_matches_dense_definition():
    """RB[t0+lag+d][j] += w over the connection multiset, for a replay list."""
    cfg = W.tiny(model=0, n=60, k=15, seed=13, d_lo=5, d_hi=12)
    net = oracle.Net(cfg)
    src_tm, dly_tm, _ = net.target_major()
    _, _, _, w_tm = brute.connections(cfg)
    s, l = W.replay_spikes(60, 50, 5, seed=1)
    net.deliver(s, l, 0)
    ref = np.zeros((32, 60))
    K = 15
    spiking = {}
    for a, b in zip(s.tolist(), l.tolist()):
        spiking.setdefault(a, []).append(b)
    for e in range(60 * K):
        j = e // K
        for lag in spiking.get(int(src_tm[e]), []):
            ref[lag + dly_tm[e], j] += w_tm.reshape(-1)[e]
    assert np.allclose(net.ring(), ref, atol=1e-12)


def test_deliver_rejects_past_arrivals():
    cfg = W.tiny(model=0, n=20, k=5, seed=1, d_lo=3, d_hi=5)
    net = oracle.Net(cfg)
    net.simulate(10)
    with pytest.raises(RuntimeError):
        net.deliver(np.arange(20, dtype=np.uint32), np.zeros(20, np.uint8), 0)


# --------------------------------------------------------------------------
# closed forms of the neuron dynamics
# --------------------------------------------------------------------------
def _isolated(model, **over):
    base = W.tiny(model=model, n=10, k=0, seed=3)
    base.update(k_exc=0, k_inh=0, drive_rate_hz=0.0)
    base.update(over)
    return base


@pytest.mark.parametrize("model", [0, 1])
def test_subthreshold_relaxation(model):
    """No input: V(t) = V_inf + (V0 - V_inf) exp(-t/tau_m), V_inf = E_L + I_e tau_m / C."""
    cfg = _isolated(model, i_e=300.0, e_l=-5.0, v0_lo=-5.0, v0_hi=5.0, v_th=1e9)
    net = oracle.Net(cfg)
    v0 = net.state()["V"].copy()
    vinf = cfg["e_l"] + cfg["i_e"] * cfg["tau_m"] / cfg["c_m"]
    for n in (1, 7, 100, 1000):
        net2 = oracle.Net(cfg)
        net2.simulate(n)
        ref = vinf + (v0 - vinf) * math.exp(-n * cfg["h"] / cfg["tau_m"])
        assert np.allclose(net2.state()["V"], ref, rtol=0, atol=1e-11)


@pytest.mark.parametrize("model", [0, 1])
def test_regular_firing_period(model):
    """Constant suprathreshold current: first spike and inter-spike interval
    from the analytic relaxation, quantised to the grid."""
    cfg = _isolated(model, i_e=600.0, v0_lo=0.0, v0_hi=0.0, v_reset=0.0)
    # V_inf = 600*tau_m/250
    net = oracle.Net(cfg)
    st, idx = net.simulate(3000)
    h, tm = cfg["h"], cfg["tau_m"]
    vinf = cfg["i_e"] * tm / cfg["c_m"]
    ref = int(round(cfg["t_ref"] / h))
    m = math.ceil(tm / h * math.log((vinf - 0.0) / (vinf - cfg["v_th"])))
    expect = []
    t = m - 1
    while t < 3000:
        expect.append(t)
        t += ref + m
    for j in range(10):
        assert st[idx == j].tolist() == expect


def test_alpha_psp_closed_form():
    """A single delivered input of weight w: V(t) = (w e / (C tau_s))
    (e^{-t/tau_m} - e^{-t/tau_s} (1 + a t)) / a^2, a = 1/tau_s - 1/tau_m,
    sampled n steps after arrival; superposed over every synapse."""
    cfg = W.tiny(model=1, n=30, k=4, seed=17, d_lo=3, d_hi=6)
    cfg.update(drive_rate_hz=0.0, v0_lo=0.0, v0_hi=0.0, w_exc=10.0)
    net = oracle.Net(cfg)
    row, tgt, dly, w = net.source_major()
    s = 0
    while row[s + 1] - row[s] < 2:
        s += 1
    net.deliver(np.array([s], np.uint32), np.array([0], np.uint8), 0)
    C, ts, tm, h = cfg["c_m"], cfg["tau_syn"], cfg["tau_m"], cfg["h"]
    a = 1 / ts - 1 / tm

    def psp(t, wt):
        if t <= 0:
            return 0.0
        return wt * math.e / (C * ts) * (math.exp(-t / tm) - math.exp(-t / ts) * (1 + a * t)) / a**2

    for step in range(40):
        net.update(1)
        v = net.state()["V"]
        ref = np.zeros(30)
        for e in range(row[s], row[s + 1]):
            ref[tgt[e]] += psp((step - int(dly[e])) * h, w[e])
        assert np.allclose(v, ref, rtol=0, atol=1e-12)


def test_delta_jump_then_decay():
    cfg = W.tiny(model=0, n=30, k=4, seed=17, d_lo=3, d_hi=6)
    cfg.update(drive_rate_hz=0.0, v0_lo=0.0, v0_hi=0.0)
    net = oracle.Net(cfg)
    row, tgt, dly, w = net.source_major()
    s = 0
    while row[s + 1] - row[s] < 2:
        s += 1
    net.deliver(np.array([s], np.uint32), np.array([1], np.uint8), 0)
    tm, h = cfg["tau_m"], cfg["h"]
    for step in range(30):
        net.update(1)
        ref = np.zeros(30)
        for e in range(row[s], row[s + 1]):
            n = step - (1 + int(dly[e]))
            if n >= 0:
                ref[tgt[e]] += w[e] * math.exp(-n * h / tm)
        # inhibition may drive V below 0; nothing reaches threshold here
        assert np.allclose(net.state()["V"], ref, rtol=0, atol=1e-12)


def test_poisson_drive_statistics():
    cfg = W.tiny(model=0, n=10, k=0, seed=3)
    cfg.update(k_exc=0, k_inh=0, drive_rate_hz=2500.0)
    net = oracle.Net(cfg)
    c = np.array([net.drive_count(j, t) for j in range(10) for t in range(4000)])
    assert abs(c.mean() - 0.25) < 0.01
    assert abs(c.var() - 0.25) < 0.015


def test_open_loop_source_rate():
    cfg = dict(W.ALPHA_BRAIN_SHARE, n_src_exc=80000, n_src_inh=20000, src_rate_hz=8.0)
    s, l = oracle.open_loop_spikes(cfg, 0, 10)
    p = -math.expm1(-8.0 * 1e-4)
    n = 100000 * 10
    assert abs(len(s) - n * p) < 5 * math.sqrt(n * p)
    # (lag, src) order
    key = l.astype(np.int64) * 10**8 + s
    assert np.all(np.diff(key) > 0)


# --------------------------------------------------------------------------
# closed-loop rate against mean-field theory
# --------------------------------------------------------------------------
def _mean_field_rate(c: dict) -> float:
    """Self-consistent stationary rate (Hz) of the delta-synapse balanced
    network in the diffusion approximation (Brunel 2000, J. Comput.
    Neurosci. 8:183, the Siegert first-passage rate of the leaky integrator
    with Gaussian input): 1/nu = t_ref + tau_m sqrt(pi) * integral of
    exp(u^2)(1 + erf u) = erfcx(-u) from (V_reset - mu)/sigma to
    (V_th - mu)/sigma, where mu and sigma^2 sum J*rate*tau_m and
    J^2*rate*tau_m over the Poisson drive and the K_E excitatory (J) and
    K_I inhibitory (-g J) inputs firing at nu.  Written from scipy's
    quadrature, independently of the oracle."""
    from scipy.integrate import quad
    from scipy.optimize import brentq
    from scipy.special import erfcx

    tau, t_ref = c["tau_m"] * 1e-3, c["t_ref"] * 1e-3
    J, g, ke, ki = c["w_exc"], c["g"], c["k_exc"], c["k_inh"]
    nu_x, jx = c["drive_rate_hz"], c["drive_w"]

    def phi(nu):
        mu = tau * (jx * nu_x + nu * (ke * J - ki * g * J))
        sig = math.sqrt(tau * (jx * jx * nu_x + nu * (ke * J * J + ki * (g * J) ** 2)))
        integral, _ = quad(lambda u: erfcx(-u), (c["v_reset"] - mu) / sig, (c["v_th"] - mu) / sig)
        return 1.0 / (t_ref + tau * math.sqrt(math.pi) * integral)

    return brentq(lambda nu: phi(nu) - nu, 1e-3, 1.0 / t_ref - 1e-6)


@pytest.mark.parametrize("over", [
    dict(g=6.0),                                              # stronger inhibition
    dict(drive_rate_hz=2000.0),                               # weaker drive
    dict(w_exc=0.4, drive_w=0.4, drive_rate_hz=5000.0),       # smaller jumps
])
def test_closed_loop_rate_matches_mean_field(over):
    """The oracle's whole closed loop (generation, delivery, Poisson drive,
    exact update with threshold, reset and refractoriness) against theory:
    the population rate over [0.2, 1) s, averaged over three seeds of the
    1,250-neuron delta net (Sec. 2.2's balanced random network), lies within
    8% of the mean-field rate.  Measured: 0.97-1.02 of it at these points.
    Planted in the oracle's parameters, a reset to 0 mV, 10% weaker
    inhibition or half the membrane time constant move the ratio to
    0.51-0.75 or 1.21-1.32 at every point, and a dropped refractory period
    to 1.35-1.44 at the first two (feedback compensates it at the third).
    A point where simulation and the diffusion approximation part (a
    0.5 ms refractory period: 15% above theory) is not used.  CV has no
    such reference and stays unpinned."""
    from helpers import rate_cv

    c = dict(W.DELTA_SMALL, **over)
    n = c["n_exc"] + c["n_inh"]
    rates = []
    for seed in (1, 2, 3):
        st, idx = oracle.Net(dict(c, seed=seed)).simulate(10000)
        rates.append(rate_cv(st, idx, n, 2000, 10000, c["h"])[0])
    ratio = float(np.mean(rates)) / _mean_field_rate(c)
    assert abs(ratio - 1.0) <= 0.08, (rates, ratio)
