"""Pins of the oracle's RNG, tables and propagators against independent
library routines and closed forms (CPU only)."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.special
import scipy.stats
import torch

import oracle
from oracle import brute
from paper_2109_12855_amd import workloads as W


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (1, 2)),
    ((12345, 678, 0, 0), (2022, 3)),
    ((2**64 - 1, 5, 0, 0), (2**63 + 11, 4)),
    ((0, 1, 0, 0), (99, 1)),
])
def test_philox_matches_numpy(ctr, key):
    """Philox4x64-10 equals numpy's Philox bit generator block for block
    (numpy increments the counter before producing a block)."""
    c = ctr[0] + (ctr[1] << 64) + (ctr[2] << 128) + (ctr[3] << 192)
    prev = (c - 1) % (1 << 256)
    arr = np.array([(prev >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], np.uint64)
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=arr)
    ref = bg.random_raw(4)
    got = oracle.philox4x64_10(ctr, key)
    assert np.array_equal(got, ref)


def test_philox_many_counters():
    rng = np.random.default_rng(0)
    for _ in range(200):
        c0, c1 = (int(x) for x in rng.integers(0, 2**63, size=2))
        seed = int(rng.integers(0, 2**63))
        got = oracle.philox4x64_10((c0, c1, 0, 0), (seed, 3))
        ref = brute.philox_words(seed, 3, c0, c1)
        assert [int(x) for x in got] == ref


def test_ndtri_against_scipy():
    p = np.concatenate([np.linspace(1e-6, 1 - 1e-6, 2001),
                        [1e-300, 1e-100, 1e-20, 1e-10, 0.0250, 0.075, 0.924, 1 - 1e-12],
                        (np.arange(65536) + 0.5) / 65536.0])
    for x in p:
        a = oracle.ndtri(float(x))
        b = float(scipy.special.ndtri(float(x)))
        assert abs(a - b) <= 2e-15 * max(1.0, abs(b)), (x, a, b)


def test_weight_table_quantiles_and_moments():
    cfg = W.ALPHA_112K
    we, wi = oracle.weight_tables(cfg)
    z = scipy.special.ndtri((np.arange(65536) + 0.5) / 65536.0)
    ref_e = (cfg["w_exc"] * (1 + cfg["w_cv"] * z)).astype(np.float32)
    ref_i = (-cfg["g"] * cfg["w_exc"] * (1 + cfg["w_cv"] * z)).astype(np.float32)
    assert np.max(np.abs(we.astype(np.float64) - ref_e)) <= 1e-5 * 45.6
    assert np.max(np.abs(wi.astype(np.float64) - ref_i)) <= 1e-5 * 228.0
    # FP32-rounded quantiles agree bitwise with scipy's except where an FP64
    # last-bit difference straddles an FP32 rounding boundary
    assert np.mean(we == ref_e) > 0.999
    # discretised N(45.6, 2.28): moments of the midpoint quantiles
    assert abs(we.astype(np.float64).mean() - 45.6) < 1e-4
    assert abs(we.astype(np.float64).std() / 45.6 - 0.05) < 1e-3
    assert np.all(np.diff(we) >= 0)
    assert np.allclose(wi, -5.0 * we, rtol=1e-6)


@pytest.mark.parametrize("lam", [0.25, 2.0860428, 0.001, 5.0])
def test_poisson_thresholds(lam):
    t = oracle.poisson_thresholds(lam)
    ref = brute.poisson_thresholds(lam)
    assert len(t) == len(ref)
    # recurrence vs scipy's cdf: within a few units of 2^-32 resolution
    assert np.max(np.abs(t.astype(np.int64) - np.array(ref, np.int64))) <= 4
    # the count map reproduces the Poisson pmf on a fine grid of u
    u = np.arange(0, 2**32, 2**12, dtype=np.uint64)
    counts = (u[:, None] >= t[None, :].astype(np.uint64)).sum(1)
    freq = np.bincount(counts, minlength=len(t) + 1) / len(u)
    pmf = scipy.stats.poisson.pmf(np.arange(len(freq)), lam)
    assert np.max(np.abs(freq - pmf)) < 2e-6


def test_poisson_threshold_values_delta_net():
    # lambda = 0.25: T_0 = floor(2^32 e^-0.25) by hand
    t = oracle.poisson_thresholds(0.25)
    assert int(t[0]) == math.floor(2**32 * math.exp(-0.25))
    assert int(t[1]) == math.floor(2**32 * math.exp(-0.25) * 1.25)


def _expm_mp(cfg):
    """Propagators from a 50-digit matrix exponential (mpmath)."""
    import mpmath
    mpmath.mp.dps = 50
    h, tm, ts, C = (mpmath.mpf(repr(cfg[k])) for k in ("h", "tau_m", "tau_syn", "c_m"))
    A = mpmath.matrix([[-1 / ts, 0, 0, 0], [1, -1 / ts, 0, 0], [0, 1 / C, -1 / tm, 1 / C],
                       [0, 0, 0, 0]])
    P = mpmath.expm(A * h)
    return dict(P11=P[0, 0], P21=P[1, 0], P22=P[1, 1], P31=P[2, 0], P32=P[2, 1], P33=P[2, 2],
                P30=P[2, 3])


@pytest.mark.parametrize("cfg", [W.ALPHA_112K, W.DELTA_SMALL,
                                 dict(W.ALPHA_112K, tau_syn=2.0, tau_m=15.0, h=0.25),
                                 dict(W.ALPHA_112K, tau_syn=0.1, tau_m=30.0, h=1.0)])
def test_propagators_vs_expm(cfg):
    """Closed-form propagators against a high-precision matrix exponential,
    and against scipy's double-precision expm to its own accuracy."""
    P = oracle.propagators(cfg)
    M = _expm_mp(cfg)
    R = brute.propagators(cfg)
    keys = ("P33", "P30") if cfg["model"] == 0 else ("P11", "P21", "P22", "P31", "P32", "P33", "P30")
    for k in keys:
        exact = float(M[k])
        assert abs(P[k] - exact) <= 4e-15 * abs(exact), (k, P[k], exact)
        assert abs(R[k] - exact) <= 1e-13 * abs(exact), (k, R[k], exact)


def test_propagator_values_alpha():
    # tabulated values for C=250 pF, tau_m=10 ms, tau_s=0.32582722 ms, h=0.1 ms
    P = oracle.propagators(W.ALPHA_112K)
    assert abs(P["P11"] - math.exp(-0.1 / 0.32582722)) < 1e-16
    assert abs(P["P33"] - math.exp(-0.01)) < 1e-16
    assert abs(P["P21"] - 0.1 * math.exp(-0.1 / 0.32582722)) < 1e-16
    assert abs(P["P32"] / 3.42639702e-4 - 1) < 1e-8
    assert abs(P["P31"] / 1.62854486e-5 - 1) < 1e-8


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(45.6, 2.28, 20000), -5 * rng.normal(45.6, 2.28, 20000),
                        rng.normal(0, 0.05, 20000), [0.8, -4.0, 1.0, 45.6]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([oracle.bf16_round(float(v)) for v in x], np.float32)
    assert np.array_equal(got, ref)
    assert oracle.bf16_round(0.8) == 0.80078125
    assert oracle.bf16_round(45.6) == 45.5


def test_residual_decode():
    cfg = dict(W.ALPHA_112K, wform=2)
    we, wi = oracle.weight_tables(cfg)
    for i in (0, 1, 100, 32767, 32768, 65535):
        for inh, w in ((0, we[i]), (1, wi[i])):
            mu = np.float32(-cfg["g"] * cfg["w_exc"]) if inh else np.float32(cfg["w_exc"])
            d = torch.tensor([float(np.float32(float(w) / float(mu) - 1.0))]).to(
                torch.bfloat16).float().item()
            ref = float(np.float32(float(mu) + float(mu) * d))
            assert oracle.decode_weight(cfg, inh, float(w)) == ref
            # error of the residual form: BF16 unit roundoff 2^-8 of delta, times mu
            assert abs(ref - float(w)) <= 2.0**-8 * abs(float(w) - float(mu)) + 4e-6 * abs(float(w))
    # the delta net's weights are exact in the residual form
    cd = dict(W.DELTA_SMALL, wform=2)
    assert oracle.decode_weight(cd, 0, 0.8) == np.float32(0.8)
    assert oracle.decode_weight(cd, 1, -4.0) == -4.0
    assert oracle.decode_weight(dict(W.DELTA_SMALL, wform=1), 0, np.float32(0.8)) == 0.80078125


def test_ref_steps():
    assert oracle.ref_steps(W.DELTA_SMALL) == 20
    assert oracle.ref_steps(W.ALPHA_112K) == 5
