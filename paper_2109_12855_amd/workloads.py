"""Workload parameters and seeded input generators.

This module holds parameters and seeded synthetic inputs only -- none of the
method's arithmetic.  Both the GPU path and the CPU oracle take their inputs
from here, so a test can feed both sides the same network description and
the same replay spike lists.

The benchmark network is the balanced random network of Sec. 2.2 of the
paper (Brunel-type, static synapses).  Its parameter tables are not in the
paper; the values below are the workload definitions this project uses
(delta-current net with J = 0.8 mV, g = 5, eta = 2; alpha-current net of
112,500 neurons at in-degree 11,250 with 45.6 pA weights; its one-GPU
brain-scale share; a batched parameter sweep).
"""
from __future__ import annotations

import math

import numpy as np

_BASE = dict(
    model=0, wform=0, n_src_exc=0, n_src_inh=0, ring_len=32, h=0.1, i_e=0.0,
    e_l=0.0, src_rate_hz=0.0, tgt_lo=0, tgt_hi=0, seed=1,
)

# Poisson drive of the delta net: eta times the rate nu_th = V_th/(J K_E tau_m)
# that drives the mean membrane potential to threshold, per external synapse,
# times K_E external synapses (Brunel 2000).
def _delta_drive(eta: float, v_th: float, j: float, k_e: int, tau_m: float) -> float:
    nu_th_per_ms = v_th / (j * k_e * tau_m)
    return eta * nu_th_per_ms * 1000.0 * k_e


DELTA_SMALL = dict(
    _BASE,
    name="delta_1250",
    model=0,
    n_exc=1000, n_inh=250, k_exc=100, k_inh=25,
    d_lo=15, d_hi=15, d_min=15, d_max=15,
    w_exc=0.8, w_cv=0.0, g=5.0,
    tau_m=20.0, c_m=250.0, tau_syn=1.0, v_th=20.0, v_reset=10.0, t_ref=2.0,
    v0_lo=0.0, v0_hi=20.0,
    drive_rate_hz=_delta_drive(2.0, 20.0, 0.8, 100, 20.0),  # 2500 Hz, lambda 0.25
    drive_w=0.8,
    t_sim_ms=1000.0,
)

# Alpha-current net.  Neuron parameters are the usual ones of this benchmark
# class (C_m 250 pF, tau_m 10 ms, tau_syn 0.32582722 ms, V_th 20 mV,
# V_reset 0, t_ref 0.5 ms); a 45.6 pA weight then gives a 0.14 mV PSP peak.
# The drive is the rate eta * nu_th * K_E with eta = 1.685 and
# nu_th = V_th C_m / (J K_E e tau_m tau_syn), tuned for ~8 Hz.
_ALPHA_NEURON = dict(
    model=1, tau_m=10.0, c_m=250.0, tau_syn=0.32582722, v_th=20.0, v_reset=0.0,
    t_ref=0.5, v0_lo=0.0, v0_hi=20.0, w_exc=45.6, w_cv=0.05, g=5.0, drive_w=45.6,
    d_lo=10, d_hi=20, d_min=10, d_max=20,
)


def _alpha_drive(eta: float, k_e: int) -> float:
    p = _ALPHA_NEURON
    nu_th_per_ms = p["v_th"] * p["c_m"] / (p["w_exc"] * k_e * math.e * p["tau_m"] * p["tau_syn"])
    return eta * nu_th_per_ms * 1000.0 * k_e


ALPHA_ETA = 1.685

ALPHA_112K = dict(
    _BASE, **_ALPHA_NEURON,
    name="alpha_112500_fp32",
    n_exc=90000, n_inh=22500, k_exc=9000, k_inh=2250,
    drive_rate_hz=_alpha_drive(ALPHA_ETA, 9000),
    t_sim_ms=1000.0,
)

ALPHA_112K_BF16 = dict(ALPHA_112K, name="alpha_112500_bf16", wform=2)
ALPHA_112K_PACKED = dict(ALPHA_112K, name="alpha_112500_bf16_packed", wform=3)

# the oracle decodes the packed form's weights exactly like the residual form
ORACLE_WFORM = {0: 0, 1: 1, 2: 2, 3: 2}

# One GPU's share of a brain-scale net: 1,125,000 local targets whose
# 11,250 sources each come from a virtual 10M population (8M E, 2M I) that
# fires open loop at 8 Hz.
ALPHA_BRAIN_SHARE = dict(
    _BASE, **_ALPHA_NEURON,
    name="alpha_share_1125000_bf16",
    wform=2,
    n_exc=900000, n_inh=225000, k_exc=9000, k_inh=2250,
    n_src_exc=8_000_000, n_src_inh=2_000_000, src_rate_hz=8.0,
    drive_rate_hz=_alpha_drive(ALPHA_ETA, 9000),
    t_sim_ms=500.0,
)

# Short minimum delay: the 112,500-neuron net with delays uniform over 1..20
# steps (0.1-2 ms), so a slice is a single 0.1 ms step -- ten times as many
# slices per simulated second, each delivering a tenth of the spikes, which
# stresses the per-slice cost (packed 4-byte records).
ALPHA_112K_SHORT_DELAY = dict(ALPHA_112K, name="alpha_112500_dmin1_packed", wform=3,
                              d_lo=1, d_hi=20, d_min=1, d_max=20)

WORKLOADS = {w["name"]: w for w in (DELTA_SMALL, ALPHA_112K, ALPHA_112K_BF16, ALPHA_BRAIN_SHARE,
                                    ALPHA_112K_SHORT_DELAY)}


def plastic(cfg: dict, a_plus: float = 0.01, a_minus: float = 0.0105, w_max: float = 2.0,
            tau_plus: float = 20.0, tau_minus: float = 20.0) -> dict:
    """The network with plastic excitatory synapses: amplitudes and the upper
    weight bound as multiples of the mean excitatory weight, time constants
    in ms (pair windows of the classic spike-timing experiments)."""
    w = cfg["w_exc"]
    out = dict(cfg, plastic=1, stdp_tau_plus=tau_plus, stdp_tau_minus=tau_minus,
               stdp_a_plus=a_plus * w, stdp_a_minus=a_minus * w, stdp_w_max=w_max * w)
    out["name"] = cfg.get("name", "net") + "_plastic"
    return out


def tiny(model: int = 0, n: int = 40, k: int = 8, seed: int = 7, d_lo: int | None = None,
         d_hi: int | None = None, wform: int = 0, w_cv: float | None = None, **over) -> dict:
    """A small balanced net of the same structure (80% E) for brute-force checks."""
    n_e = int(round(0.8 * n))
    k_e = int(round(0.8 * k))
    if model == 0:
        base = dict(DELTA_SMALL)
        base.update(d_lo=d_lo or 3, d_hi=d_hi or 7, d_min=d_lo or 3, d_max=d_hi or 7,
                    drive_rate_hz=_delta_drive(2.0, 20.0, 0.8, max(k_e, 1), 20.0) * 1.5,
                    w_exc=0.8 * math.sqrt(100.0 / max(k_e, 1)) * 2.0,
                    drive_w=0.8 * math.sqrt(100.0 / max(k_e, 1)) * 2.0,
                    w_cv=0.0 if w_cv is None else w_cv)
    else:
        base = dict(ALPHA_112K)
        base.update(d_lo=d_lo or 3, d_hi=d_hi or 7, d_min=d_lo or 3, d_max=d_hi or 7,
                    w_exc=45.6 * 20.0, drive_w=45.6 * 10.0,
                    drive_rate_hz=8000.0, w_cv=0.05 if w_cv is None else w_cv)
    base.update(name=f"tiny_{'alpha' if model else 'delta'}_{n}", model=model, n_exc=n_e,
                n_inh=n - n_e, k_exc=k_e, k_inh=k - k_e, seed=seed, wform=wform, ring_len=32)
    base.update(over)
    return base


def replay_spikes(n_src: int, n_spikes: int, d_min: int, seed: int):
    """Seeded replay spike list: distinct (lag, src) pairs in (lag, src) order."""
    rng = np.random.default_rng(seed)
    n_spikes = min(n_spikes, n_src * d_min)
    flat = rng.choice(n_src * d_min, size=n_spikes, replace=False)
    flat.sort()
    lag = (flat // n_src).astype(np.uint8)
    src = (flat % n_src).astype(np.uint32)
    return src, lag


def sweep_nets(n_nets: int = 64, seed: int = 2022, wform: int = 0):
    """Batched parameter sweep: delta nets with N ~ U{2000..40000},
    K ~ U{500..5000}, g in {4,5,6}, eta in {1.5,2,3}, each with its own seed.
    J_E scales as 0.8 mV * sqrt(100 / K_E) to keep the delta net's regime."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_nets):
        n = int(rng.integers(2000, 40001))
        k = int(rng.integers(500, 5001))
        g = float(rng.choice([4.0, 5.0, 6.0]))
        eta = float(rng.choice([1.5, 2.0, 3.0]))
        n_e = int(round(0.8 * n))
        k_e = int(round(0.8 * k))
        j = 0.8 * math.sqrt(100.0 / k_e)
        d = dict(DELTA_SMALL)
        d.update(name=f"sweep_{i}", n_exc=n_e, n_inh=n - n_e, k_exc=k_e, k_inh=k - k_e, g=g,
                 w_exc=j, drive_w=j, drive_rate_hz=_delta_drive(eta, 20.0, j, k_e, 20.0),
                 seed=int(rng.integers(1, 2**62)), wform=wform)
        out.append(d)
    return out
