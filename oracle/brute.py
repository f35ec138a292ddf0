"""Brute-force dense reference for tiny networks (test infrastructure only).

A second, independent formulation used to pin the C oracle: numpy's own
Philox bit generator supplies the random words, scipy's ``expm`` supplies the
propagators and ``ndtri`` the weight quantiles, connectivity is held as dense
per-delay matrices, and the input of neuron j at step t is the plain sum

    x_j(t) = sum_d sum_s W_d[j, s] * spike_s(t - d)

with no ring buffers, no target segments and no slices (Sec. 1 / Sec. 2.1:
a spike emitted at step t takes effect after its delay).  Any mistake in the
oracle's ring indexing, slicing, transposition or delivery order shows up as
a disagreement with this.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
import scipy.special
import scipy.stats

_M64 = (1 << 64) - 1
STREAM_SYN, STREAM_INIT, STREAM_DRIVE = 1, 2, 3


def philox_words(seed: int, stream: int, c0: int, c1: int) -> list[int]:
    """Philox4x64-10 at counter (c0, c1, 0, 0), key (seed, stream), from numpy.

    numpy's generator advances its counter by one before each block, so the
    block for counter c is the first block of a generator started at c - 1."""
    c = (c0 + (c1 << 64) - 1) % (1 << 256)
    ctr = np.array([(c >> (64 * i)) & _M64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([seed, stream], dtype=np.uint64), counter=ctr)
    return [int(x) for x in bg.random_raw(4)]


def propagators(cfg: dict) -> dict:
    """Matrix exponential of the linear system over one step h, with the
    constant current I_e carried as a fourth, constant state."""
    h, tm, ts, C = cfg["h"], cfg["tau_m"], cfg["tau_syn"], cfg["c_m"]
    A = np.array([[-1.0 / ts, 0.0, 0.0, 0.0],
                  [1.0, -1.0 / ts, 0.0, 0.0],
                  [0.0, 1.0 / C, -1.0 / tm, 1.0 / C],
                  [0.0, 0.0, 0.0, 0.0]])
    P = scipy.linalg.expm(A * h)
    return dict(P11=P[0, 0], P21=P[1, 0], P22=P[1, 1], P31=P[2, 0], P32=P[2, 1], P33=P[2, 2],
                P30=P[2, 3])


def poisson_thresholds(lam: float) -> list[int]:
    out = []
    k = 0
    while True:
        t = math.floor(scipy.stats.poisson.cdf(k, lam) * 2.0**32)
        if t >= 2**32 - 1:
            break
        out.append(t)
        k += 1
        if k > 200:
            break
    return out


def weight_value(cfg: dict, inh: bool, widx: int) -> float:
    if cfg["w_cv"] == 0.0:
        w = np.float32(-cfg["g"] * cfg["w_exc"]) if inh else np.float32(cfg["w_exc"])
    else:
        z = scipy.special.ndtri((widx + 0.5) / 65536.0)
        we = cfg["w_exc"] * (1.0 + cfg["w_cv"] * z)
        w = np.float32(-cfg["g"] * we) if inh else np.float32(we)
    return float(w)


def connections(cfg: dict):
    """Target-major draws: one Philox block per (target j, slot k)."""
    n = cfg["n_exc"] + cfg["n_inh"]
    k_tot = cfg["k_exc"] + cfg["k_inh"]
    src = np.zeros((n, k_tot), np.int64)
    dly = np.zeros((n, k_tot), np.int64)
    widx = np.zeros((n, k_tot), np.int64)
    w = np.zeros((n, k_tot), np.float64)
    nd = cfg["d_hi"] - cfg["d_lo"] + 1
    for j in range(n):
        for k in range(k_tot):
            r = philox_words(cfg["seed"], STREAM_SYN, j, k)
            inh = k >= cfg["k_exc"]
            if inh:
                s = cfg["n_exc"] + ((r[0] * cfg["n_inh"]) >> 64)
            else:
                s = (r[0] * cfg["n_exc"]) >> 64
            src[j, k] = s
            dly[j, k] = cfg["d_lo"] + ((r[1] * nd) >> 64)
            widx[j, k] = r[2] >> 48
            w[j, k] = weight_value(cfg, inh, int(widx[j, k]))
    return src, dly, widx, w


def dense_matrices(cfg: dict, src, dly, w):
    n = cfg["n_exc"] + cfg["n_inh"]
    W = np.zeros((cfg["d_max"] + 1, n, n))
    Cn = np.zeros((cfg["d_max"] + 1, n, n), np.int64)
    for j in range(n):
        for k in range(src.shape[1]):
            W[dly[j, k], j, src[j, k]] += w[j, k]
            Cn[dly[j, k], j, src[j, k]] += 1
    return W, Cn


def initial_v(cfg: dict, n: int) -> np.ndarray:
    v = np.zeros(n)
    for j in range(n):
        r = philox_words(cfg["seed"], STREAM_INIT, j, 0)
        u = (r[0] >> 11) * 2.0**-53
        v[j] = float(np.float32(cfg["v0_lo"] + (cfg["v0_hi"] - cfg["v0_lo"]) * u))
    return v


def simulate(cfg: dict, n_steps: int):
    """Dense time-stepped simulation; returns spikes, per-step inputs and
    the final state."""
    n = cfg["n_exc"] + cfg["n_inh"]
    src, dly, widx, w = connections(cfg)
    W, Cn = dense_matrices(cfg, src, dly, w)
    P = propagators(cfg)
    thr = poisson_thresholds(cfg["drive_rate_hz"] * cfg["h"] * 1e-3)
    ref = int(round(cfg["t_ref"] / cfg["h"]))
    V = initial_v(cfg, n)
    y1 = np.zeros(n)
    y2 = np.zeros(n)
    r = np.zeros(n, np.int64)
    S = np.zeros((n_steps, n))
    inputs = np.zeros((n_steps, n))
    drive_cache = {}
    spikes = []
    e_over_ts = math.e / cfg["tau_syn"]
    for t in range(n_steps):
        x = np.zeros(n)
        for d in range(cfg["d_min"], cfg["d_max"] + 1):
            if t - d >= 0:
                x += W[d] @ S[t - d]
        inputs[t] = x
        for j in range(n):
            key = (j, t >> 3)
            if key not in drive_cache:
                drive_cache[key] = philox_words(cfg["seed"], STREAM_DRIVE, j, t >> 3)
            words = drive_cache[key]
            wd = words[(t & 7) >> 1]
            u = (wd >> 32) if (t & 1) else (wd & 0xFFFFFFFF)
            c = sum(1 for T in thr if u >= T)
            drive = c * cfg["drive_w"]
            if cfg["model"] == 0:
                if r[j] > 0:
                    r[j] -= 1
                else:
                    V[j] = cfg["e_l"] + P["P33"] * (V[j] - cfg["e_l"]) + P["P30"] * cfg["i_e"] + x[j] + drive
            else:
                a1, a2 = y1[j], y2[j]
                if r[j] == 0:
                    V[j] = (cfg["e_l"] + P["P31"] * a1 + P["P32"] * a2 + P["P33"] * (V[j] - cfg["e_l"])
                            + P["P30"] * cfg["i_e"])
                else:
                    r[j] -= 1
                y2[j] = P["P21"] * a1 + P["P22"] * a2
                y1[j] = P["P11"] * a1 + e_over_ts * (x[j] + drive)
            if V[j] >= cfg["v_th"]:
                V[j] = cfg["v_reset"]
                r[j] = ref
                S[t, j] = 1.0
                spikes.append((t, j))
    return dict(spikes=spikes, S=S, W=W, Cn=Cn, inputs=inputs, V=V, y1=y1, y2=y2, r=r,
                src=src, dly=dly, widx=widx, w=w)


def pending_ring(res: dict, cfg: dict, t_now: int, t_delivered: int, n_slots: int):
    """Ring contents for steps [t_now, t_now + n_slots) holding contributions
    of every spike emitted before step t_delivered."""
    W, Cn, S = res["W"], res["Cn"], res["S"]
    n = W.shape[1]
    rb = np.zeros((n_slots, n))
    cnt = np.zeros((n_slots, n), np.int64)
    for i in range(n_slots):
        s = t_now + i
        for d in range(cfg["d_min"], cfg["d_max"] + 1):
            t_sp = s - d
            if 0 <= t_sp < t_delivered:
                rb[i] += W[d] @ S[t_sp]
                cnt[i] += Cn[d] @ S[t_sp].astype(np.int64)
    return rb, cnt


STREAM_SRC = 4


def open_loop_spikes(cfg: dict, t0: int, n_steps: int):
    """Open-loop virtual sources, drawn independently of the C oracle.

    Source s fires at step t when the 32-bit uniform of step t (the low half
    of word (t mod 8) // 2 of the Philox block at counter (s, t // 8) for even
    t, the high half for odd t) lies below floor(2^32 p), with
    p = 1 - exp(-rate h) the Bernoulli probability of one step.  Returns
    (src, lag) in (lag, src) order, lag = t - t0.  numpy supplies every
    Philox block; each block is drawn once and its eight halves reused."""
    n_src = cfg["n_src_exc"] + cfg["n_src_inh"]
    p = -math.expm1(-cfg["src_rate_hz"] * cfg["h"] * 1e-3)
    thr = math.floor(p * 2.0**32)
    c_lo, c_hi = t0 >> 3, (t0 + n_steps - 1) >> 3
    # halves[s, c - c_lo, q]: uniform of step 8 c + q
    halves = np.zeros((n_src, c_hi - c_lo + 1, 8), np.uint64)
    for s in range(n_src):
        for c in range(c_lo, c_hi + 1):
            words = philox_words(cfg["seed"], STREAM_SRC, s, c)
            for q in range(8):
                w = words[q >> 1]
                halves[s, c - c_lo, q] = (w >> 32) if (q & 1) else (w & 0xFFFFFFFF)
    src, lag = [], []
    for l in range(n_steps):
        t = t0 + l
        u = halves[:, (t >> 3) - c_lo, t & 7]
        for s in np.flatnonzero(u < thr):
            src.append(int(s))
            lag.append(l)
    return np.array(src, np.uint32), np.array(lag, np.uint8)


def simulate_plastic(cfg: dict, n_steps: int):
    """Dense time-stepped simulation with plastic excitatory synapses.

    A second formulation of the plasticity reading: synapses are held target-
    major (as drawn) with per-synapse weights; when a source fires at step t
    each of its excitatory synapses (j, d) is updated at once from the raster
    so far -- the latest spike of j at or before t - d, and the source's
    previous spike -- and the updated weight is scheduled to arrive at j at
    step t + d.  No ring buffers, no slices, no source-major table."""
    n = cfg["n_exc"] + cfg["n_inh"]
    src, dly, widx, w = connections(cfg)
    w = w.copy()
    P = propagators(cfg)
    thr = poisson_thresholds(cfg["drive_rate_hz"] * cfg["h"] * 1e-3)
    ref = int(round(cfg["t_ref"] / cfg["h"]))
    V = initial_v(cfg, n)
    y1 = np.zeros(n)
    y2 = np.zeros(n)
    r = np.zeros(n, np.int64)
    S = np.zeros((n_steps, n), bool)
    arrive = np.zeros((n_steps + cfg["d_max"] + 1, n))
    last_pre = np.full(n, -1, np.int64)
    by_src = {}
    for j in range(n):
        for k in range(src.shape[1]):
            by_src.setdefault(int(src[j, k]), []).append((j, k))
    h = cfg["h"]
    spikes = []
    e_over_ts = math.e / cfg["tau_syn"]
    drive_cache = {}
    for t in range(n_steps):
        x = arrive[t]
        fired = []
        for j in range(n):
            key = (j, t >> 3)
            if key not in drive_cache:
                drive_cache[key] = philox_words(cfg["seed"], STREAM_DRIVE, j, t >> 3)
            wd = drive_cache[key][(t & 7) >> 1]
            u = (wd >> 32) if (t & 1) else (wd & 0xFFFFFFFF)
            drive = sum(1 for T in thr if u >= T) * cfg["drive_w"]
            if cfg["model"] == 0:
                if r[j] > 0:
                    r[j] -= 1
                else:
                    V[j] = cfg["e_l"] + P["P33"] * (V[j] - cfg["e_l"]) + P["P30"] * cfg["i_e"] + x[j] + drive
            else:
                a1, a2 = y1[j], y2[j]
                if r[j] == 0:
                    V[j] = (cfg["e_l"] + P["P31"] * a1 + P["P32"] * a2 + P["P33"] * (V[j] - cfg["e_l"])
                            + P["P30"] * cfg["i_e"])
                else:
                    r[j] -= 1
                y2[j] = P["P21"] * a1 + P["P22"] * a2
                y1[j] = P["P11"] * a1 + e_over_ts * (x[j] + drive)
            if V[j] >= cfg["v_th"]:
                V[j] = cfg["v_reset"]
                r[j] = ref
                S[t, j] = True
                spikes.append((t, j))
                fired.append(j)
        for s in fired:
            for (j, k) in by_src.get(s, []):
                d = int(dly[j, k])
                if s < cfg["n_exc"]:
                    seen = np.flatnonzero(S[: t - d + 1, j]) if t - d >= 0 else []
                    if len(seen):
                        tl = int(seen[-1])
                        if last_pre[s] >= 0 and tl + d > last_pre[s]:
                            w[j, k] = min(cfg["stdp_w_max"], w[j, k] + cfg["stdp_a_plus"] *
                                          math.exp(-(tl + d - last_pre[s]) * h / cfg["stdp_tau_plus"]))
                        w[j, k] = max(0.0, w[j, k] - cfg["stdp_a_minus"] *
                                      math.exp(-(t - tl - d) * h / cfg["stdp_tau_minus"]))
                arrive[t + d, j] += w[j, k]
            last_pre[s] = t
    return dict(spikes=spikes, w=w, src=src, dly=dly, V=V, y1=y1, y2=y2, r=r)
