"""Shared test helpers: tie-aware raster comparison and firing statistics.

A raster mismatch between the FP32 GPU path and the FP64 oracle is
*explained* only when the oracle's membrane potential at that step lay within
``eps`` of threshold (a rounding-level tie); after the first explained
mismatch the comparison stops, since the network is chaotic.
"""
from __future__ import annotations

import numpy as np

import oracle


def _by_step(st, idx):
    d = {}
    for t, j in zip(st.tolist(), idx.tolist()):
        d.setdefault(t, set()).add(j)
    return d


def compare_rasters(cfg: dict, gpu_st, gpu_idx, horizon: int, eps: float):
    """Return (first_mismatch_step or None, explained, details)."""
    ost, oidx = oracle.Net(cfg).simulate(horizon)
    g = _by_step(np.asarray(gpu_st)[np.asarray(gpu_st) < horizon],
                 np.asarray(gpu_idx)[np.asarray(gpu_st) < horizon])
    o = _by_step(ost, oidx)
    steps = sorted(set(g) | set(o))
    for t in steps:
        a, b = g.get(t, set()), o.get(t, set())
        if a != b:
            diff = sorted(a ^ b)
            ref = oracle.Net(cfg)
            ref.simulate(t + 1)
            vpre = ref.vpre()
            margins = [abs(vpre[j] - cfg["v_th"]) for j in diff]
            return t, all(m <= eps for m in margins), dict(diff=diff, margins=margins)
    return None, True, {}


def rate_cv(st, idx, n: int, t_lo: int, t_hi: int, h: float):
    """Population rate (Hz) and mean ISI CV over neurons with >= 3 spikes."""
    st = np.asarray(st)
    idx = np.asarray(idx)
    m = (st >= t_lo) & (st < t_hi)
    st, idx = st[m], idx[m]
    rate = len(st) / (n * (t_hi - t_lo) * h * 1e-3)
    order = np.lexsort((st, idx))
    st, idx = st[order], idx[order]
    cvs = []
    starts = np.flatnonzero(np.r_[True, idx[1:] != idx[:-1]])
    ends = np.r_[starts[1:], len(idx)]
    for a, b in zip(starts, ends):
        if b - a >= 3:
            isi = np.diff(st[a:b]).astype(np.float64)
            cvs.append(isi.std() / isi.mean())
    return rate, float(np.mean(cvs)) if cvs else float("nan")
