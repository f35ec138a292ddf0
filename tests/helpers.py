"""Shared test helpers: tie-aware raster comparison and firing statistics.

A raster mismatch between the FP32 GPU path and the FP64 oracle is
*explained* only when the oracle's membrane potential at that step lay within
a tolerance of threshold (a rounding-level tie), the tolerance derived from
the measured FP32 drift; after the first explained mismatch the comparison
stops, since the network is chaotic.
"""
from __future__ import annotations

import numpy as np

import oracle


def _by_step(st, idx):
    d = {}
    for t, j in zip(st.tolist(), idx.tolist()):
        d.setdefault(t, set()).add(j)
    return d


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


def _ulp32(x: float) -> float:
    return float(np.spacing(np.float32(abs(x))))


def spike_exact(cfg: dict, gpu, ref_factory, horizon: int, min_exact: int, safety: float = 2.0,
                tgt=None, raster: list | None = None):
    """Tie-aware raster comparison with a tolerance derived from measurement.

    ``gpu`` is a built context (record_spikes on, at step 0) and
    ``ref_factory()`` returns a fresh oracle at step 0 (``oracle.Net`` or
    ``oracle.Partitioned``).  Both advance ``min_exact`` = m steps.  If their
    rasters agree there, the largest |V_gpu - V_oracle| after those m steps
    is the FP32 rounding drift of the update replayed from the same state;
    drift from per-step errors d grows as d (1 - P33^m) / (1 - P33) toward
    d / (1 - P33), so eps = safety * drift / (1 - P33^m) (at least ``safety``
    FP32 ulps of V_th) bounds it for the rest of the run.  A mismatch inside
    the first m steps is held to the a-priori bound of m steps of FP32
    rounding, safety * 2 m ulp(V_th) (two roundings per step).  Both then
    advance to ``horizon``; a mismatch is explained only if the oracle's V
    before the threshold test lay within the tolerance of V_th for every
    neuron involved, and the comparison stops at the first one (chaos).
    ``tgt`` = (lo, hi): the oracle holds only those targets (open loop) and
    only they are compared.  ``raster``: a list that receives the GPU's
    compared (steps, ids), which this call drains from the context.  Returns
    (eps, first mismatch step or None, spikes compared, the oracle advanced
    to ``horizon``)."""
    lo, hi = tgt if tgt is not None else (0, int(cfg["n_exc"] + cfg["n_inh"]))

    def spikes():
        st, idx = gpu.spikes()
        m = (idx >= lo) & (idx < hi)
        return st[m], idx[m]

    ref = ref_factory()
    gpu.simulate_steps(min_exact)
    ost1, oid1 = ref.simulate(min_exact)
    g_st, g_id = spikes()
    eps_a = safety * 2 * min_exact * _ulp32(cfg["v_th"])
    if np.array_equal(g_st, ost1) and np.array_equal(g_id, oid1):
        dv = float(np.abs(gpu.state()["V"][lo:hi].astype(np.float64) - ref.state()["V"]).max())
        p33 = np.exp(-cfg["h"] / cfg["tau_m"])
        eps = safety * max(dv / (1.0 - p33 ** min_exact), _ulp32(cfg["v_th"]))
    else:
        eps = eps_a
    gpu.simulate_steps(horizon - min_exact)
    ost2, oid2 = ref.simulate(horizon - min_exact)
    g2_st, g2_id = spikes()
    if raster is not None:
        raster.append((np.concatenate([g_st, g2_st]), np.concatenate([g_id, g2_id])))
    g = _by_step(np.concatenate([g_st, g2_st]), np.concatenate([g_id, g2_id]))
    o = _by_step(np.concatenate([ost1, ost2]), np.concatenate([oid1, oid2]))
    n_cmp = 0
    for t in sorted(set(g) | set(o)):
        a, b = g.get(t, set()), o.get(t, set())
        if a != b:
            tol = eps_a if t < min_exact else eps
            diff = sorted(a ^ b)
            chk = ref_factory()
            chk.simulate(t + 1)
            vpre = chk.vpre()
            margins = [abs(vpre[j - lo] - cfg["v_th"]) for j in diff]
            assert all(m <= tol for m in margins), \
                f"unexplained mismatch at step {t}: {diff} margins {margins} tolerance {tol}"
            return tol, t, n_cmp, ref
        n_cmp += len(a)
    return eps, None, n_cmp, ref


# --------------------------------------------------------------------------
# realization ensembles of chaotic runs
# --------------------------------------------------------------------------
def kicked(V, r: int, seed: int = 1):
    """Initial V of realization ``r`` of a chaotic run: realization 0 is the
    seeded initial state; realization r > 0 raises 20 neurons' V by 5 mV,
    which moves some of their first spikes and, through the recurrent
    chaos, the whole raster within a few hundred ms (a kick of a single
    neuron can die out before it moves a spike)."""
    V = np.array(V, copy=True)
    if r:
        idx = np.random.default_rng([seed, r]).choice(len(V), 20, replace=False)
        V[idx] += 5.0
    return V


def realization_z(a, b) -> float:
    """|mean(a) - mean(b)| in standard errors, with the pooled sample sd of
    the two realization samples (b may hold a single value)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    ss = ((a - a.mean()) ** 2).sum() + ((b - b.mean()) ** 2).sum()
    s = np.sqrt(ss / (len(a) + len(b) - 2))
    return float(abs(a.mean() - b.mean()) / (s * np.sqrt(1.0 / len(a) + 1.0 / len(b))))
