"""Benchmark: synaptic events delivered per second on one MI355X.

A step is one slice of the simulation cycle (Sec. 1 / Sec. 2.1 of the
paper): the slice's spikes are routed through the connection table into the
ring buffers (Alg. REF result, Sec. 3.2), and every neuron is updated
through the next d_min steps with spike compaction.

Headline workload: one GPU's share of a brain-scale network -- 1,125,000
alpha-current neurons at in-degree 11,250 drawn from a virtual population of
10,000,000 sources firing at 8 Hz (1.27e10 synapses), BF16-residual weights,
open loop, 1 ms slices.  A slice is two launches on the context's stream
(the binning pass and the fused accumulate/update kernel); ``value`` is
synaptic events per second over the timed slices, the roofline fraction is
algorithmic bytes per slice (5 B per synapse for the BF16 forms) over the
measured time per slice, against 8 TB/s.

Also reported: the same share in the FP32 form, the 112,500-neuron closed-
loop net in its four storage forms (timed after an untimed 200 ms settle),
ring / rate / CV errors against the FP64 oracle, one-step slices, the
batched 64-network sweep (FP32 and BF16), the FP64 oracle on the host's
cores, and the paper's CPU delivery algorithms.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_PROBE_BYTES = 256 << 20
PROFILES = os.path.join(ROOT, "profiles")
SHARE_TRAFFIC = os.path.join(PROFILES, "k_bin_k_slice1_alpha_share_1125000_bf16_resid.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2109_12855_amd", "csrc", f)
                  for f in ("sd_kernels.hip", "sd_internal.h")]
SETTLE_SLICES = 200          # untimed biological settle of the closed-loop net (200 ms)
B_SYN = {0: 9, 1: 5, 2: 5, 3: 4}   # algorithmic bytes per synapse of each storage form


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_json(path: str):
    """The ``traffic_json`` line of a committed rocprofv3 summary (HBM bytes
    per launch from FETCH_SIZE / WRITE_SIZE scaled by a copy of known size,
    and the L2 hit rate), or None when it is missing or was taken on other
    kernel sources."""
    try:
        with open(path) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"^traffic_json: (\{.*\})$", text, re.M)
    if not m:
        return None
    t = json.loads(m.group(1))
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t


def copy_probe():
    """A plain elementwise copy (read and write COPY_PROBE_BYTES each): its
    FETCH_SIZE / WRITE_SIZE counters calibrate the slice kernels'."""
    import torch

    n = COPY_PROBE_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    _log(f"copy probe: 3 x {COPY_PROBE_BYTES} B read + written")


def copy_bandwidth(nbytes: int = 1 << 31, reps: int = 10) -> dict:
    """Achieved HBM bandwidth of a plain device copy (read + write of nbytes
    each), timed with HIP events: the practical ceiling the slice's
    algorithmic GB/s is also compared with."""
    import torch

    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_each_way": nbytes, "us": round(ms * 1e3, 1),
            "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def _log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(events: float, spikes: float, n: int, d_min: int, b_syn: int,
                      s_state: int, b_spike: int = 5) -> float:
    """Bytes one slice must move: synapses of every delivered event, one ring
    write and one read per neuron-step, neuron state read + write, and the
    spike list (5 B per entry)."""
    return events * b_syn + n * d_min * 8 + n * 2 * s_state + spikes * b_spike


# Plastic synapses (FP32 form): each event reads its 9-byte record and writes
# its 4-byte weight back; each neuron's state adds a 12-byte spike history;
# each spike-list entry adds a lag mask and the source's previous spike.
PLASTIC_B_EVENT, PLASTIC_S_STATE, PLASTIC_B_SPIKE = 13, 16 + 12, 13


def _free(obj):
    import torch

    obj.close()
    del obj
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def time_net(cfg: dict, steps: int, warmup: int, settle: int = 0, open_loop: bool = False):
    """Build, run settle + warmup untimed slices, then time ``steps`` slices
    with HIP events on the context's stream (torch's current stream: nothing
    else is launched there in the timed region, so the time per slice is the
    mean over its launches)."""
    import torch

    from paper_2109_12855_amd import sdeliver

    t0 = time.time()
    net = sdeliver.Net(cfg).build()
    torch.cuda.synchronize()
    t_build = time.time() - t0
    d_min = cfg["d_min"]
    _log(f"{cfg['name']}: built {net.n_syn:.3e} synapses in {t_build:.1f} s")
    if open_loop:
        net.prepare_input((settle + warmup + steps + 2) * d_min)
    net.simulate_steps((settle + warmup) * d_min)
    torch.cuda.synchronize()
    s0 = net.stats()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    net.simulate_steps(steps * d_min)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    s1 = net.stats()
    ev = s1["events_delivered"] - s0["events_delivered"]
    spk = s1["spikes_delivered"] - s0["spikes_delivered"]
    emitted = s1["spikes_emitted"] - s0["spikes_emitted"]
    slices = s1["slices"] - s0["slices"]
    n = net.n_local
    b_syn = B_SYN[cfg["wform"]]
    s_state = 16 if cfg["model"] == 1 else 8
    b_spk = 5
    if cfg.get("plastic"):
        b_syn, s_state, b_spk = PLASTIC_B_EVENT, PLASTIC_S_STATE, PLASTIC_B_SPIKE
    b_alg = algorithmic_bytes(ev / slices, spk / slices, n, d_min, b_syn, s_state, b_spk)
    us = ms * 1e3 / slices
    out = dict(name=cfg["name"], synapses=net.n_syn, build_s=round(t_build, 2),
               layout="source_major" if net.sizes["layout"] == 2 else "block_major",
               block_neurons=net.sizes["block_neurons"], bin_cap=net.sizes["bin_cap"],
               stored_bytes_per_synapse=net.sizes["bytes_per_synapse"],
               alg_bytes_per_synapse=b_syn, slices=slices, ms_total=ms, us_per_slice=us,
               events_per_slice=ev / slices, spikes_in_per_slice=spk / slices,
               events_per_s=ev / (ms * 1e-3),
               rate_hz=emitted / (n * steps * d_min * cfg["h"] * 1e-3),
               alg_bytes_per_slice=b_alg, alg_gbs=b_alg / (us * 1e-6) / 1e9)
    out["roofline_frac"] = out["alg_gbs"] / HBM_PEAK_GBS
    _free(net)
    return out


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def share_cfg(wform: int) -> dict:
    from paper_2109_12855_amd import workloads

    name = {0: "alpha_share_1125000_fp32", 2: "alpha_share_1125000_bf16_resid"}[wform]
    return dict(workloads.ALPHA_BRAIN_SHARE, wform=wform, name=name)


def share_tuning(targets=(1256, 1353), cap_scales=(1.0, 1.5)) -> dict:
    """The binning parameters of the brain-scale share picked by the
    autotuner (sd_autotune_bins: block sizes for the given block counts x
    region capacities relative to the automatic one, each built and timed
    over 20 slices).  The headline itself runs the default parameters, the
    configuration the committed profile covers."""
    from paper_2109_12855_amd import sdeliver

    cfg = share_cfg(2)
    t0 = time.time()
    bn, cap, us = sdeliver.autotune_bins(cfg, targets=targets, cap_scales=cap_scales, warmup=5,
                                         slices=20)
    z = sdeliver.query_sizes(cfg)
    return {"targets": list(targets), "cap_scales": list(cap_scales),
            "default": {"block_neurons": z["block_neurons"], "bin_cap": z["bin_cap"]},
            "chosen": {"block_neurons": bn, "bin_cap": cap}, "us_per_slice": us,
            "tune_s": round(time.time() - t0, 1)}


def alpha_forms():
    from paper_2109_12855_amd import workloads

    base = workloads.ALPHA_112K
    return {"fp32": dict(base, wform=0, name="alpha_112500_fp32"),
            "bf16": dict(base, wform=1, name="alpha_112500_bf16"),
            "bf16_resid": dict(base, wform=2, name="alpha_112500_bf16_resid"),
            "bf16_packed": dict(base, wform=3, name="alpha_112500_bf16_packed")}


def short_delay(slices: int = 5000, warmup: int = 1000) -> dict:
    """The 112,500-neuron net with delays of 1..20 steps (packed records):
    one-step slices, ten times as many per simulated second, each with a
    tenth of the spikes -- the per-slice cost dominates."""
    from paper_2109_12855_amd import workloads

    r = time_net(dict(workloads.ALPHA_112K_SHORT_DELAY), slices, warmup)
    r["slice_ms"] = 0.1
    return r


def sweep(slices: int = 120, warmup: int = 20) -> dict:
    """The batched sweep: 64 independent delta networks (N 2,000-40,000, K
    500-5,000) advanced together, FP32 and plain-BF16 weights.  Block sizes
    come from the autotuner (timed here on the FP32 variant, no cache, batch
    candidates timed through the captured graph) and serve both variants;
    steady-state slices replay the captured graph.  Aggregate events/s and
    algorithmic bytes over all members."""
    import torch

    from paper_2109_12855_amd import sdeliver, workloads

    cfgs32 = workloads.sweep_nets(64)
    t0 = time.time()
    bn, tune_us = sdeliver.autotune(cfgs32, targets=(8, 16, 32, 64, 128, 256), warmup=10,
                                    slices=20)
    t_tune = time.time() - t0
    out = {"workload": "sweep_64_delta_nets", "networks": len(cfgs32), "slice_ms": 1.5,
           "tune_s": round(t_tune, 1), "block_neurons_range": [min(bn), max(bn)]}
    for key, wform in (("fp32", 0), ("bf16", 1)):
        cfgs = workloads.sweep_nets(64, wform=wform)
        bt = sdeliver.Batch([dict(c, block_neurons=b) for c, b in zip(cfgs, bn)]).build()
        bt.set_graph(True)
        d_min = cfgs[0]["d_min"]
        bt.simulate_steps(warmup * d_min)
        torch.cuda.synchronize()
        st0 = [m.stats() for m in bt.members]
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        bt.simulate_steps(slices * d_min)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        st1 = [m.stats() for m in bt.members]
        ev = sum(y["events_delivered"] - x["events_delivered"] for x, y in zip(st0, st1))
        b_alg = 0.0
        for m, x, y, c in zip(bt.members, st0, st1, cfgs):
            b_alg += algorithmic_bytes((y["events_delivered"] - x["events_delivered"]) / slices,
                                       (y["spikes_delivered"] - x["spikes_delivered"]) / slices,
                                       m.n_local, d_min, B_SYN[wform], 8)
        us = ms * 1e3 / slices
        out[key] = {"synapses": int(sum(m.n_syn for m in bt.members)),
                    "blocks": int(sum(m.sizes["n_blocks"] for m in bt.members)),
                    "slices": slices, "us_per_slice": us, "events_per_s": ev / (ms * 1e-3),
                    "alg_bytes_per_slice": b_alg, "alg_gbs": b_alg / (us * 1e-6) / 1e9,
                    "roofline_frac": b_alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                    "graph_replays": bt.graph_launches}
        _free(bt)
    return out


# ---------------------------------------------------------------------------
# errors against the FP64 oracle
# ---------------------------------------------------------------------------
def rate_cv(st, idx, n: int, t_lo: int, t_hi: int, h: float):
    """Population rate (Hz) over steps [t_lo, t_hi) and the mean ISI CV of
    the neurons with at least 3 spikes there."""
    m = (st >= t_lo) & (st < t_hi)
    st, idx = st[m], idx[m]
    rate = len(st) / (n * (t_hi - t_lo) * h * 1e-3)
    order = np.lexsort((st, idx))
    st, idx = st[order], idx[order]
    starts = np.flatnonzero(np.r_[True, idx[1:] != idx[:-1]])
    ends = np.r_[starts[1:], len(idx)]
    cvs = [np.diff(st[a:b]).std() / np.diff(st[a:b]).mean() for a, b in zip(starts, ends)
           if b - a >= 3]
    return rate, float(np.mean(cvs)) if cvs else float("nan")


def _err_block(got, ref):
    d = got.astype(np.float64) - ref
    return {"normwise": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "max_cell_over_max_ref": float(np.abs(d).max() / np.abs(ref).max())}


def ring_errors(forms: dict, share: bool = True, n_spikes: int = 900, seed: int = 2021) -> dict:
    """Ring contents after one delivery against the FP64 oracle holding the
    FP32 table weights (the exact weights of the network), on target
    samples: each storage form of the 112,500-neuron net fed one synthetic
    slice (900 spikes), and the brain-scale share's residual-BF16 form fed
    its first open-loop input slice."""
    import torch

    import oracle
    from paper_2109_12855_amd import sdeliver, workloads

    out = {"vs": "FP64 oracle, FP32 table weights", "alpha_112500": {}}
    base = workloads.ALPHA_112K
    n = base["n_exc"] + base["n_inh"]
    lo, hi = 40_000, 47_168                        # 16 blocks of 448 targets
    src, lag = workloads.replay_spikes(n, n_spikes, base["d_min"], seed=seed)
    ref = oracle.Net(dict(base, wform=0, tgt_lo=lo, tgt_hi=hi))
    ref.deliver(src, lag, 0)
    exact = ref.ring()
    d_src = torch.from_numpy(src.view(np.int32)).cuda()
    d_lag = torch.from_numpy(lag).cuda()
    for name, cfg in forms.items():
        net = sdeliver.Net(cfg).build()
        net.deliver(d_src, d_lag, 0)
        out["alpha_112500"][name] = _err_block(net.ring()[:, lo:hi], exact)
        _free(net)
    out["alpha_112500_sample"] = f"targets [{lo}, {hi}), {len(src)} spikes"
    if share:
        cfg = share_cfg(2)
        net = sdeliver.Net(cfg).build()
        net.prepare_input(20)
        net.simulate_steps(10)
        net.deliver()
        s_lo, s_hi = 517_000, 519_496
        got = net.ring(20)[:, s_lo:s_hi]
        _free(net)
        osrc, olag = oracle.open_loop_spikes(cfg, 0, 10, cap=1 << 20)
        ref = oracle.Net(dict(cfg, wform=0, tgt_lo=s_lo, tgt_hi=s_hi))
        ref.deliver(osrc, olag, 0)
        rows = [(10 + q) % cfg["ring_len"] for q in range(20)]
        out["alpha_share_1125000_bf16_resid"] = _err_block(got, ref.ring()[rows])
        out["alpha_share_sample"] = f"targets [{s_lo}, {s_hi}), {len(osrc)} input spikes"
    return out


def _kick(V, r: int):
    """Realization r of a chaotic run: 20 neurons' initial V raised by 5 mV
    (r = 0: the seeded start)."""
    V = np.array(V, copy=True)
    if r:
        idx = np.random.default_rng([1, r]).choice(len(V), 20, replace=False)
        V[idx] += 5.0
    return V


def rate_cv_errors(forms: dict, t_ms: float = 500.0, threads: int = 16,
                   realizations: int = 8) -> dict:
    """Population rate and mean ISI CV (after the first 100 ms) of each
    storage form's closed-loop run of the 112,500-neuron net, against the
    FP64 oracle with the FP32 table weights, split into target ranges over
    host threads.  The network is chaotic: past the first rounding-level
    tie the GPU and oracle runs are different realizations.  The oracle and
    each form therefore run from the same ``realizations`` starts (the
    seeded one and starts with 20 neurons kicked by 5 mV), and the report
    gives the seeded runs' difference, the ensemble means' difference, the
    realization sds, and the two-sample z of the means (pooled sd)."""
    import oracle
    from paper_2109_12855_amd import sdeliver

    base = forms["fp32"]
    steps = int(round(t_ms / base["h"]))
    n = base["n_exc"] + base["n_inh"]

    def z2(a, b):
        ss = ((a - a.mean()) ** 2).sum() + ((b - b.mean()) ** 2).sum()
        sd = np.sqrt(ss / (len(a) + len(b) - 2))
        return float((a.mean() - b.mean()) / (sd * np.sqrt(1.0 / len(a) + 1.0 / len(b))))

    t0 = time.time()
    o = []
    for r in range(realizations):
        part = oracle.Partitioned(dict(base, wform=0), 16, threads=threads)
        if r:
            part.set_state(V=_kick(part.state()["V"], r))
        ost, oid = part.simulate(steps)
        part.close()
        o.append(rate_cv(ost, oid, n, 1000, steps, base["h"]))
    o = np.array(o)
    om, osd = o.mean(0), o.std(0, ddof=1)
    out = {"vs": "FP64 oracle, FP32 table weights", "t_ms": t_ms, "window_ms": [100, t_ms],
           "realizations": realizations,
           "oracle": {"rate_hz": o[0, 0], "cv": o[0, 1], "mean_rate_hz": om[0], "mean_cv": om[1],
                      "rate_rel_sd": osd[0] / om[0], "cv_rel_sd": osd[1] / om[1],
                      "threads": threads, "wall_s": round(time.time() - t0, 1)}}
    for name, cfg in forms.items():
        g = []
        for r in range(realizations):
            net = sdeliver.Net(dict(cfg, record_spikes=1)).build()
            if r:
                net.set_state(V=_kick(net.state()["V"], r))
            net.simulate_steps(steps)
            st, idx = net.spikes()
            _free(net)
            g.append(rate_cv(st, idx, n, 1000, steps, cfg["h"]))
        g = np.array(g)
        m, sd = g.mean(0), g.std(0, ddof=1)
        out[name] = {"rate_hz": g[0, 0], "cv": g[0, 1],
                     "rate_rel_err": (g[0, 0] - o[0, 0]) / o[0, 0],
                     "cv_rel_err": (g[0, 1] - o[0, 1]) / o[0, 1],
                     "mean_rate_hz": m[0], "mean_cv": m[1],
                     "mean_rate_rel_err": (m[0] - om[0]) / om[0],
                     "mean_cv_rel_err": (m[1] - om[1]) / om[1],
                     "rate_rel_sd": sd[0] / m[0], "cv_rel_sd": sd[1] / m[1],
                     "rate_z": z2(g[:, 0], o[:, 0]), "cv_z": z2(g[:, 1], o[:, 1])}
    return out


# ---------------------------------------------------------------------------
# host baselines
# ---------------------------------------------------------------------------
def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(threads: int, budget_s: float = 10.0, per_thread: int = 4096) -> dict:
    """The FP64 oracle on the host, on the headline workload: oracles holding
    ``per_thread`` targets of the brain-scale share each (all 10M sources),
    fed the same synthetic open-loop-shaped input lists (80,000 (src, lag)
    pairs per 1 ms slice, drawn outside the timed region), delivering and
    updating slice after slice.  One thread alone, then ``threads`` threads
    at once, each with its own target range; synaptic events on the held
    targets per wall-clock second."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_2109_12855_amd import workloads

    cfg = share_cfg(2)
    d_min = cfg["d_min"]
    n_src = cfg["n_src_exc"] + cfg["n_src_inh"]
    spikes = int(round(n_src * cfg["src_rate_hz"] * d_min * cfg["h"] * 1e-3))
    lists = [workloads.replay_spikes(n_src, spikes, d_min, seed=900 + k) for k in range(4)]
    pool = ThreadPoolExecutor(max_workers=threads)
    t0 = time.time()
    nets = list(pool.map(lambda i: oracle.Net(cfg, tgt_lo=i * per_thread,
                                              tgt_hi=(i + 1) * per_thread), range(threads)))
    _log(f"oracle samples built ({threads} x {per_thread} targets) in {time.time() - t0:.1f} s")

    def run(net, deadline):
        ev = 0
        k = 0
        while time.perf_counter() < deadline:
            src, lag = lists[k % len(lists)]
            t_del = net.t_now - d_min if net.t_now >= d_min else 0
            ev += net.deliver(src, lag, t_del)[1]
            net.update(d_min, cap=net.n_local * d_min + 1)
            k += 1
        return ev, k

    out = {"unit": "synaptic events/s", "kind": "oracle", "cpu": cpu_model()}
    t = time.perf_counter()
    ev, k = run(nets[0], t + budget_s)
    dt1 = time.perf_counter() - t
    single = {"value": ev / dt1, "cores": 1, "slices": k, "wall_s": round(dt1, 1)}
    t = time.perf_counter()
    res = list(pool.map(lambda nt: run(nt, t + budget_s), nets))
    dtn = time.perf_counter() - t
    evn = sum(r[0] for r in res)
    out.update(value=evn / dtn, cores=threads, single_core=single,
               sample=f"{threads} oracles of {per_thread} of 1,125,000 targets (all 10M sources, "
                      f"{per_thread * 11250:.2e} synapses each), {spikes} input spikes per 1 ms "
                      f"slice, FP64 deliver + update, {sum(r[1] for r in res)} slices in "
                      f"{dtn:.1f} s on {threads} threads; one thread alone: {k} slices in "
                      f"{dt1:.1f} s",
               nproc=os.cpu_count())
    for nt in nets:
        nt.__del__()
    pool.shutdown()
    return out


def cpu_paper_algorithms(slices: int = 30, threads: int | None = None) -> dict:
    """The paper's own delivery algorithms on the host (Alg. REF, Sec. 3.2;
    Alg. bwTSRB* with B_TS = B_RB = 16, Sec. 4.4): each thread owns a share
    of the 112,500 targets with its own source-indexed table (Sec. 3.1), all
    of the 1.27e9-synapse network in FP64, drawn on the host.  Delivery only,
    of the GPU run's ~900 spikes per 1 ms slice; the same seeded lists for
    both algorithms."""
    from paper_2109_12855_amd import sdcpu, workloads

    base = workloads.ALPHA_112K
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    n = base["n_exc"] + base["n_inh"]
    t0 = time.time()
    net = sdcpu.CpuNet.generate(n_tgt=n, n_src_exc=base["n_exc"], n_src_inh=base["n_inh"],
                                k_exc=base["k_exc"], k_inh=base["k_inh"], d_lo=base["d_lo"],
                                d_hi=base["d_hi"], w_exc=base["w_exc"], g=base["g"],
                                seed=base["seed"], ring_len=base["ring_len"], n_threads=threads)
    build_s = time.time() - t0
    d_min = base["d_min"]
    spikes = int(round(n * 8.0 * d_min * base["h"] * 1e-3))
    lists = [workloads.replay_spikes(n, spikes, d_min, seed=5000 + k) for k in range(slices + 2)]
    out = {"workload": "alpha_112500 tables on the host (1.27e9 synapses, FP64 weights), "
                       "delivery only",
           "threads": net.n_threads, "synapses": net.n_synapses, "build_s": round(build_s, 1),
           "spikes_per_slice": spikes, "slices": slices, "b_ts": 16, "b_rb": 16}
    # ring buffers packed back to back (the GPU path's layout), then inside
    # 1 KB neuron objects (stride 128 cells), as in the simulator the paper
    # studies, where the ring-buffer accesses miss the caches
    for layout, stride in (("packed", base["ring_len"]), ("objects_1kb", 128)):
        net.set_ring_stride(stride)
        for name, alg in (("ref", sdcpu.REF), ("bwtsrb", sdcpu.BWTSRB)):
            net.clear()
            for k in range(2):  # warm-up
                net.deliver(*lists[k], k * d_min, alg=alg)
            ev = 0
            t = time.perf_counter()
            for k in range(slices):
                ev += net.deliver(*lists[k + 2], (k + 2) * d_min, alg=alg)
            dt = time.perf_counter() - t
            key = name if layout == "packed" else f"{name}_{layout}"
            out[key] = {"events_per_s": ev / dt, "ms_per_slice": dt / slices * 1e3}
    net.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500,
                    help="timed slices (1 ms each; 500 = the share's configured 0.5 s)")
    ap.add_argument("--warmup", type=int, default=20, help="untimed slices before timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-threads", type=int, default=None,
                    help="threads of the all-cores oracle baseline (default: all, at most 16)")
    ap.add_argument("--no-cpu-paper", action="store_true",
                    help="skip the multithreaded CPU REF / bwTSRB* comparator")
    ap.add_argument("--forms", default="fp32,bf16,bf16_resid,bf16_packed",
                    help="storage forms of the 112,500-neuron net")
    ap.add_argument("--no-share-fp32", action="store_true",
                    help="skip the FP32 form of the brain-scale share")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the ring errors against the FP64 oracle")
    ap.add_argument("--no-rate-cv", action="store_true",
                    help="skip the rate / CV errors against the FP64 oracle")
    ap.add_argument("--no-plastic", action="store_true",
                    help="skip the plastic-synapse variant of the 112,500-neuron net")
    ap.add_argument("--no-short-delay", action="store_true",
                    help="skip the one-step-slice (d_min = 0.1 ms) workload")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the autotuned 64-network batched sweep")
    ap.add_argument("--no-share-repetitions", action="store_true",
                    help="skip the headline's repetitions with seeds 1, 2, 3")
    ap.add_argument("--no-share-tuning", action="store_true",
                    help="skip the binning-parameter autotuning of the brain-scale share")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain copy of known size (counter calibration)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the brain-scale share's BF16 form (profiling runs)")
    ap.add_argument("--forms-only", action="store_true",
                    help="only the 112,500-neuron net's --forms (profiling runs; the JSON line "
                         "then holds those legs alone)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.headline_only:
        args.no_cpu = args.no_cpu_paper = args.no_share_fp32 = args.no_precision = True
        args.no_rate_cv = args.no_short_delay = args.no_sweep = args.no_plastic = True
        args.no_share_tuning = args.no_share_repetitions = True
        args.forms = ""
    if args.forms_only:
        forms_all = alpha_forms()
        alpha = {f: time_net(forms_all[f], args.steps, args.warmup, settle=SETTLE_SLICES)
                 for f in args.forms.split(",") if f}
        if args.copy_probe:
            copy_probe()
        print(json.dumps({"alpha_112500": alpha, "steps": args.steps, "warmup": args.warmup,
                          "settle_slices": SETTLE_SLICES}), flush=True)
        return
    # headline: the brain-scale share, BF16-residual weights
    head = time_net(share_cfg(2), args.steps, args.warmup, open_loop=True)
    _log("brain share bf16_resid: " + json.dumps(head))
    if args.copy_probe:
        copy_probe()
    share = {"bf16_resid": head}
    if not args.no_share_repetitions:
        reps = [time_net(dict(share_cfg(2), seed=sd, name=f"alpha_share_1125000_bf16_resid_seed{sd}"),
                         args.steps, args.warmup, open_loop=True) for sd in (1, 2, 3)]
        ev = np.array([r["events_per_s"] for r in reps])
        share["repetitions"] = {"seeds": [1, 2, 3],
                                "us_per_slice": [r["us_per_slice"] for r in reps],
                                "events_per_s": ev.tolist(), "mean_events_per_s": float(ev.mean()),
                                "sd_events_per_s": float(ev.std(ddof=1)),
                                "mean_roofline_frac": float(np.mean([r["roofline_frac"] for r in reps]))}
        _log("brain share repetitions: " + json.dumps(share["repetitions"]))
    if not args.no_share_fp32:
        share["fp32"] = time_net(share_cfg(0), args.steps, args.warmup, open_loop=True)
        _log("brain share fp32: " + json.dumps(share["fp32"]))
        share["bf16_over_fp32_events_per_s"] = head["events_per_s"] / share["fp32"]["events_per_s"]
    if not args.no_share_tuning:
        share["tuning"] = share_tuning()
        _log("brain share tuning: " + json.dumps(share["tuning"]))
    forms_all = alpha_forms()
    forms = {f: forms_all[f] for f in args.forms.split(",") if f}
    alpha = {}
    for f, cfg in forms.items():
        alpha[f] = time_net(cfg, args.steps, args.warmup, settle=SETTLE_SLICES)
        _log(f"alpha_112500 {f}: " + json.dumps(alpha[f]))
    pl = None
    if not args.no_plastic:
        from paper_2109_12855_amd import workloads

        pl = time_net(workloads.plastic(forms_all["fp32"]), args.steps, args.warmup,
                      settle=SETTLE_SLICES)
        pl["bytes_per_event"] = PLASTIC_B_EVENT
        if "fp32" in alpha:
            pl["over_static_fp32_events_per_s"] = pl["events_per_s"] / alpha["fp32"]["events_per_s"]
        _log("plastic: " + json.dumps(pl))
    prec = None
    if not args.no_precision and forms:
        prec = ring_errors(forms)
        _log("ring errors: " + json.dumps(prec))
    threads = args.cpu_threads or min(16, os.cpu_count() or 1)
    rcv = None
    if not args.no_rate_cv and "fp32" in forms:
        rcv = rate_cv_errors(forms, threads=threads)
        _log("rate/cv: " + json.dumps(rcv))
    sd = None
    if not args.no_short_delay:
        sd = short_delay()
        _log("short delay: " + json.dumps(sd))
    sw = None
    if not args.no_sweep:
        sw = sweep()
        _log("sweep: " + json.dumps(sw))
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(threads)
        _log("cpu baseline: " + json.dumps(cpu))
    cpu_paper = None
    if not args.no_cpu_paper:
        cpu_paper = cpu_paper_algorithms()
        _log("cpu paper algorithms: " + json.dumps(cpu_paper))
    prof = profile_json(SHARE_TRAFFIC)
    # (not in the profiled headline-only runs: the counter calibration copy
    # must be the only copy there)
    copy = None if args.headline_only else copy_bandwidth()
    if copy:
        _log("copy reference: " + json.dumps(copy))
    roof = {"bound": "hbm", "achieved": round(head["alg_gbs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(head["alg_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": (round(prof["fetch_bytes_per_slice"] + prof["write_bytes_per_slice"])
                        if prof else None),
            "kernel": "one slice: binning pass + fused accumulate/update kernel",
            "alg_bytes_per_slice": head["alg_bytes_per_slice"],
            "l2_hit_rate": prof.get("l2_hit_rate") if prof else None,
            "copy_reference_gbs": round(copy["gbs"], 1) if copy else None,
            "frac_of_copy": round(head["alg_gbs"] / copy["gbs"], 4) if copy else None}
    line = {
        "metric": "synaptic events delivered/s",
        "value": head["events_per_s"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["us_per_slice"] * 1e-3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "alpha_share_1125000_k11250_open_loop", "neurons": 1125000,
                   "in_degree": 11250, "virtual_sources": 10_000_000, "source_rate_hz": 8.0,
                   "synapses": head["synapses"], "slice_ms": 1.0,
                   "weight_storage": "bf16_resid", "layout": head["layout"],
                   "block_neurons": head["block_neurons"], "bin_cap": head["bin_cap"],
                   "parallelism": "single_gpu"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "brain_share": share,
        "alpha_112500": alpha,
        "plastic": pl,
        "ring_errors": prec,
        "rate_cv_errors": rcv,
        "short_delay": sd,
        "sweep": sw,
        "cpu_paper_algorithms": cpu_paper,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
