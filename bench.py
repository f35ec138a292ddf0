"""Benchmark: synaptic events delivered per second on one MI355X.

A step is one slice of the simulation cycle (Sec. 1 / Sec. 2.1 of the
paper): deliver the completed slice's spikes through the connection table
into the ring buffers, then update every neuron through the next d_min
steps with spike compaction -- one fused kernel launch.  The workload is the
112,500-neuron alpha-current balanced random net at in-degree 11,250
(1.27e9 synapses), run closed loop in its self-consistent state; both the
FP32 form (9 B/synapse) and the BF16-residual form (5 B/synapse) are timed,
the latter is the headline ``value``.

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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_slice_alpha_112500_bf16_packed_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2109_12855_amd", "csrc", f)
                  for f in ("sd_kernels.hip", "sd_internal.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per slice launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by what the counter reads
    for a plain copy of known size), or None when the summary is missing or
    was taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
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
    FETCH_SIZE / WRITE_SIZE counters calibrate the slice kernel's."""
    import torch

    n = COPY_PROBE_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    _log(f"copy probe: 3 x {COPY_PROBE_BYTES} B read + written")


def _log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(events: float, spikes: float, n: int, d_min: int, b_syn: int,
                      s_state: int) -> float:
    """Bytes one slice must move: synapses of every delivered event, one ring
    write and one read per neuron-step, neuron state read + write, and the
    spike list (5 B per entry)."""
    return events * b_syn + n * d_min * 8 + n * 2 * s_state + spikes * 5


def run_form(cfg: dict, steps: int, warmup: int, per_launch: bool = True) -> dict:
    import torch

    from paper_2109_12855_amd import sdeliver

    t0 = time.time()
    net = sdeliver.Net(cfg).build()
    torch.cuda.synchronize()
    t_build = time.time() - t0
    d_min = cfg["d_min"]
    _log(f"{cfg['name']}: built {net.n_syn:.3e} synapses in {t_build:.1f} s")
    net.simulate_steps(warmup * d_min)
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
    events = s1["events_delivered"] - s0["events_delivered"]
    spikes = s1["spikes_delivered"] - s0["spikes_delivered"]
    emitted = s1["spikes_emitted"] - s0["spikes_emitted"]
    launches = s1["slices"] - s0["slices"]
    # Every timed step is one fused slice launch and nothing else runs on
    # the stream (torch's current stream is the context's), so the events
    # around the timed region give the kernel's average launch duration.
    k_ms = ms / launches if per_launch and launches > 0 else None
    n = net.n_local
    b_syn = {0: 9, 1: 5, 2: 5, 3: 4}[cfg["wform"]]
    s_state = 16 if cfg["model"] == 1 else 8
    b_alg = algorithmic_bytes(events / steps, spikes / steps, n, d_min, b_syn, s_state)
    out = dict(
        name=cfg["name"], build_s=round(t_build, 2), ms_total=ms, ms_per_step=ms / steps,
        events_per_s=events / (ms * 1e-3), events_per_step=events / steps,
        spikes_per_step=spikes / steps, rate_hz=emitted / (n * steps * d_min * cfg["h"] * 1e-3),
        alg_bytes_per_step=b_alg, alg_gbs=b_alg / (ms / steps * 1e-3) / 1e9,
    )
    if k_ms is not None:
        b_l = algorithmic_bytes(events / launches, spikes / launches, n, d_min, b_syn, s_state)
        out.update(kernel_ms=k_ms, launches=launches, kernel_alg_bytes=b_l,
                   kernel_gbs=b_l / (k_ms * 1e-3) / 1e9)
    net.close()
    del net
    torch.cuda.empty_cache()
    return out


def brain_share(slices: int = 100, warmup: int = 20) -> dict:
    """The one-GPU share of the brain-scale network (1,125,000 alpha
    neurons, in-degree 11,250 from a 10M virtual population firing at 8 Hz,
    1.27e10 synapses, residual-BF16 weights, source-major layout): open-loop
    input precomputed outside the timed region, then timed slices."""
    import torch

    from paper_2109_12855_amd import sdeliver, workloads

    cfg = dict(workloads.ALPHA_BRAIN_SHARE)
    d_min = cfg["d_min"]
    t0 = time.time()
    net = sdeliver.Net(cfg).build()
    torch.cuda.synchronize()
    t_build = time.time() - t0
    net.prepare_input((warmup + slices + 2) * d_min)
    net.simulate_steps(warmup * d_min)
    torch.cuda.synchronize()
    s0 = net.stats()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    net.simulate_steps(slices * d_min)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    s1 = net.stats()
    events = s1["events_delivered"] - s0["events_delivered"]
    spikes = s1["spikes_delivered"] - s0["spikes_delivered"]
    n = net.n_local
    b_syn = net.sizes["bytes_per_synapse"]
    b_alg = algorithmic_bytes(events / slices, spikes / slices, n, d_min, b_syn, 16)
    out = {"workload": "alpha_share_1125000_k11250_open_loop", "synapses": net.n_syn,
           "layout": "source_major", "bytes_per_synapse": b_syn, "build_s": round(t_build, 2),
           "slices": slices, "ms_per_slice": ms / slices, "events_per_slice": events / slices,
           "spikes_per_slice": spikes / slices, "events_per_s": events / (ms * 1e-3),
           "alg_gbs": b_alg / (ms / slices * 1e-3) / 1e9,
           "local_rate_hz": (s1["spikes_emitted"] - s0["spikes_emitted"]) /
                            (n * slices * d_min * cfg["h"] * 1e-3)}
    out["roofline_frac"] = out["alg_gbs"] / HBM_PEAK_GBS
    net.close()
    del net
    torch.cuda.empty_cache()
    return out


def short_delay(slices: int = 5000, warmup: int = 1000) -> dict:
    """The 112,500-neuron net with delays of 1..20 steps (packed records):
    one-step slices, ten times as many per simulated second, each with a
    tenth of the spikes -- the per-slice cost dominates."""
    from paper_2109_12855_amd import workloads

    cfg = dict(workloads.ALPHA_112K_SHORT_DELAY)
    r = run_form(cfg, slices, warmup)
    return {"workload": "alpha_112500_k11250_dmin_0.1ms", "slice_ms": cfg["h"] * cfg["d_min"],
            "slices": slices, "us_per_slice": r["kernel_ms"] * 1e3,
            "events_per_slice": r["events_per_step"], "spikes_per_slice": r["spikes_per_step"],
            "events_per_s": r["events_per_s"], "alg_gbs": r["kernel_gbs"],
            "roofline_frac": r["kernel_gbs"] / HBM_PEAK_GBS, "rate_hz": r["rate_hz"]}


def sweep(slices: int = 120, warmup: int = 20) -> dict:
    """The batched sweep: 64 independent delta networks (N 2,000-40,000, K
    500-5,000, FP32 weights) advanced together, block sizes from the
    autotuner (timed here, no cache), steady-state slices replayed from the
    captured graph; aggregate events/s over all members."""
    import torch

    from paper_2109_12855_amd import sdeliver, workloads

    cfgs = workloads.sweep_nets(64)
    t0 = time.time()
    bn, tune_us = sdeliver.autotune(cfgs, targets=(8, 16, 32, 64, 128, 256), warmup=10,
                                    slices=20)
    t_tune = time.time() - t0
    bt = sdeliver.Batch([dict(c, block_neurons=b) for c, b in zip(cfgs, bn)]).build()
    bt.set_graph(True)
    d_min = cfgs[0]["d_min"]
    bt.simulate_steps(warmup * d_min)
    torch.cuda.synchronize()
    ev0 = sum(m.stats()["events_delivered"] for m in bt.members)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    bt.simulate_steps(slices * d_min)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    ev1 = sum(m.stats()["events_delivered"] for m in bt.members)
    out = {"workload": "sweep_64_delta_nets", "networks": len(cfgs),
           "synapses": int(sum(m.n_syn for m in bt.members)), "slice_ms": d_min * cfgs[0]["h"],
           "tune_s": round(t_tune, 1), "block_neurons_range": [min(bn), max(bn)],
           "blocks": int(sum(m.sizes["n_blocks"] for m in bt.members)),
           "slices": slices, "ms_per_slice": ms / slices,
           "events_per_s": (ev1 - ev0) / (ms * 1e-3), "graph_replays": bt.graph_launches}
    bt.close()
    del bt
    torch.cuda.empty_cache()
    return out


def ring_errors(base: dict, forms: list, n_spikes: int = 900, seed: int = 2021) -> dict:
    """Ring contents of each BF16 storage form against the FP32 form after
    delivering the same replay list (one slice's worth of spikes): normwise
    relative error over all cells, and the largest cell error relative to
    the largest FP32 cell."""
    import torch

    from paper_2109_12855_amd import sdeliver, workloads

    n = base["n_exc"] + base["n_inh"]
    src, lag = workloads.replay_spikes(n, n_spikes, base["d_min"], seed=seed)
    d_src = torch.from_numpy(src.view(np.int32)).cuda()
    d_lag = torch.from_numpy(lag).cuda()
    rings = {}
    for name, wf in [("fp32", 0)] + [(f, {"bf16": 1, "bf16_resid": 2, "bf16_packed": 3}[f])
                                     for f in forms if f != "fp32"]:
        net = sdeliver.Net(dict(base, wform=wf)).build()
        net.deliver(d_src, d_lag, 0)
        rings[name] = net.ring(base["ring_len"]).astype(np.float64)
        net.close()
        del net
        torch.cuda.empty_cache()
    ref = rings.pop("fp32")
    norm = float(np.linalg.norm(ref))
    out = {}
    for name, r in rings.items():
        d = r - ref
        out[name] = {"normwise": float(np.linalg.norm(d) / norm),
                     "max_cell_over_max_ref": float(np.abs(d).max() / np.abs(ref).max())}
    return {"vs": "fp32 form", "spikes": int(len(src)), "forms": out}


def cpu_baseline(cfg: dict, budget_s: float = 12.0, frac: int = 16) -> dict:
    """The FP64 oracle on the host: delivery + update of a 1/frac target
    sample of the same network, fed seeded synthetic spike lists at the
    GPU run's spike count per slice."""
    import oracle
    from paper_2109_12855_amd import workloads

    n = cfg["n_exc"] + cfg["n_inh"]
    n_t = n // frac
    t0 = time.time()
    ref = oracle.Net(cfg, tgt_lo=0, tgt_hi=n_t)
    _log(f"oracle sample built ({ref.n_syn:.2e} synapses) in {time.time() - t0:.1f} s")
    d_min = cfg["d_min"]
    spikes_per_slice = int(round(n * 8.0 * d_min * cfg["h"] * 1e-3))
    events = 0
    slices = 0
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < budget_s:
        src, lag = workloads.replay_spikes(n, spikes_per_slice, d_min, seed=1000 + slices)
        _, ne = ref.deliver(src, lag, ref.t_now - d_min if ref.t_now >= d_min else 0)
        ref.update(d_min)
        events += ne
        slices += 1
    dt = time.perf_counter() - t_start
    return {"value": events / dt, "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_t} of {n} targets (all sources), {slices} slices of "
                      f"{spikes_per_slice} spikes, FP64 deliver+update, single thread, "
                      f"{dt:.1f} s"}


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
    # ring buffers packed back to back (this build's layout), then inside
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
    ap.add_argument("--steps", type=int, default=1000, help="timed slices (1 ms each)")
    ap.add_argument("--warmup", type=int, default=200, help="untimed slices before timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-cpu-paper", action="store_true",
                    help="skip the multithreaded CPU REF / bwTSRB* comparator")
    ap.add_argument("--forms", default="fp32,bf16_resid,bf16_packed")
    ap.add_argument("--no-brain-share", action="store_true",
                    help="skip the 1.27e10-synapse brain-scale share measurement")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the BF16-vs-FP32 ring error report")
    ap.add_argument("--no-short-delay", action="store_true",
                    help="skip the one-step-slice (d_min = 0.1 ms) workload")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the autotuned 64-network batched sweep")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2109_12855_amd import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    base = workloads.ALPHA_112K
    forms = {"fp32": dict(base, wform=0, name="alpha_112500_fp32"),
             "bf16": dict(base, wform=1, name="alpha_112500_bf16"),
             "bf16_resid": dict(base, wform=2, name="alpha_112500_bf16_resid"),
             "bf16_packed": dict(base, wform=3, name="alpha_112500_bf16_packed")}
    res = {}
    for f in args.forms.split(","):
        _log(f"form {f}")
        res[f] = run_form(forms[f], args.steps, args.warmup)
        _log(json.dumps(res[f]))
    if args.copy_probe:
        copy_probe()
    share = None
    if not args.no_brain_share:
        share = brain_share()
        _log("brain share: " + json.dumps(share))
    sd = None
    if not args.no_short_delay:
        sd = short_delay()
        _log("short delay: " + json.dumps(sd))
    sw = None
    if not args.no_sweep:
        sw = sweep()
        _log("sweep: " + json.dumps(sw))
    prec = None
    if not args.no_precision:
        prec = ring_errors(dict(base, name="precision"),
                           [f for f in args.forms.split(",") if f != "fp32"])
        _log("precision: " + json.dumps(prec))
    head_name = next((f for f in ("bf16_packed", "bf16_resid") if f in res), next(iter(res)))
    head = res[head_name]
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(dict(base, wform=0))
    cpu_paper = None
    if not args.no_cpu_paper:
        cpu_paper = cpu_paper_algorithms()
        _log("cpu paper algorithms: " + json.dumps(cpu_paper))
    roof = None
    if "kernel_ms" in head:
        tr = measured_traffic() if head_name == "bf16_packed" else None
        roof = {"bound": "hbm", "achieved": round(head["kernel_gbs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(head["kernel_gbs"] / HBM_PEAK_GBS, 4),
                "traffic": (round(tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"])
                            if tr else None)}
    line = {
        "metric": "synaptic events delivered/s",
        "value": head["events_per_s"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "alpha_112500_k11250_closed_loop", "neurons": 112500,
                   "in_degree": 11250, "synapses": 112500 * 11250, "slice_ms": 1.0,
                   "weight_storage": head_name,
                   "parallelism": "single_gpu"},
        "achieved_alg_gbs": head["alg_gbs"],
        "forms": res,
        "precision": prec,
        "brain_share": share,
        "short_delay": sd,
        "sweep": sw,
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_paper_algorithms": cpu_paper,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
