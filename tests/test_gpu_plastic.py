"""Plastic synapses on the GPU against the oracle (through the C ABI).

The block-major FP32 delivery variant updates every excitatory weight of a
delivered spike by the nearest-spike pair rule before adding it (Sec. 6
reading, see the oracle), reading the target's recent spikes from a 64-step
history in LDS and writing the weight back into the table.  Checked against
the FP64 oracle: spike-exact rasters (tie-aware, tolerance from the measured
drift), then every weight (FP32 against FP64, within the rounding of the
updates) and the ring buffers; zero amplitudes reproduce the static kernel
bit for bit; the unsupported calls are refused.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2109_12855_amd import sdeliver
from paper_2109_12855_amd import workloads as W

from helpers import spike_exact

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


def _weights_close(cfg, w_gpu, w_ref, n_updates_bound):
    """FP32 weights against FP64: each update rounds w and adds a rounded
    FP32 exponential term (exp2 to a few ulps), so the gap grows by a few
    ulps of w_max per update."""
    tol = n_updates_bound * 8 * np.spacing(np.float32(cfg["stdp_w_max"])) + 1e-7 * cfg["stdp_w_max"]
    err = np.abs(w_gpu.astype(np.float64) - w_ref)
    assert err.max() <= tol, (float(err.max()), tol)


@pytest.mark.parametrize("model,n,k,seed,d_lo,d_hi", [
    (0, 300, 60, 3, 4, 9), (1, 300, 60, 5, 4, 9), (1, 2111, 300, 8, 10, 20),
])
def test_plastic_tiny_vs_oracle(model, n, k, seed, d_lo, d_hi):
    cfg = W.plastic(W.tiny(model=model, n=n, k=k, seed=seed, d_lo=d_lo, d_hi=d_hi),
                    a_plus=0.05, a_minus=0.06)
    cfg["record_spikes"] = 1
    net = sdeliver.Net(cfg).build()
    steps = 60 * cfg["d_min"]
    eps, t_bad, n_cmp, ref = spike_exact(cfg, net, lambda: oracle.Net(cfg), horizon=steps,
                                         min_exact=steps // 3)
    assert n_cmp > 20, n_cmp
    if t_bad is None:
        # identical rasters: every weight and the rings follow the oracle's
        row, tgt, dly, w = net.connections()
        orow, otgt, odly, ow = ref.source_major()
        assert np.array_equal(row, orow) and np.array_equal(tgt, otgt)
        w0 = oracle.Net(dict(cfg, plastic=0)).weights()
        assert (np.abs(ow - w0) > 0).any(), "no weight changed"
        _weights_close(cfg, w, ow, n_updates_bound=steps // cfg["d_min"])
        rb, orb = net.ring().astype(np.float64), ref.ring()
        assert np.allclose(rb, orb, rtol=0, atol=1e-5 * cfg["stdp_w_max"] * cfg["k_exc"])


def test_plastic_delta_1250_spike_exact():
    cfg = W.plastic(dict(W.DELTA_SMALL), a_plus=0.01, a_minus=0.0105)
    cfg["record_spikes"] = 1
    net = sdeliver.Net(cfg).build()
    eps, t_bad, n_cmp, ref = spike_exact(cfg, net, lambda: oracle.Net(cfg), horizon=500,
                                         min_exact=150)
    assert n_cmp > 100, n_cmp


def test_plastic_alpha_112500_spike_exact():
    """The full-size 112,500-neuron net with plastic excitatory synapses:
    50 ms spike-exact against the oracle split over host threads."""
    cfg = W.plastic(dict(W.ALPHA_112K, wform=0))
    cfg["record_spikes"] = 1
    net = sdeliver.Net(cfg).build()

    def ref():
        return oracle.Partitioned(cfg, 16, threads=THREADS)

    eps, t_bad, n_cmp, part = spike_exact(cfg, net, ref, horizon=500, min_exact=5)
    part.close()
    assert n_cmp > 200, n_cmp


def test_zero_amplitudes_equal_static_kernel():
    base = W.tiny(model=1, n=2111, k=300, seed=8, d_lo=10, d_hi=20)
    runs = []
    for cfg in (dict(base, record_spikes=1),
                dict(W.plastic(base, a_plus=0.0, a_minus=0.0), record_spikes=1)):
        net = sdeliver.Net(cfg).build()
        net.simulate_steps(400)
        runs.append((net.spikes(), net.ring(), net.state(), net.connections()[3]))
        net.close()
    (sa, ra, xa, wa), (sb, rb, xb, wb) = runs
    assert len(sa[0]) > 50
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
    assert np.array_equal(ra.view(np.uint32), rb.view(np.uint32))
    assert np.array_equal(xa["V"], xb["V"])
    assert np.array_equal(wa, wb)


def test_plastic_refusals():
    cfg = W.plastic(W.tiny(model=1, n=300, k=60, seed=5, d_lo=4, d_hi=9))
    net = sdeliver.Net(cfg).build()
    s = torch.zeros(1, dtype=torch.int32, device="cuda")
    l = torch.zeros(1, dtype=torch.uint8, device="cuda")
    for call in (lambda: net.deliver(s, l, 0), lambda: net.set_count_mode(True),
                 lambda: net.save_state()):
        with pytest.raises(sdeliver.SdError) as e:
            call()
        assert e.value.status == sdeliver.SD_EUNSUPPORTED
    for bad in (dict(wform=2), dict(layout=sdeliver.SD_LAYOUT_SOURCE), dict(d_lo=20, d_hi=50,
                                                                             d_min=20, d_max=50,
                                                                             ring_len=96)):
        with pytest.raises(sdeliver.SdError):
            sdeliver.Net(dict(cfg, **bad))
