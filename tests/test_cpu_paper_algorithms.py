"""The paper's delivery algorithms on the CPU (Alg. REF, Sec. 3.2; Alg.
bwTSRB*, Sec. 4.4), multithreaded over thread-local tables (Sec. 3.1).

bwTSRB* only regroups the accesses: the weights of every ring-buffer cell
are added in the same order as in REF (spike entries in list order, a
segment's synapses in table order).  So for any thread count and batch sizes
the rings are bitwise equal to REF's, and to the FP64 oracle, which runs REF
over the same source-major table.
"""
import numpy as np
import pytest

import oracle
from paper_2109_12855_amd import sdcpu
from paper_2109_12855_amd import workloads as W


def _oracle_case(seed=11, n=700, k=120, d_lo=2, d_hi=9):
    cfg = W.tiny(model=1, n=n, k=k, seed=seed, d_lo=d_lo, d_hi=d_hi)
    ref = oracle.Net(cfg)
    row, tgt, dly, w = ref.source_major()
    return cfg, ref, (row, tgt, dly, w)


@pytest.mark.parametrize("threads", [1, 2, 5])
@pytest.mark.parametrize("b_ts,b_rb", [(16, 16), (1, 1), (3, 7), (64, 5)])
@pytest.mark.parametrize("stride", [0, 45])
def test_bwtsrb_equals_ref_and_oracle_bitwise(threads, b_ts, b_rb, stride):
    cfg, ref, (row, tgt, dly, w) = _oracle_case()
    n = cfg["n_exc"] + cfg["n_inh"]
    src, lag = W.replay_spikes(n, 300, cfg["d_min"], seed=4)
    t0 = 5
    ws, ne = ref.deliver(src, lag, t0)
    rings = []
    for alg in (sdcpu.REF, sdcpu.BWTSRB):
        net = sdcpu.CpuNet.from_csr(row, tgt, dly, w, n, cfg["ring_len"], threads)
        assert net.n_threads == threads
        if stride:  # ring buffers inside larger neuron objects
            net.set_ring_stride(stride)
        ev = net.deliver(src, lag, t0, alg=alg, b_ts=b_ts, b_rb=b_rb)
        assert ev == ne
        rings.append(net.ring())
        net.close()
    # bitwise: the same FP64 additions in the same order per cell
    assert np.array_equal(rings[0], rings[1])
    assert np.array_equal(rings[0], ref.ring())
    assert rings[0].sum() != 0.0


def test_repeated_deliveries_and_wrap():
    """Several slices into the same rings, arrival steps wrapping the ring."""
    cfg, ref, (row, tgt, dly, w) = _oracle_case(seed=3, n=400, k=60, d_lo=3, d_hi=7)
    n = cfg["n_exc"] + cfg["n_inh"]
    a = sdcpu.CpuNet.from_csr(row, tgt, dly, w, n, cfg["ring_len"], 3)
    b = sdcpu.CpuNet.from_csr(row, tgt, dly, w, n, cfg["ring_len"], 2)
    L = cfg["ring_len"]
    for k in range(4):
        src, lag = W.replay_spikes(n, 80, cfg["d_min"], seed=20 + k)
        t0 = 22 + k * cfg["d_min"]  # arrivals past step L wrap
        a.deliver(src, lag, t0, alg=sdcpu.REF)
        b.deliver(src, lag, t0, alg=sdcpu.BWTSRB, b_ts=16, b_rb=16)
    ra, rb = a.ring(), b.ring()
    assert np.array_equal(ra, rb)
    # every weight of every delivered synapse is in the rings: totals agree
    # with the table (summed per source, in a different order)
    tot = 0.0
    for k in range(4):
        src, _ = W.replay_spikes(n, 80, cfg["d_min"], seed=20 + k)
        for s in src.tolist():
            tot += float(w[row[s]:row[s + 1]].sum())
    assert ra.sum() == pytest.approx(tot, rel=1e-12, abs=1e-9)
    a.clear()
    assert not a.ring().any()
    assert L == a.ring_len


def test_empty_list_and_invalid_arguments():
    cfg, ref, (row, tgt, dly, w) = _oracle_case(seed=5, n=200, k=40)
    n = cfg["n_exc"] + cfg["n_inh"]
    net = sdcpu.CpuNet.from_csr(row, tgt, dly, w, n, cfg["ring_len"], 2)
    e = np.zeros(0, np.uint32)
    assert net.deliver(e, e.astype(np.uint8), 0, alg=sdcpu.BWTSRB) == 0
    assert not net.ring().any()
    with pytest.raises(ValueError):
        net.deliver(np.array([n + 5], np.uint32), np.zeros(1, np.uint8), 0)  # source out of range
    with pytest.raises(ValueError):
        net.deliver(np.array([0], np.uint32), np.zeros(1, np.uint8), 0, alg=sdcpu.BWTSRB, b_ts=0)
    with pytest.raises(ValueError):
        net.deliver(np.array([0], np.uint32), np.zeros(1, np.uint8), 0, alg=7)
    with pytest.raises(ValueError):
        net.set_ring_stride(cfg["ring_len"] - 1)  # rings would overlap
    bad = dly.copy()
    bad[0] = cfg["ring_len"]  # delay does not fit the ring
    with pytest.raises(ValueError):
        sdcpu.CpuNet.from_csr(row, tgt, bad, w, n, cfg["ring_len"], 2)
    bad_row = row.copy()
    bad_row[3], bad_row[4] = bad_row[4], bad_row[3] - 1  # decreasing offsets
    with pytest.raises(ValueError):
        sdcpu.CpuNet.from_csr(bad_row, tgt, dly, w, n, cfg["ring_len"], 2)
    bad_tgt = tgt.copy()
    bad_tgt[-1] = n  # target out of range
    with pytest.raises(ValueError):
        sdcpu.CpuNet.from_csr(row, bad_tgt, dly, w, n, cfg["ring_len"], 2)


def test_generated_network_thread_invariant():
    """The drawn benchmark network: K synapses per target, the same rings
    for any thread count and both algorithms, every event delivered."""
    kw = dict(n_tgt=3000, n_src_exc=8000, n_src_inh=2000, k_exc=80, k_inh=20, d_lo=10, d_hi=20,
              w_exc=45.6, g=5.0, seed=9, ring_len=32)
    nets = [sdcpu.CpuNet.generate(n_threads=t, **kw) for t in (1, 4)]
    assert all(x.n_synapses == 3000 * 100 for x in nets)
    rng = np.random.default_rng(1)
    src = rng.choice(10000, size=500, replace=False).astype(np.uint32)
    lag = rng.integers(0, 10, size=500).astype(np.uint8)
    ev = [nets[0].deliver(src, lag, 7, alg=sdcpu.REF),
          nets[1].deliver(src, lag, 7, alg=sdcpu.BWTSRB, b_ts=16, b_rb=16)]
    assert ev[0] == ev[1] > 0
    r0, r1 = nets[0].ring(), nets[1].ring()
    assert np.array_equal(r0, r1)
    # mean in-degree per target: K * n_spikes / n_src events per target
    assert ev[0] == pytest.approx(3000 * 100 * 500 / 10000, rel=0.05)
    # arrivals only at slots (7 + lag + d) mod 32 with d in [10, 20]
    used = np.nonzero(np.abs(r0).sum(axis=1))[0]
    assert set(used.tolist()) <= {(7 + l + d) % 32 for l in range(10) for d in range(10, 21)}
