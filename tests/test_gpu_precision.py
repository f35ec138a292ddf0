"""BF16 storage forms against the FP32 form on the GPU.

The FP32 form stores the FP32 weight of every synapse; the BF16 forms store
either the weight rounded to BF16, or the BF16 rounding of its residual
d = w / mu_pop - 1 (decoded as mu_pop * (1 + d)).  Fed the same spikes, the
rings differ only by the weight encodings; the bounds below follow from the
BF16 unit roundoff 2^-8 (relative, per weight) and, for the residual, from
|d| being small (weights have a 5% spread).
"""
import numpy as np
import pytest

import oracle
from paper_2109_12855_amd import sdeliver
from paper_2109_12855_amd import workloads as W

from test_gpu_parity import _dev

pytestmark = pytest.mark.gpu

CFG = dict(W.ALPHA_112K, name="alpha_10000", n_exc=8000, n_inh=2000, k_exc=800, k_inh=200)


def _ring(wform, src, lag):
    net = sdeliver.Net(dict(CFG, wform=wform)).build()
    net.deliver(*_dev(src, lag), 0)
    r = net.ring(CFG["ring_len"]).astype(np.float64)
    net.close()
    return r


def _abs_weight_sums(src, lag):
    """Sum of |w| per ring cell from the FP64 oracle's table (FP32 weights)."""
    ref = oracle.Net(dict(CFG, wform=0))
    row, tgt, dly, w = ref.source_major()
    L = CFG["ring_len"]
    out = np.zeros((L, CFG["n_exc"] + CFG["n_inh"]))
    for s, l in zip(src.tolist(), lag.tolist()):
        sl = slice(row[s], row[s + 1])
        np.add.at(out, ((l + dly[sl].astype(np.int64)) % L, tgt[sl]), np.abs(w[sl]))
    return out


def test_bf16_forms_against_fp32():
    n = CFG["n_exc"] + CFG["n_inh"]
    src, lag = W.replay_spikes(n, 600, CFG["d_min"], seed=77)
    fp32 = _ring(0, src, lag)
    bf16 = _ring(1, src, lag)
    resid = _ring(2, src, lag)
    packed = _ring(3, src, lag)
    absw = _abs_weight_sums(src, lag)
    norm = np.linalg.norm(fp32)
    # residual forms: both decode the same residual, and the window sums are
    # exact integers, so the two rings are identical
    assert np.array_equal(resid, packed)
    e_res = np.linalg.norm(resid - fp32) / norm
    e_bf = np.linalg.norm(bf16 - fp32) / norm
    print(f"normwise ring error vs FP32: bf16 {e_bf:.3e}, residual {e_res:.3e}")
    assert e_res <= 1e-3
    # per cell: the residual's error per weight is at most |mu d| 2^-8 <=
    # 2^-8 * 0.34 |w| for |d| < 0.25 (5 sigma); plus FP32 rounding of the
    # window read-out
    assert np.all(np.abs(resid - fp32) <= 2e-3 * absw + 1e-6 * absw + 1e-30)
    # plain BF16 (8 significant bits): at most 2^-8 of each |w| (round to
    # nearest)
    assert np.all(np.abs(bf16 - fp32) <= (2.0 ** -8 + 1e-6) * absw + 1e-30)
    # the residual form is the more accurate of the two by a wide margin
    assert e_res < 0.2 * e_bf
