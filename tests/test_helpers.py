"""The raster comparison used by the GPU parity tests, checked on the CPU
with the oracle standing in for the GPU: identical runs compare clean,
rounding-level perturbations are explained, a real difference is not."""
import numpy as np
import pytest

import oracle
from paper_2109_12855_amd import workloads as W

from helpers import kicked, realization_z, spike_exact


class _OracleAsGpu:
    """An oracle run behind the GPU context's interface (drained raster)."""

    def __init__(self, cfg, V=None):
        self.net = oracle.Net(cfg)
        if V is not None:
            self.net.set_state(V=V)
        self.buf = []

    def simulate_steps(self, n):
        self.buf.append(self.net.simulate(n))

    def spikes(self):
        st = np.concatenate([b[0] for b in self.buf]) if self.buf else np.zeros(0, np.int64)
        idx = np.concatenate([b[1] for b in self.buf]) if self.buf else np.zeros(0, np.uint32)
        self.buf = []
        return st, idx

    def state(self):
        return self.net.state()


CFG = W.tiny(model=0, n=300, k=40, seed=3, d_lo=4, d_hi=9)


def test_identical_runs_compare_clean():
    eps, t_bad, n_cmp, ref = spike_exact(CFG, _OracleAsGpu(CFG), lambda: oracle.Net(CFG),
                                         horizon=300, min_exact=20)
    assert t_bad is None and n_cmp > 100
    assert ref.t_now == 300


def test_rounding_level_perturbation_is_explained():
    V = oracle.Net(CFG).state()["V"] + 1e-9
    eps, t_bad, n_cmp, ref = spike_exact(CFG, _OracleAsGpu(CFG, V), lambda: oracle.Net(CFG),
                                         horizon=300, min_exact=20)
    assert ref.t_now == 300


@pytest.mark.parametrize("min_exact", [20, 400])
def test_real_difference_is_not_explained(min_exact):
    """A 5 mV kick of 20 neurons changes spikes by far more than any FP32
    rounding: the comparison fails inside or after the first window."""
    V = kicked(oracle.Net(CFG).state()["V"], 1)
    with pytest.raises(AssertionError, match="unexplained mismatch"):
        spike_exact(CFG, _OracleAsGpu(CFG, V), lambda: oracle.Net(CFG), horizon=400,
                    min_exact=min_exact)


def test_realization_z():
    rng = np.random.default_rng(5)
    a = rng.normal(10.0, 0.2, 16)
    b = rng.normal(10.0, 0.2, 6)
    assert realization_z(a, b) < 4.5
    assert realization_z(a, b + 1.0) > 4.5
    # one value against a sample: the sample's sd alone
    s = a.std(ddof=1)
    assert np.isclose(realization_z(a, [a.mean() + s]), 1.0 / np.sqrt(1 + 1 / 16))
