"""CPU checks of the C ABI: the library loads, exports every declared symbol,
computes its host tables bit-identically to the oracle, and validates
configurations -- all without a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2109_12855_amd import sdeliver
from paper_2109_12855_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sdeliver.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sd_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = sdeliver.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(sdeliver.EXPORTS)


def test_config_struct_layout_matches_header():
    # size of sd_config as the C compiler lays it out, vs ctypes
    import subprocess
    import tempfile
    src = '#include "sdeliver.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(){printf("%zu %zu %zu %zu\\n", sizeof(sd_config), offsetof(sd_config, seed), sizeof(sd_sizes), sizeof(sd_stats));}\n'
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "t.c")
        open(p, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), p, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == C.sizeof(sdeliver.sd_config)
    assert int(out[1]) == sdeliver.sd_config.seed.offset
    assert int(out[2]) == C.sizeof(sdeliver.sd_sizes)
    assert int(out[3]) == C.sizeof(sdeliver.sd_stats)


@pytest.mark.parametrize("name", ["alpha_112500_fp32", "delta_1250"])
@pytest.mark.parametrize("wform", [0, 1, 2])
def test_host_tables_match_oracle_bitwise(name, wform):
    cfg = dict(W.WORKLOADS[name], wform=wform)
    lt = sdeliver.host_tables(cfg)
    we, wi = oracle.weight_tables(cfg)
    if cfg["w_cv"] == 0.0:
        we[:] = np.float32(cfg["w_exc"])
        wi[:] = np.float32(-cfg["g"] * cfg["w_exc"])
    dec_e = np.array([oracle.decode_weight(cfg, 0, float(x)) for x in we[::97]], np.float32)
    dec_i = np.array([oracle.decode_weight(cfg, 1, float(x)) for x in wi[::97]], np.float32)
    assert np.array_equal(lt["w_e"][::97], dec_e)
    assert np.array_equal(lt["w_i"][::97], dec_i)
    if wform == 0:
        assert np.array_equal(lt["w_e"], we) and np.array_equal(lt["w_i"], wi)
    thr = oracle.poisson_thresholds(cfg["drive_rate_hz"] * cfg["h"] * 1e-3)
    assert np.array_equal(lt["thr"], thr)


def test_sizes_of_workloads():
    s = sdeliver.query_sizes(W.ALPHA_112K)
    assert s["n_syn"] == 112500 * 11250
    assert s["bytes_per_synapse"] == 9
    assert s["block_neurons"] % 64 == 0
    assert s["n_blocks"] * s["block_neurons"] >= 112500
    s3 = sdeliver.query_sizes(W.ALPHA_112K_BF16)
    assert s3["bytes_per_synapse"] == 5
    assert s3["arena_bytes"] < s["arena_bytes"]
    s1 = sdeliver.query_sizes(W.DELTA_SMALL)
    assert s1["n_syn"] == 1250 * 125


@pytest.mark.parametrize("over,code", [
    (dict(d_min=0), sdeliver.SD_EINVAL),
    (dict(d_lo=9), sdeliver.SD_EINVAL),          # below d_min
    (dict(d_hi=21), sdeliver.SD_EINVAL),         # above d_max
    (dict(ring_len=29), sdeliver.SD_EINVAL),     # < d_min + d_max
    (dict(model=7), sdeliver.SD_EINVAL),
    (dict(wform=5), sdeliver.SD_EINVAL),
    (dict(n_exc=0, n_inh=0), sdeliver.SD_EINVAL),
    (dict(block_neurons=100), sdeliver.SD_EINVAL),
    (dict(tau_syn=10.0), sdeliver.SD_EINVAL),    # tau_s == tau_m singularity
    (dict(block_neurons=8192, layout=1), sdeliver.SD_EUNSUPPORTED),  # window > LDS
    (dict(layout=3), sdeliver.SD_EINVAL),
    (dict(block_neurons=2048, layout=2), sdeliver.SD_EINVAL),  # > 1 neuron per thread
])
def test_invalid_configs_rejected(over, code):
    with pytest.raises(sdeliver.SdError) as e:
        sdeliver.query_sizes(W.ALPHA_112K, **over)
    assert e.value.status == code


def test_brain_share_takes_source_major_layout():
    """1.27e10 synapses from 10M virtual sources: beyond the block-major
    layout's 32-bit pointers, so the automatic choice is source-major."""
    s = sdeliver.query_sizes(W.ALPHA_BRAIN_SHARE)
    assert s["layout"] == sdeliver.SD_LAYOUT_SOURCE
    assert s["n_syn"] == 1125000 * 11250
    assert s["n_src"] == 10_000_000
    assert s["bytes_per_synapse"] == 5     # u32 offset|delay|weight high byte + u8
    assert s["arena_bytes"] < 100 * 2**30
    with pytest.raises(sdeliver.SdError) as e:
        sdeliver.query_sizes(W.ALPHA_BRAIN_SHARE, layout=1)
    assert e.value.status == sdeliver.SD_EUNSUPPORTED


def test_layout_choice():
    assert sdeliver.query_sizes(W.ALPHA_112K)["layout"] == sdeliver.SD_LAYOUT_BLOCK
    s = sdeliver.query_sizes(W.ALPHA_112K, layout=2)
    assert s["layout"] == sdeliver.SD_LAYOUT_SOURCE
    assert s["bytes_per_synapse"] == 8
    assert sdeliver.query_sizes(W.ALPHA_112K_BF16, layout=2)["bytes_per_synapse"] == 5


def test_sizes_report_bin_cap():
    """The region capacity in use: the automatic one follows its stated rule
    (expected records per (block, binning workgroup) region at the source
    rate, x1.25 + 6 sd + 64, rounded up to 64), a configured one is kept,
    and block-major layouts report 0."""
    import math

    c = W.ALPHA_BRAIN_SHARE
    s = sdeliver.query_sizes(c)
    spikes = (c["n_src_exc"] + c["n_src_inh"]) * c["src_rate_hz"] * c["d_min"] * c["h"] * 1e-3
    e = spikes / 256 * (s["n_syn"] / s["n_src"]) / s["n_blocks"]
    want = int(math.ceil(1.25 * e + 6 * math.sqrt(e) + 64))
    assert s["bin_cap"] == (want + 63) // 64 * 64 == 576
    assert sdeliver.query_sizes(c, bin_cap=320)["bin_cap"] == 320
    assert sdeliver.query_sizes(W.ALPHA_112K)["bin_cap"] == 0


def test_autotune_bins_rejects_bad_arguments():
    """Argument checks that need no device: a block-major network, empty or
    non-positive candidate lists."""
    with pytest.raises(sdeliver.SdError) as e:
        sdeliver.autotune_bins(W.ALPHA_112K)
    assert e.value.status == sdeliver.SD_EINVAL
    for over in (dict(targets=()), dict(cap_scales=()), dict(cap_scales=(1.0, -0.5)),
                 dict(targets=(0, 8))):
        with pytest.raises(sdeliver.SdError) as e:
            sdeliver.autotune_bins(W.ALPHA_BRAIN_SHARE, **over)
        assert e.value.status == sdeliver.SD_EINVAL
