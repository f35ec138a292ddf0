"""sd_deliver_spikes_noalloc (fixed device scratch array, no allocation)
against sd_deliver_spikes (the context's own list buffer), through the C ABI.

Both pack the same list and run the same delivery kernels; the window sums
are exact integers, so the rings must be bitwise equal after every call.
Two calls in a row, the second with a smaller list (the array keeps the
first call's longer contents), on both table layouts, then a closed-loop
run continued from the externally delivered state.
"""
import numpy as np
import pytest
import torch

from paper_2109_12855_amd import sdeliver
from paper_2109_12855_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(src, lag):
    return (torch.from_numpy(np.ascontiguousarray(src).view(np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(lag)).cuda())


@pytest.mark.parametrize("layout", [sdeliver.SD_LAYOUT_BLOCK, sdeliver.SD_LAYOUT_SOURCE])
@pytest.mark.parametrize("wform", [0, 3])
def test_noalloc_matches_deliver_spikes(layout, wform):
    if layout == sdeliver.SD_LAYOUT_SOURCE and wform == 3:
        pytest.skip("the packed form is block-major only")
    cfg = dict(W.tiny(model=1, n=2111, k=300, seed=8, d_lo=10, d_hi=20), wform=wform,
               layout=layout, record_spikes=1)
    n = cfg["n_exc"] + cfg["n_inh"]
    a = sdeliver.Net(cfg).build()
    b = sdeliver.Net(cfg).build()
    calls = [(W.replay_spikes(n, 5000, cfg["d_min"], seed=1), 0),
             (W.replay_spikes(n, 700, cfg["d_min"], seed=2), 0)]   # smaller second list
    for (src, lag), t0 in calls:
        ds, dl = _dev(src, lag)
        a.deliver(ds, dl, t0)
        b.deliver_noalloc(ds, dl, t0)
        torch.cuda.synchronize()
        ra, rb = a.ring(), b.ring()
        assert np.abs(ra).sum() > 0
        assert np.array_equal(ra.view(np.uint32), rb.view(np.uint32))
        sa, sb = a.stats(), b.stats()
        assert sa["events_delivered"] == sb["events_delivered"] > 0
        assert sa["overflow"] == sb["overflow"] == 0
    # both contexts go on identically from the delivered rings
    a.update(cfg["d_min"])
    b.update(cfg["d_min"])
    a.simulate_steps(95)
    b.simulate_steps(95)
    sa, ia = a.spikes()
    sb, ib = b.spikes()
    assert len(sa) > 0
    assert np.array_equal(sa, sb) and np.array_equal(ia, ib)


def test_noalloc_limits_and_invalid_entries():
    cfg = W.tiny(model=0, n=1000, k=100, seed=6, d_lo=10, d_hi=20)
    net = sdeliver.Net(cfg).build()
    # beyond the context's list capacity (smaller than the array here)
    big = net.sizes["n_blocks"] * net.sizes["block_neurons"] * cfg["d_min"] + 1
    ds, dl = _dev(np.zeros(big, np.uint32), np.zeros(big, np.uint8))
    with pytest.raises(sdeliver.SdError) as e:
        net.deliver_noalloc(ds, dl, 0)
    assert e.value.status == sdeliver.SD_EINVAL
    # an invalid entry delivers nothing and raises the sticky flag
    ref = sdeliver.Net(cfg).build()
    src = np.array([3, 10**6, 7], np.uint32)
    lag = np.array([0, 1, 2], np.uint8)
    net.deliver_noalloc(*_dev(src, lag), 0)
    ref.deliver(*_dev(src[[0, 2]], lag[[0, 2]]), 0)
    assert np.array_equal(net.ring().view(np.uint32), ref.ring().view(np.uint32))
    with pytest.raises(sdeliver.SdError) as e:
        net.stats()
    assert e.value.status == sdeliver.SD_EINVAL
