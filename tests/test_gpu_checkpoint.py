"""Checkpoint / resume on the GPU: a run saved at step t and resumed in a
fresh context equals the uninterrupted run (spikes, state, statistics)."""
import numpy as np
import pytest

from paper_2109_12855_amd import sdeliver
from paper_2109_12855_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,t_save,t_end", [
    (dict(W.DELTA_SMALL, record_spikes=1), 237, 500),
    (dict(W.tiny(model=1, n=300, k=30, seed=4), record_spikes=1), 300, 610),
    (dict(W.ALPHA_112K, wform=3, record_spikes=1), 150, 300),
    (dict(W.tiny(model=1, n=300, k=30, seed=4), record_spikes=1,
          layout=sdeliver.SD_LAYOUT_SOURCE), 300, 610),
])
def test_resume_equals_uninterrupted(cfg, t_save, t_end):
    a = sdeliver.Net(cfg).build()
    a.simulate_steps(t_save)
    blob = a.save_state()
    a.simulate_steps(t_end - t_save)
    st_a, id_a = a.spikes()
    b = sdeliver.Net(cfg).build()
    b.load_state(blob)
    assert b.t_now == t_save
    b.simulate_steps(t_end - t_save)
    st_b, id_b = b.spikes()  # the raster is not part of the checkpoint
    late = st_a >= t_save
    assert np.array_equal(st_a[late], st_b) and np.array_equal(id_a[late], id_b)
    sa, sb = a.state(), b.state()
    for k in ("V", "y1", "y2", "r"):
        assert np.array_equal(sa[k], sb[k]), k
    xa, xb = a.stats(), b.stats()
    for k in ("t_now", "events_delivered", "spikes_delivered", "spikes_emitted", "slices"):
        assert xa[k] == xb[k], k


@pytest.mark.parametrize("layout", [sdeliver.SD_LAYOUT_BLOCK, sdeliver.SD_LAYOUT_SOURCE])
def test_resume_open_loop(layout):
    """Open loop: the resumed context prepares the input schedule from the
    checkpoint's step on and continues exactly."""
    from test_gpu_source_major import _open_loop_small
    cfg = dict(_open_loop_small(), layout=layout)
    a = sdeliver.Net(cfg).build()
    a.prepare_input(600)
    a.simulate_steps(255)
    blob = a.save_state()
    a.simulate_steps(245)
    b = sdeliver.Net(cfg).build()
    b.load_state(blob)
    b.prepare_input(245)
    b.simulate_steps(245)
    st_a, id_a = a.spikes()
    st_b, id_b = b.spikes()
    late = st_a >= 255
    assert late.sum() > 0
    assert np.array_equal(st_a[late], st_b) and np.array_equal(id_a[late], id_b)
    for k in ("V", "y1", "y2", "r"):
        assert np.array_equal(a.state()[k], b.state()[k]), k
    for k in ("events_delivered", "spikes_delivered", "slices"):
        assert a.stats()[k] == b.stats()[k], k


def test_load_rejects_other_configuration():
    a = sdeliver.Net(W.DELTA_SMALL).build()
    a.simulate_steps(20)
    blob = a.save_state()
    b = sdeliver.Net(dict(W.DELTA_SMALL, seed=2)).build()
    with pytest.raises(sdeliver.SdError) as e:
        b.load_state(blob)
    assert e.value.status == sdeliver.SD_EINVAL
    with pytest.raises(sdeliver.SdError):
        b.load_state(b"not a state buffer" * 10)
