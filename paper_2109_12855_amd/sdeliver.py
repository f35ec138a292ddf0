"""Python binding of the C ABI in ``include/sdeliver.h`` (ctypes).

Argument marshalling only: every step of the hot path runs in the gfx950
kernels of ``libsdeliver.so``.  PyTorch supplies the device memory (one
arena tensor per context) and the HIP stream.  If the library has not been
built, :func:`lib` raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdeliver.so")

SD_OK, SD_EINVAL, SD_ENOMEM, SD_EHIP, SD_EOVERFLOW, SD_ESTATE, SD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "SD_OK", -1: "SD_EINVAL", -2: "SD_ENOMEM", -3: "SD_EHIP", -4: "SD_EOVERFLOW",
                -5: "SD_ESTATE", -6: "SD_EUNSUPPORTED"}
SD_IAF_PSC_DELTA, SD_IAF_PSC_ALPHA = 0, 1
SD_W_FP32, SD_W_BF16, SD_W_BF16_RESID, SD_W_BF16_PACKED = 0, 1, 2, 3
SD_LAYOUT_AUTO, SD_LAYOUT_BLOCK, SD_LAYOUT_SOURCE = 0, 1, 2


class SdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class sd_config(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("wform", C.c_int32),
        ("n_exc", C.c_int64), ("n_inh", C.c_int64),
        ("n_src_exc", C.c_int64), ("n_src_inh", C.c_int64),
        ("k_exc", C.c_int32), ("k_inh", C.c_int32),
        ("d_lo", C.c_int32), ("d_hi", C.c_int32),
        ("d_min", C.c_int32), ("d_max", C.c_int32),
        ("ring_len", C.c_int32),
        ("h", C.c_double),
        ("w_exc", C.c_double), ("w_cv", C.c_double), ("g", C.c_double),
        ("tau_m", C.c_double), ("c_m", C.c_double), ("tau_syn", C.c_double),
        ("e_l", C.c_double), ("v_th", C.c_double), ("v_reset", C.c_double),
        ("t_ref", C.c_double), ("i_e", C.c_double),
        ("v0_lo", C.c_double), ("v0_hi", C.c_double),
        ("drive_rate_hz", C.c_double), ("drive_w", C.c_double),
        ("src_rate_hz", C.c_double),
        ("seed", C.c_uint64),
        ("block_neurons", C.c_int32),
        ("record_spikes", C.c_int32),
        ("record_cap", C.c_int64),
        ("layout", C.c_int32),
        ("bin_cap", C.c_int32),
        ("plastic", C.c_int32),
        ("stdp_tau_plus", C.c_double), ("stdp_tau_minus", C.c_double),
        ("stdp_a_plus", C.c_double), ("stdp_a_minus", C.c_double),
        ("stdp_w_max", C.c_double),
    ]


class sd_sizes(C.Structure):
    _fields_ = [
        ("n_local", C.c_int64), ("n_src", C.c_int64), ("n_syn", C.c_int64),
        ("block_neurons", C.c_int32), ("n_blocks", C.c_int32),
        ("table_bytes", C.c_int64), ("arena_bytes", C.c_int64),
        ("bytes_per_synapse", C.c_int32),
        ("layout", C.c_int32),
        ("bin_cap", C.c_int32),
    ]


class sd_stats(C.Structure):
    _fields_ = [
        ("t_now", C.c_int64), ("spikes_emitted", C.c_int64), ("events_delivered", C.c_int64),
        ("spikes_delivered", C.c_int64), ("slices", C.c_int64), ("spikes_recorded", C.c_int64),
        ("overflow", C.c_int32),
    ]


# every symbol include/sdeliver.h declares
EXPORTS = (
    "sd_query_sizes", "sd_create", "sd_destroy", "sd_last_error", "sd_build_connections",
    "sd_update_neurons", "sd_deliver_spikes", "sd_deliver_pending", "sd_simulate", "sd_simulate_steps",
    "sd_set_count_mode", "sd_set_persistent", "sd_set_barrier_spin", "sd_prepare_input", "sd_t_now", "sd_get_sizes", "sd_get_stats",
    "sd_read_ring", "sd_read_state", "sd_write_state", "sd_get_spikes", "sd_get_pending",
    "sd_export_connections", "sd_export_segments", "sd_export_block", "sd_get_tables",
    "sd_host_tables", "sd_batch_create", "sd_batch_destroy", "sd_batch_last_error",
    "sd_batch_size", "sd_batch_member", "sd_batch_build", "sd_batch_simulate_steps",
    "sd_batch_simulate", "sd_batch_set_graph", "sd_batch_graph_launches", "sd_save_state",
    "sd_load_state", "sd_autotune", "sd_autotune_bins", "sd_deliver_spikes_noalloc",
)

_lib = None


def lib():
    """Load libsdeliver.so (built by ``paper_2109_12855_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    P, vp, i32, i64, dbl = C.POINTER, C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "sd_query_sizes": ([P(sd_config), P(sd_sizes)], i32),
        "sd_create": ([P(sd_config), vp, vp, C.c_size_t, P(vp)], i32),
        "sd_destroy": ([vp], None),
        "sd_last_error": ([vp], C.c_char_p),
        "sd_build_connections": ([vp], i32),
        "sd_update_neurons": ([vp, i32], i32),
        "sd_deliver_spikes": ([vp, vp, vp, i64, i64], i32),
        "sd_deliver_spikes_noalloc": ([vp, vp, vp, i64, i64], i32),
        "sd_deliver_pending": ([vp], i32),
        "sd_simulate": ([vp, dbl], i32),
        "sd_simulate_steps": ([vp, i64], i32),
        "sd_set_count_mode": ([vp, i32], i32),
        "sd_set_persistent": ([vp, i32], i32),
        "sd_set_barrier_spin": ([vp, i64], i32),
        "sd_prepare_input": ([vp, i64], i32),
        "sd_t_now": ([vp], i64),
        "sd_get_sizes": ([vp, P(sd_sizes)], i32),
        "sd_get_stats": ([vp, P(sd_stats)], i32),
        "sd_read_ring": ([vp, vp, i32], i32),
        "sd_read_state": ([vp, vp, vp, vp, vp], i32),
        "sd_write_state": ([vp, vp, vp, vp, vp], i32),
        "sd_get_spikes": ([vp, vp, vp, i64, P(i64)], i32),
        "sd_get_pending": ([vp, vp, vp, i64, P(i64), P(i64)], i32),
        "sd_export_connections": ([vp, vp, vp, vp, vp], i32),
        "sd_export_segments": ([vp, i64, vp, vp], i32),
        "sd_get_tables": ([vp, vp, vp, vp, P(i32), vp, vp], i32),
        "sd_export_block": ([vp, i32, vp, vp, vp, vp, P(i64)], i32),
        "sd_host_tables": ([P(sd_config), vp, vp, vp, P(i32)], i32),
        "sd_save_state": ([vp, vp, C.c_size_t, P(C.c_size_t)], i32),
        "sd_load_state": ([vp, vp, C.c_size_t], i32),
        "sd_batch_create": ([P(sd_config), i32, vp, P(vp)], i32),
        "sd_batch_destroy": ([vp], None),
        "sd_batch_last_error": ([vp], C.c_char_p),
        "sd_batch_size": ([vp], i32),
        "sd_batch_member": ([vp, i32], vp),
        "sd_batch_build": ([vp], i32),
        "sd_batch_simulate_steps": ([vp, i64], i32),
        "sd_batch_simulate": ([vp, dbl], i32),
        "sd_batch_set_graph": ([vp, i32], i32),
        "sd_batch_graph_launches": ([vp], i64),
        "sd_autotune": ([P(sd_config), i32, vp, i32, i32, i32, C.c_char_p, vp, P(dbl)], i32),
        "sd_autotune_bins": ([P(sd_config), vp, i32, vp, i32, i32, i32, C.c_char_p,
                              P(C.c_int32), P(C.c_int32), P(dbl)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def make_config(d: dict, **over) -> sd_config:
    p = dict(d)
    p.update(over)
    c = sd_config()
    names = {f[0] for f in sd_config._fields_}
    for k, v in p.items():
        if k in names:
            setattr(c, k, v)
    return c


def query_sizes(cfg: dict, **over) -> dict:
    c = make_config(cfg, **over)
    s = sd_sizes()
    rc = lib().sd_query_sizes(C.byref(c), C.byref(s))
    if rc != SD_OK:
        raise SdError(rc, "sd_query_sizes")
    return {f[0]: getattr(s, f[0]) for f in sd_sizes._fields_}


def host_tables(cfg: dict, **over) -> dict:
    """Weight tables (decoded to the storage form) and Poisson thresholds the
    library computes on the host; needs no device."""
    c = make_config(cfg, **over)
    we = np.zeros(65536, np.float32)
    wi = np.zeros(65536, np.float32)
    thr = np.zeros(64, np.uint32)
    n = C.c_int32()
    rc = lib().sd_host_tables(C.byref(c), _ptr(we), _ptr(wi), _ptr(thr), C.byref(n))
    if rc != SD_OK:
        raise SdError(rc, "sd_host_tables")
    return {"w_e": we, "w_i": wi, "thr": thr[: n.value].copy()}


def _ptr(a) -> C.c_void_p:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())  # torch tensor


class Net:
    """One network on the current CUDA/HIP device.

    ``Net(cfg)`` creates the context (arena from torch, stream from torch),
    ``build()`` draws and lays out the connections, ``simulate(t_ms)`` runs
    the fused slice cycle; ``update`` / ``deliver`` expose the two phases.
    """

    def __init__(self, cfg: dict, stream=None, torch_arena: bool = True, **over):
        """torch_arena: carve the context's device memory out of one torch
        tensor (default) or let the library allocate it with hipMalloc."""
        import torch

        self.cfg = dict(cfg)
        self.cfg.update(over)
        self._c = make_config(self.cfg)
        self.sizes = query_sizes(self.cfg)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.arena = None
        if torch_arena:
            self.arena = torch.empty(int(self.sizes["arena_bytes"]), dtype=torch.uint8,
                                     device=self.device)
        h = C.c_void_p()
        rc = lib().sd_create(C.byref(self._c), C.c_void_p(self.stream.cuda_stream),
                             C.c_void_p(self.arena.data_ptr()) if torch_arena else None,
                             int(self.arena.numel()) if torch_arena else 0, C.byref(h))
        self._h = h
        if rc != SD_OK:
            msg = lib().sd_last_error(h).decode() if h else ""
            if h:
                lib().sd_destroy(h)
            self._h = None
            raise SdError(rc, msg)
        self.n_local = int(self.sizes["n_local"])
        self.n_src = int(self.sizes["n_src"])
        self.n_syn = int(self.sizes["n_syn"])
        self.ring_len = int(self.cfg["ring_len"])

    # -- helpers --------------------------------------------------------------
    def _check(self, rc: int, what: str):
        if rc != SD_OK:
            raise SdError(rc, f"{what}: {lib().sd_last_error(self._h).decode()}")

    @classmethod
    def _member(cls, cfg: dict, handle, owner):
        """A batch member: a borrowed context (the batch owns and frees it)."""
        self = cls.__new__(cls)
        self.cfg = dict(cfg)
        self._c = make_config(self.cfg)
        self.sizes = query_sizes(self.cfg)
        self.arena = None
        self._h = C.c_void_p(handle)
        self._owner = owner
        self.n_local = int(self.sizes["n_local"])
        self.n_src = int(self.sizes["n_src"])
        self.n_syn = int(self.sizes["n_syn"])
        self.ring_len = int(self.cfg["ring_len"])
        return self

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self._h = None  # borrowed from a batch
            return
        if getattr(self, "_h", None):
            lib().sd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the four calls of the method -------------------------------------------
    def build(self):
        self._check(lib().sd_build_connections(self._h), "sd_build_connections")
        return self

    def update(self, n_steps: int):
        self._check(lib().sd_update_neurons(self._h, int(n_steps)), "sd_update_neurons")

    def deliver(self, src=None, lag=None, t0: int = 0):
        """Deliver a device spike list (torch uint32-as-int32 / uint8 tensors), or
        the context's completed slice when ``src`` is None."""
        if src is None:
            rc = lib().sd_deliver_pending(self._h)
        else:
            rc = lib().sd_deliver_spikes(self._h, _ptr(src), _ptr(lag), int(src.numel()), int(t0))
        self._check(rc, "sd_deliver_spikes")

    def deliver_noalloc(self, src, lag, t0: int = 0):
        """Deliver a device spike list with the library's fixed scratch array
        (sd_deliver_spikes_noalloc: no allocation; at most 2^20 entries)."""
        rc = lib().sd_deliver_spikes_noalloc(self._h, _ptr(src), _ptr(lag), int(src.numel()),
                                             int(t0))
        self._check(rc, "sd_deliver_spikes_noalloc")

    def simulate(self, t_ms: float):
        self._check(lib().sd_simulate(self._h, float(t_ms)), "sd_simulate")

    def simulate_steps(self, n: int):
        self._check(lib().sd_simulate_steps(self._h, int(n)), "sd_simulate_steps")

    def prepare_input(self, n_steps: int):
        self._check(lib().sd_prepare_input(self._h, int(n_steps)), "sd_prepare_input")

    def set_count_mode(self, on: bool):
        self._check(lib().sd_set_count_mode(self._h, int(bool(on))), "sd_set_count_mode")

    def set_persistent(self, max_slices: int):
        """Run up to max_slices whole slices per persistent launch (0: one
        launch per slice)."""
        self._check(lib().sd_set_persistent(self._h, int(max_slices)), "sd_set_persistent")

    def set_barrier_spin(self, polls: int):
        """Polls a persistent launch's grid barrier waits before it gives up
        (overflow bit 16); < 0 restores the default."""
        self._check(lib().sd_set_barrier_spin(self._h, int(polls)), "sd_set_barrier_spin")

    # -- read-back --------------------------------------------------------------
    @property
    def t_now(self) -> int:
        return int(lib().sd_t_now(self._h))

    def stats(self) -> dict:
        s = sd_stats()
        rc = lib().sd_get_stats(self._h, C.byref(s))
        out = {f[0]: getattr(s, f[0]) for f in sd_stats._fields_}
        if rc not in (SD_OK, SD_EOVERFLOW):
            self._check(rc, "sd_get_stats")
        return out

    def ring(self, n_slots: int | None = None) -> np.ndarray:
        n_slots = self.ring_len if n_slots is None else n_slots
        out = np.zeros((n_slots, self.n_local), np.float32)
        self._check(lib().sd_read_ring(self._h, _ptr(out), int(n_slots)), "sd_read_ring")
        return out

    def state(self) -> dict:
        n = self.n_local
        v, y1, y2 = (np.zeros(n, np.float32) for _ in range(3))
        r = np.zeros(n, np.int32)
        self._check(lib().sd_read_state(self._h, _ptr(v), _ptr(y1), _ptr(y2), _ptr(r)),
                    "sd_read_state")
        return {"V": v, "y1": y1, "y2": y2, "r": r}

    def set_state(self, V=None, y1=None, y2=None, r=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dt)
                for a, dt in ((V, np.float32), (y1, np.float32), (y2, np.float32), (r, np.int32))]
        self._check(lib().sd_write_state(self._h, *[_ptr(a) for a in arrs]), "sd_write_state")

    def spikes(self, cap: int | None = None):
        """Drain the raster: (step, id) arrays sorted by (step, id)."""
        cap = cap or max(1, self.stats()["spikes_recorded"])
        st = np.zeros(cap, np.int64)
        idx = np.zeros(cap, np.uint32)
        n = C.c_int64()
        rc = lib().sd_get_spikes(self._h, _ptr(st), _ptr(idx), cap, C.byref(n))
        if rc not in (SD_OK,):
            self._check(rc, "sd_get_spikes")
        st, idx = st[: n.value], idx[: n.value]
        order = np.lexsort((idx, st))
        return st[order], idx[order]

    def save_state(self) -> bytes:
        """Checkpoint of the dynamic state (see sd_save_state)."""
        n = C.c_size_t()
        self._check(lib().sd_save_state(self._h, None, 0, C.byref(n)), "sd_save_state")
        buf = C.create_string_buffer(n.value)
        self._check(lib().sd_save_state(self._h, buf, n.value, C.byref(n)), "sd_save_state")
        return buf.raw[: n.value]

    def load_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._check(lib().sd_load_state(self._h, buf, len(data)), "sd_load_state")

    def pending(self):
        cap = self.n_local * int(self.cfg["d_min"])
        src = np.zeros(cap, np.uint32)
        lag = np.zeros(cap, np.uint8)
        n = C.c_int64()
        t0 = C.c_int64()
        self._check(lib().sd_get_pending(self._h, _ptr(src), _ptr(lag), cap, C.byref(n),
                                         C.byref(t0)), "sd_get_pending")
        return src[: n.value], lag[: n.value], t0.value

    def connections(self):
        row = np.zeros(self.n_src + 1, np.int64)
        tgt = np.zeros(self.n_syn, np.int32)
        dly = np.zeros(self.n_syn, np.uint8)
        w = np.zeros(self.n_syn, np.float32)
        self._check(lib().sd_export_connections(self._h, _ptr(row), _ptr(tgt), _ptr(dly), _ptr(w)),
                    "sd_export_connections")
        return row, tgt, dly, w

    def block_table(self, b: int):
        """Synapses into target block b, source-major (row relative to the block)."""
        row = np.zeros(self.n_src + 1, np.int64)
        n = C.c_int64()
        self._check(lib().sd_export_block(self._h, int(b), _ptr(row), None, None, None, C.byref(n)),
                    "sd_export_block")
        tgt = np.zeros(n.value, np.int32)
        dly = np.zeros(n.value, np.uint8)
        w = np.zeros(n.value, np.float32)
        self._check(lib().sd_export_block(self._h, int(b), _ptr(row), _ptr(tgt), _ptr(dly), _ptr(w),
                                          C.byref(n)), "sd_export_block")
        return row, tgt, dly, w

    def segments(self, src: int):
        """(start, length) of source src's segment in every target block."""
        nb = int(self.sizes["n_blocks"])
        start = np.zeros(nb, np.int64)
        length = np.zeros(nb, np.int64)
        self._check(lib().sd_export_segments(self._h, int(src), _ptr(start), _ptr(length)),
                    "sd_export_segments")
        return start, length

    def tables(self) -> dict:
        we = np.zeros(65536, np.float32)
        wi = np.zeros(65536, np.float32)
        thr = np.zeros(64, np.uint32)
        n = C.c_int32()
        p64 = np.zeros(7, np.float64)
        p32 = np.zeros(8, np.float32)
        self._check(lib().sd_get_tables(self._h, _ptr(we), _ptr(wi), _ptr(thr), C.byref(n),
                                        _ptr(p64), _ptr(p32)), "sd_get_tables")
        return {"w_e": we, "w_i": wi, "thr": thr[: n.value].copy(), "prop": p64, "prop32": p32}


class Batch:
    """Independent networks advanced together, one fused launch per slice.

    ``Batch(cfgs)`` creates one context per config (library-allocated
    device memory, torch's current stream), ``build()`` lays out every
    member, ``simulate_steps(n)`` advances all members; ``members[i]`` is a
    borrowed ``Net`` for read-back (spikes, state, ring, stats).
    """

    def __init__(self, cfgs, stream=None):
        import torch

        self.cfgs = [dict(c) for c in cfgs]
        arr = (sd_config * len(self.cfgs))(*[make_config(c) for c in self.cfgs])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = lib().sd_batch_create(arr, len(self.cfgs), C.c_void_p(self.stream.cuda_stream),
                                   C.byref(h))
        self._h = h
        if rc != SD_OK:
            msg = lib().sd_batch_last_error(h).decode() if h else ""
            lib().sd_batch_destroy(h)
            self._h = None
            raise SdError(rc, msg)
        self.members = [Net._member(c, lib().sd_batch_member(self._h, i), self)
                        for i, c in enumerate(self.cfgs)]

    def _check(self, rc: int, what: str):
        if rc != SD_OK:
            raise SdError(rc, f"{what}: {lib().sd_batch_last_error(self._h).decode()}")

    def build(self):
        self._check(lib().sd_batch_build(self._h), "sd_batch_build")
        return self

    def simulate_steps(self, n: int):
        self._check(lib().sd_batch_simulate_steps(self._h, int(n)), "sd_batch_simulate_steps")

    def simulate(self, t_ms: float):
        self._check(lib().sd_batch_simulate(self._h, float(t_ms)), "sd_batch_simulate")

    def set_graph(self, on: bool = True):
        """Run steady-state stretches as replays of a captured HIP graph."""
        self._check(lib().sd_batch_set_graph(self._h, int(bool(on))), "sd_batch_set_graph")
        return self

    @property
    def graph_launches(self) -> int:
        return int(lib().sd_batch_graph_launches(self._h))

    def close(self):
        if getattr(self, "_h", None):
            for m in self.members:
                m._h = None
            lib().sd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(cfgs, targets=(16, 32, 64, 128, 256), warmup: int = 10, slices: int = 20,
             cache: str | None = None):
    """Block sizes for one network (a single config) or a batch (several):
    the fastest of the candidates ceil(N / T) over the targets T, timed on
    the current device (``sd_autotune``).  Returns (block_neurons list,
    microseconds per slice)."""
    cfgs = [dict(c) for c in cfgs]
    arr = (sd_config * len(cfgs))(*[make_config(c) for c in cfgs])
    tg = np.ascontiguousarray(targets, np.int32)
    out = np.zeros(len(cfgs), np.int32)
    us = C.c_double()
    rc = lib().sd_autotune(arr, len(cfgs), _ptr(tg), len(tg), int(warmup), int(slices),
                           cache.encode() if cache else None, _ptr(out), C.byref(us))
    if rc != SD_OK:
        raise SdError(rc, "sd_autotune")
    return [int(x) for x in out], float(us.value)


def autotune_bins(cfg: dict, targets=(1024, 1280, 1536), cap_scales=(0.75, 1.0, 1.5),
                  warmup: int = 5, slices: int = 10, cache: str | None = None):
    """Block size and region capacity of a source-major network's binning
    pass, the fastest pair timed on the current device
    (``sd_autotune_bins``).  Returns (block_neurons, bin_cap, microseconds
    per slice)."""
    c = make_config(dict(cfg))
    tg = np.ascontiguousarray(targets, np.int32)
    sc = np.ascontiguousarray(cap_scales, np.float64)
    bn, cap, us = C.c_int32(), C.c_int32(), C.c_double()
    rc = lib().sd_autotune_bins(C.byref(c), _ptr(tg), len(tg), _ptr(sc), len(sc), int(warmup),
                                int(slices), cache.encode() if cache else None, C.byref(bn),
                                C.byref(cap), C.byref(us))
    if rc != SD_OK:
        raise SdError(rc, "sd_autotune_bins")
    return int(bn.value), int(cap.value), float(us.value)
