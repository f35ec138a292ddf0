"""FP64 CPU oracle for spike delivery (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of ``bench.py`` may
import this package.  The product library never does, and this package never
imports the product library: the two share no code.

``liboracle.so`` is built from ``oracle.c`` with the host C compiler; see
:func:`build`.  Everything numeric happens in the C code; this module only
marshals arguments (ctypes) and numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DELTA, ALPHA = 0, 1
W_FP32, W_BF16, W_BF16_RESID = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Config(C.Structure):
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
        ("tgt_lo", C.c_int64), ("tgt_hi", C.c_int64),
        ("plastic", C.c_int32),
        ("stdp_tau_plus", C.c_double), ("stdp_tau_minus", C.c_double),
        ("stdp_a_plus", C.c_double), ("stdp_a_minus", C.c_double),
        ("stdp_w_max", C.c_double),
    ]


def make_config(d: dict, **over) -> Config:
    """Fill the oracle's config struct from a plain parameter dict."""
    p = dict(d)
    p.update(over)
    c = Config()
    names = {f[0] for f in Config._fields_}
    for k, v in p.items():
        if k in names:
            setattr(c, k, v)
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER
        L.or_philox4x64_10.argtypes = [P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
        L.or_ndtri.argtypes = [C.c_double]
        L.or_ndtri.restype = C.c_double
        L.or_weight_tables.argtypes = [P(Config), C.c_void_p, C.c_void_p]
        L.or_poisson_thresholds.argtypes = [C.c_double, C.c_void_p, C.c_int]
        L.or_poisson_thresholds.restype = C.c_int
        L.or_propagators.argtypes = [P(Config), C.c_void_p]
        L.or_bf16_round.argtypes = [C.c_float]
        L.or_bf16_round.restype = C.c_float
        L.or_decode_weight.argtypes = [P(Config), C.c_int, C.c_float]
        L.or_decode_weight.restype = C.c_float
        L.or_ref_steps.argtypes = [P(Config)]
        L.or_ref_steps.restype = C.c_int32
        L.or_net_create.argtypes = [P(Config)]
        L.or_net_create.restype = C.c_void_p
        L.or_net_destroy.argtypes = [C.c_void_p]
        L.or_last_error.restype = C.c_char_p
        for f in ("or_n_local", "or_n_src", "or_n_syn", "or_t_now"):
            getattr(L, f).argtypes = [C.c_void_p]
            getattr(L, f).restype = C.c_int64
        L.or_export_target_major.argtypes = [C.c_void_p] + [C.c_void_p] * 3
        L.or_export_source_major.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.or_out_weight.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_simulate.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64]
        L.or_simulate.restype = C.c_int64
        L.or_update.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64]
        L.or_update.restype = C.c_int64
        L.or_deliver.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                 P(C.c_double), P(C.c_int64)]
        L.or_deliver.restype = C.c_int
        L.or_read_rb.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.or_read_counts.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.or_read_state.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.or_write_state.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.or_pending.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, P(C.c_int64)]
        L.or_pending.restype = C.c_int64
        L.or_open_loop_spikes.argtypes = [P(Config), C.c_int64, C.c_int32, C.c_void_p,
                                          C.c_void_p, C.c_int64]
        L.or_open_loop_spikes.restype = C.c_int64
        L.or_open_loop_spikes_range.argtypes = [P(Config), C.c_int64, C.c_int32, C.c_int64,
                                                C.c_int64, C.c_void_p, C.c_void_p, C.c_int64]
        L.or_open_loop_spikes_range.restype = C.c_int64
        L.or_read_vpre.argtypes = [C.c_void_p, C.c_void_p]
        L.or_drive_count.argtypes = [C.c_void_p, C.c_int64, C.c_int64]
        L.or_drive_count.restype = C.c_int32
        L.or_stdp_update.argtypes = [P(Config), C.c_double, C.c_int64, C.c_int64, C.c_int64,
                                     C.c_int32]
        L.or_stdp_update.restype = C.c_double
        L.or_read_weights.argtypes = [C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# --- free functions ---------------------------------------------------------
def philox4x64_10(ctr, key) -> np.ndarray:
    c = (C.c_uint64 * 4)(*[int(x) for x in ctr])
    k = (C.c_uint64 * 2)(*[int(x) for x in key])
    o = (C.c_uint64 * 4)()
    lib().or_philox4x64_10(c, k, o)
    return np.array(list(o), dtype=np.uint64)


def ndtri(p: float) -> float:
    return lib().or_ndtri(float(p))


def weight_tables(cfg: dict):
    c = make_config(cfg)
    we = np.zeros(65536, np.float32)
    wi = np.zeros(65536, np.float32)
    lib().or_weight_tables(C.byref(c), _ptr(we), _ptr(wi))
    return we, wi


def poisson_thresholds(lam: float) -> np.ndarray:
    out = np.zeros(64, np.uint32)
    n = lib().or_poisson_thresholds(float(lam), _ptr(out), 64)
    return out[:n].copy()


def propagators(cfg: dict) -> dict:
    c = make_config(cfg)
    out = np.zeros(7, np.float64)
    lib().or_propagators(C.byref(c), _ptr(out))
    return dict(zip(("P11", "P21", "P22", "P31", "P32", "P33", "P30"), out.tolist()))


def bf16_round(x: float) -> float:
    return lib().or_bf16_round(float(x))


def decode_weight(cfg: dict, is_inh: bool, w32: float) -> float:
    c = make_config(cfg)
    return lib().or_decode_weight(C.byref(c), int(is_inh), float(w32))


def stdp_update(cfg: dict, w: float, t_pre: int, t_prev: int, t_last: int, d: int) -> float:
    """One plastic weight update (see or_stdp_update); -1 marks no spike."""
    c = make_config(cfg)
    return lib().or_stdp_update(C.byref(c), float(w), int(t_pre), int(t_prev), int(t_last), int(d))


def ref_steps(cfg: dict) -> int:
    c = make_config(cfg)
    return lib().or_ref_steps(C.byref(c))


def open_loop_spikes(cfg: dict, t0: int, n_steps: int, cap: int = 1 << 22, s_lo=None,
                     s_hi=None):
    """Spikes of the open-loop virtual sources in steps [t0, t0 + n_steps),
    (lag, src) order; with s_lo / s_hi only those of sources [s_lo, s_hi)."""
    c = make_config(cfg)
    src = np.zeros(cap, np.uint32)
    lag = np.zeros(cap, np.uint8)
    if s_lo is None and s_hi is None:
        n = lib().or_open_loop_spikes(C.byref(c), int(t0), int(n_steps), _ptr(src), _ptr(lag), cap)
    else:
        n = lib().or_open_loop_spikes_range(C.byref(c), int(t0), int(n_steps), int(s_lo),
                                            int(s_hi), _ptr(src), _ptr(lag), cap)
    if n < 0:
        raise RuntimeError("open-loop spike capacity exceeded")
    return src[:n].copy(), lag[:n].copy()


def _merge_lag_src(parts):
    """Concatenate (src, lag) lists and order the result by (lag, src)."""
    src = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.uint32)
    lag = np.concatenate([p[1] for p in parts]) if parts else np.zeros(0, np.uint8)
    order = np.lexsort((src, lag))
    return src[order], lag[order]


class Net:
    """One oracle network (FP64 state, FP64 ring buffers, per-cell counts)."""

    def __init__(self, cfg: dict, **over):
        self.cfg = dict(cfg)
        self.cfg.update(over)
        self._c = make_config(self.cfg)
        self._h = lib().or_net_create(C.byref(self._c))
        if not self._h:
            raise ValueError(lib().or_last_error().decode())
        self.n_local = lib().or_n_local(self._h)
        self.n_src = lib().or_n_src(self._h)
        self.n_syn = lib().or_n_syn(self._h)
        self.ring_len = int(self.cfg["ring_len"])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_net_destroy(h)
            self._h = None

    @property
    def t_now(self) -> int:
        return lib().or_t_now(self._h)

    def target_major(self):
        n = self.n_syn
        src = np.zeros(n, np.uint32)
        dly = np.zeros(n, np.uint8)
        widx = np.zeros(n, np.uint16)
        lib().or_export_target_major(self._h, _ptr(src), _ptr(dly), _ptr(widx))
        return src, dly, widx

    def source_major(self):
        row = np.zeros(self.n_src + 1, np.int64)
        tgt = np.zeros(self.n_syn, np.int32)
        dly = np.zeros(self.n_syn, np.uint8)
        w = np.zeros(self.n_syn, np.float64)
        lib().or_export_source_major(self._h, _ptr(row), _ptr(tgt), _ptr(dly), _ptr(w))
        return row, tgt, dly, w

    def out_weight(self):
        w = np.zeros(self.n_src, np.float64)
        d = np.zeros(self.n_src, np.int64)
        lib().or_out_weight(self._h, _ptr(w), _ptr(d))
        return w, d

    def simulate(self, n_steps: int, cap: int = 1 << 24):
        st = np.zeros(cap, np.int64)
        idx = np.zeros(cap, np.uint32)
        n = lib().or_simulate(self._h, int(n_steps), _ptr(st), _ptr(idx), cap)
        if n < 0:
            raise RuntimeError("oracle simulate failed: " + lib().or_last_error().decode())
        return st[:n].copy(), idx[:n].copy()

    def update(self, n_steps: int, cap: int = 1 << 22):
        st = np.zeros(cap, np.int64)
        idx = np.zeros(cap, np.uint32)
        n = lib().or_update(self._h, int(n_steps), _ptr(st), _ptr(idx), cap)
        if n < 0:
            raise RuntimeError("spike capacity exceeded")
        return st[:n].copy(), idx[:n].copy()

    def deliver(self, src, lag, t0: int):
        src = np.ascontiguousarray(src, np.uint32)
        lag = np.ascontiguousarray(lag, np.uint8)
        ws = C.c_double()
        ne = C.c_int64()
        rc = lib().or_deliver(self._h, _ptr(src), _ptr(lag), len(src), int(t0), C.byref(ws),
                              C.byref(ne))
        if rc:
            raise RuntimeError(lib().or_last_error().decode())
        return ws.value, ne.value

    def ring(self, n_slots: int | None = None) -> np.ndarray:
        n_slots = self.ring_len if n_slots is None else n_slots
        out = np.zeros((n_slots, self.n_local), np.float64)
        lib().or_read_rb(self._h, _ptr(out), n_slots)
        return out

    def counts(self, n_slots: int | None = None) -> np.ndarray:
        n_slots = self.ring_len if n_slots is None else n_slots
        out = np.zeros((n_slots, self.n_local), np.uint32)
        lib().or_read_counts(self._h, _ptr(out), n_slots)
        return out

    def state(self):
        n = self.n_local
        v, y1, y2 = (np.zeros(n, np.float64) for _ in range(3))
        r = np.zeros(n, np.int32)
        lib().or_read_state(self._h, _ptr(v), _ptr(y1), _ptr(y2), _ptr(r))
        return {"V": v, "y1": y1, "y2": y2, "r": r}

    def set_state(self, V=None, y1=None, y2=None, r=None):
        arrs = []
        for a, dt in ((V, np.float64), (y1, np.float64), (y2, np.float64), (r, np.int32)):
            arrs.append(None if a is None else np.ascontiguousarray(a, dt))
        lib().or_write_state(self._h, *[(_ptr(a) if a is not None else None) for a in arrs])

    def pending(self):
        cap = 1 << 22
        src = np.zeros(cap, np.uint32)
        lag = np.zeros(cap, np.uint8)
        t0 = C.c_int64()
        n = lib().or_pending(self._h, _ptr(src), _ptr(lag), cap, C.byref(t0))
        return src[:n].copy(), lag[:n].copy(), t0.value

    def vpre(self) -> np.ndarray:
        out = np.zeros(self.n_local, np.float64)
        lib().or_read_vpre(self._h, _ptr(out))
        return out

    def weights(self) -> np.ndarray:
        """Current weights of the source-major table (its (src, target, k)
        order); plastic nets change them at every delivery."""
        out = np.zeros(self.n_syn, np.float64)
        lib().or_read_weights(self._h, _ptr(out))
        return out

    def drive_count(self, j: int, t: int) -> int:
        return lib().or_drive_count(self._h, int(j), int(t))


class Partitioned:
    """The oracle split into target ranges that advance together, one host
    thread per range (ctypes releases the GIL, so the ranges run on separate
    cores).

    Each range is an ordinary oracle ``Net`` holding targets [lo, hi) with
    every source (target sampling).  The cycle is the paper's: every d_min
    steps the ranges are updated, their spikes are gathered into one list in
    (lag, src) order -- the order a single oracle keeps its pending slice in
    -- and that list is delivered to every range (Sec. 2.1: update,
    communicate, deliver).  Open loop, the list is the virtual sources'
    spikes, drawn in source ranges on the same threads.  Every range adds
    the same weights in the same order as an unsplit oracle, so states,
    rings and spikes equal the unsplit oracle's exactly.  ``targets`` limits
    the held neurons to [0, targets) or to a (lo, hi) range (open loop only:
    closed loop needs every neuron's spikes)."""

    def __init__(self, cfg: dict, n_parts: int, threads: int | None = None,
                 targets: int | None = None):
        from concurrent.futures import ThreadPoolExecutor

        self.cfg = dict(cfg)
        n = int(cfg["n_exc"] + cfg["n_inh"])
        self.open = int(cfg.get("n_src_exc", 0)) > 0
        lo, hi = (0, n) if targets is None else (
            (0, int(targets)) if np.isscalar(targets) else (int(targets[0]), int(targets[1])))
        if (lo, hi) != (0, n) and not self.open:
            raise ValueError("a closed-loop net needs every target")
        self.lo, self.hi = lo, hi
        self.bounds = np.linspace(lo, hi, n_parts + 1).astype(np.int64)
        self.pool = ThreadPoolExecutor(max_workers=threads or n_parts)
        self.threads = threads or n_parts
        lo_hi = [(int(a), int(b)) for a, b in zip(self.bounds[:-1], self.bounds[1:]) if b > a]
        self.parts = list(self.pool.map(lambda r: Net(self.cfg, tgt_lo=r[0], tgt_hi=r[1]), lo_hi))
        self.d_min = int(cfg["d_min"])
        self.t_now = 0
        self.pend = None          # (src, lag, t0) of the open slice, closed loop
        self.n_src = self.parts[0].n_src

    def _open_loop_list(self, t0: int):
        n_src = self.n_src
        cuts = np.linspace(0, n_src, self.threads + 1).astype(np.int64)
        cap = int(n_src * self.d_min * 0.01) + 4096
        lists = list(self.pool.map(
            lambda r: open_loop_spikes(self.cfg, t0, self.d_min, cap=cap, s_lo=r[0], s_hi=r[1]),
            [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:])]))
        return _merge_lag_src(lists)

    def simulate(self, n_steps: int):
        """Advance n_steps; returns the spikes (step, id) of the held
        neurons, ordered by (step, id)."""
        out_st, out_id = [], []
        left = int(n_steps)
        while left > 0:
            in_slice = self.t_now % self.d_min
            if in_slice == 0 and self.t_now > 0:
                t0 = self.t_now - self.d_min
                if self.open:
                    src, lag = self._open_loop_list(t0)
                else:
                    src, lag = self.pend[0], self.pend[1]
                list(self.pool.map(lambda p: p.deliver(src, lag, t0), self.parts))
            if in_slice == 0:
                self.pend = (np.zeros(0, np.uint32), np.zeros(0, np.uint8))
            m = min(left, self.d_min - in_slice)
            res = list(self.pool.map(lambda p: p.update(m, cap=p.n_local * m + 1), self.parts))
            st = np.concatenate([r[0] for r in res])
            idx = np.concatenate([r[1] for r in res])
            if not self.open and len(st):
                slice0 = self.t_now - in_slice
                self.pend = _merge_lag_src([self.pend, (idx.astype(np.uint32),
                                                        (st - slice0).astype(np.uint8))])
            out_st.append(st)
            out_id.append(idx)
            self.t_now += m
            left -= m
        st = np.concatenate(out_st) if out_st else np.zeros(0, np.int64)
        idx = np.concatenate(out_id) if out_id else np.zeros(0, np.uint32)
        order = np.lexsort((idx, st))
        return st[order], idx[order]

    def state(self):
        sts = [p.state() for p in self.parts]
        return {k: np.concatenate([s[k] for s in sts]) for k in sts[0]}

    def set_state(self, V=None, y1=None, y2=None, r=None):
        """Overwrite the held neurons' state (arrays over [lo, hi))."""
        off = self.bounds - self.lo
        for p, a, b in zip(self.parts, off[:-1], off[1:]):
            p.set_state(*[None if x is None else np.asarray(x)[a:b] for x in (V, y1, y2, r)])

    def ring(self):
        return np.concatenate([p.ring() for p in self.parts], axis=1)

    def vpre(self):
        return np.concatenate([p.vpre() for p in self.parts])

    def close(self):
        self.parts = []
        self.pool.shutdown()
