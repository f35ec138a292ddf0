"""ctypes binding of libsdcpu.so: the paper's delivery algorithms (Alg. REF,
Sec. 3.2; Alg. bwTSRB*, Sec. 4.4) as a multithreaded CPU comparator of the
GPU path.  Argument marshalling only; see include/sdcpu.h."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

REF, BWTSRB = 0, 1
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.CPU_LIB):
            _build.build_cpu()
        L = C.CDLL(_build.CPU_LIB)
        vp, i32, i64, u64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        L.sdc_create_from_csr.argtypes = [i64, i64, vp, vp, vp, vp, i32, i32]
        L.sdc_create_from_csr.restype = vp
        L.sdc_generate.argtypes = [i64, i64, i64, i32, i32, i32, i32, f64, f64, u64, i32, i32]
        L.sdc_generate.restype = vp
        L.sdc_deliver.argtypes = [vp, vp, vp, i64, i64, i32, i32, i32]
        L.sdc_deliver.restype = i64
        L.sdc_read_ring.argtypes = [vp, vp]
        L.sdc_read_ring.restype = C.c_int
        L.sdc_clear.argtypes = [vp]
        L.sdc_set_ring_stride.argtypes = [vp, i32]
        L.sdc_set_ring_stride.restype = C.c_int
        L.sdc_n_synapses.argtypes = [vp]
        L.sdc_n_synapses.restype = i64
        L.sdc_n_threads.argtypes = [vp]
        L.sdc_n_threads.restype = i32
        L.sdc_destroy.argtypes = [vp]
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class CpuNet:
    """Thread-local synapse tables and FP64 ring buffers on the host."""

    def __init__(self, handle, n_tgt: int, ring_len: int):
        if not handle:
            raise ValueError("sdc: invalid network description")
        self._h = handle
        self.n_tgt = int(n_tgt)
        self.ring_len = int(ring_len)

    @classmethod
    def from_csr(cls, row, tgt, dly, w, n_tgt: int, ring_len: int, n_threads: int):
        row = np.ascontiguousarray(row, np.int64)
        tgt = np.ascontiguousarray(tgt, np.int32)
        dly = np.ascontiguousarray(dly, np.uint8)
        w = np.ascontiguousarray(w, np.float64)
        h = lib().sdc_create_from_csr(len(row) - 1, int(n_tgt), _p(row), _p(tgt), _p(dly), _p(w),
                                      int(ring_len), int(n_threads))
        return cls(h, n_tgt, ring_len)

    @classmethod
    def generate(cls, n_tgt, n_src_exc, n_src_inh, k_exc, k_inh, d_lo, d_hi, w_exc, g, seed,
                 ring_len, n_threads):
        h = lib().sdc_generate(int(n_tgt), int(n_src_exc), int(n_src_inh), int(k_exc), int(k_inh),
                               int(d_lo), int(d_hi), float(w_exc), float(g), int(seed),
                               int(ring_len), int(n_threads))
        return cls(h, n_tgt, ring_len)

    def deliver(self, src, lag, t0: int, alg: int = REF, b_ts: int = 16, b_rb: int = 16) -> int:
        src = np.ascontiguousarray(src, np.uint32)
        lag = np.ascontiguousarray(lag, np.uint8)
        ev = lib().sdc_deliver(self._h, _p(src), _p(lag), len(src), int(t0), int(alg), int(b_ts),
                               int(b_rb))
        if ev < 0:
            raise ValueError("sdc_deliver: invalid arguments")
        return int(ev)

    def ring(self) -> np.ndarray:
        out = np.zeros((self.ring_len, self.n_tgt), np.float64)
        lib().sdc_read_ring(self._h, _p(out))
        return out

    def clear(self):
        lib().sdc_clear(self._h)

    def set_ring_stride(self, stride: int):
        """Ring buffers inside neuron objects of `stride` cells (zeroes them)."""
        if lib().sdc_set_ring_stride(self._h, int(stride)) != 0:
            raise ValueError("sdc_set_ring_stride: stride below ring_len or out of memory")

    @property
    def n_synapses(self) -> int:
        return int(lib().sdc_n_synapses(self._h))

    @property
    def n_threads(self) -> int:
        return int(lib().sdc_n_threads(self._h))

    def close(self):
        if self._h:
            lib().sdc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
