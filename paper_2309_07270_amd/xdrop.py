"""Thin ctypes binding of libxdrop.so (include/xdrop.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  If the library has not been built the import of a
binding function raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .workload import RECORD_DTYPE, RESULT_DTYPE, ReadStore, ASCII

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxdrop.so")

XDROP_OK = 0
XDROP_E_INVALID = -1
XDROP_E_NOMEM = -2
XDROP_E_DEVICE = -3
XDROP_E_TIMEOUT = -4
XDROP_E_BUSY = -5
XDROP_E_STATE = -6
MODE_PERSISTENT = 0
MODE_PLAIN = 1
MAX_X = 1 << 30

NOALLOC_BYTES = 128 << 20
NOALLOC_MAX_RECORDS = 1 << 19

EXPORTED = ("xdrop_batch_create", "xdrop_batch_submit", "xdrop_batch_submit_device", "xdrop_batch_wait",
            "xdrop_batch_destroy", "xdrop_batch_footprint", "xdrop_get_tuning", "xdrop_set_tuning",
            "xdrop_autotune", "xdrop_find_seeds", "xdrop_status_string", "xdrop_last_error",
            "xdrop_batch_run_noalloc")


class Config(ctypes.Structure):
    _fields_ = [("reads", ctypes.POINTER(ctypes.c_char_p)), ("lengths", ctypes.POINTER(ctypes.c_uint32)),
                ("n_reads", ctypes.c_uint32), ("device", ctypes.c_int32), ("mode", ctypes.c_uint32),
                ("max_inflight", ctypes.c_uint32), ("hbm_budget_bytes", ctypes.c_uint64),
                ("tuning_cache", ctypes.c_char_p), ("flags", ctypes.c_uint32)]


NUM_STAGES = 7
STAGE_NAMES = ("ingest", "narrow", "adaptive", "wide1280", "wide2048", "generic", "finalize")
FLAG_PROFILE = 1


class Stats(ctypes.Structure):
    _fields_ = [("records", ctypes.c_uint64), ("cells", ctypes.c_uint64), ("queue_ms", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("stage_ms", ctypes.c_double * NUM_STAGES), ("stage_cells", ctypes.c_uint64 * NUM_STAGES),
                ("stage_tasks", ctypes.c_uint64 * NUM_STAGES), ("stage_slots", ctypes.c_uint64 * NUM_STAGES)]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if hasattr(v, "__len__") else v
        return out


class SeedParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("stride", ctypes.c_uint32), ("lo", ctypes.c_uint32),
                ("hi", ctypes.c_uint32), ("x", ctypes.c_int32), ("match", ctypes.c_int16),
                ("mismatch", ctypes.c_int16), ("gap", ctypes.c_int16), ("pad", ctypes.c_int16)]


class SeedStats(ctypes.Structure):
    _fields_ = [("kmers", ctypes.c_uint64), ("distinct", ctypes.c_uint64), ("reliable", ctypes.c_uint64),
                ("pairs", ctypes.c_uint64), ("device_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("grow_margin", ctypes.c_int32), ("shrink_margin", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("buckets", ctypes.c_int32),
                ("generic_waves", ctypes.c_int32), ("narrow_x", ctypes.c_int32),
                ("narrow_min_records", ctypes.c_int32), ("wide_waves", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class XdropError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"xdrop status {status}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libxdrop.so; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libxdrop.so not built at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.xdrop_batch_create.argtypes = [P(Config), P(vp)]
    lib.xdrop_batch_submit.argtypes = [vp, vp, ctypes.c_size_t, vp, vp, ctypes.c_int64, P(ctypes.c_uint64)]
    lib.xdrop_batch_submit_device.argtypes = [vp, vp, ctypes.c_size_t, vp, vp, vp, P(ctypes.c_uint64)]
    lib.xdrop_batch_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_int64, P(Stats)]
    lib.xdrop_batch_run_noalloc.argtypes = [vp, vp, ctypes.c_size_t, vp, vp, vp, vp]
    lib.xdrop_batch_run_noalloc.restype = ctypes.c_int
    lib.xdrop_batch_destroy.argtypes = [vp]
    lib.xdrop_status_string.argtypes = [ctypes.c_int]
    lib.xdrop_status_string.restype = ctypes.c_char_p
    lib.xdrop_last_error.argtypes = [vp]
    lib.xdrop_last_error.restype = ctypes.c_char_p
    lib.xdrop_batch_footprint.argtypes = [vp, ctypes.c_size_t]
    lib.xdrop_batch_footprint.restype = ctypes.c_uint64
    lib.xdrop_get_tuning.argtypes = [vp, P(Tuning)]
    lib.xdrop_set_tuning.argtypes = [vp, P(Tuning)]
    lib.xdrop_autotune.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_char_p, P(ctypes.c_double)]
    lib.xdrop_find_seeds.argtypes = [vp, P(SeedParams), vp, ctypes.c_size_t, ctypes.c_int, P(ctypes.c_size_t),
                                     P(SeedStats)]
    for f in ("xdrop_get_tuning", "xdrop_set_tuning", "xdrop_autotune"):
        getattr(lib, f).restype = ctypes.c_int
    for f in ("xdrop_batch_create", "xdrop_batch_submit", "xdrop_batch_submit_device", "xdrop_batch_wait",
              "xdrop_batch_destroy"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a) -> int:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())  # torch tensor


class Context:
    """One xdrop context: a device-resident read store plus batch execution."""

    def __init__(self, reads, device: int = 0, mode: int = MODE_PERSISTENT, max_inflight: int = 4,
                 hbm_budget_bytes: int = 0, tuning_cache: str | None = None, profile: bool = False):
        self.lib = load_library()
        if isinstance(reads, ReadStore):
            seqs = [ASCII[reads.read(r)].tobytes() for r in range(reads.n)]
        else:
            seqs = [s.encode() if isinstance(s, str) else bytes(s) for s in reads]
        self._seqs = seqs
        arr = (ctypes.c_char_p * len(seqs))(*seqs)
        lens = (ctypes.c_uint32 * len(seqs))(*[len(s) for s in seqs])
        cfg = Config(arr, lens, len(seqs), device, mode, max_inflight, hbm_budget_bytes,
                     tuning_cache.encode() if tuning_cache else None, FLAG_PROFILE if profile else 0)
        h = ctypes.c_void_p()
        st = self.lib.xdrop_batch_create(ctypes.byref(cfg), ctypes.byref(h))
        self._seqs = None
        if st != XDROP_OK:
            raise XdropError(st, self.lib.xdrop_last_error(None).decode())
        self.h = h
        self.n_reads = len(seqs)
        # output buffers of outstanding tickets: the library writes them when a
        # batch completes, so they are kept alive until wait() consumes the
        # ticket or close() has drained every batch
        self._pending = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.xdrop_batch_destroy(self.h)
            self.h = None
            self._pending.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, n: int) -> int:
        """Device bytes a batch of n records takes from the HBM budget."""
        return int(self.lib.xdrop_batch_footprint(self.h, n))

    def tuning(self) -> dict:
        t = Tuning()
        self._check(self.lib.xdrop_get_tuning(self.h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning(**{**self.tuning(), **kw})
        self._check(self.lib.xdrop_set_tuning(self.h, ctypes.byref(t)))

    def autotune(self, recs: np.ndarray, cache_path: str | None = None) -> tuple:
        """Sweep launch parameters on a sample batch; returns (tuning, best device ms)."""
        recs = np.ascontiguousarray(recs, dtype=RECORD_DTYPE)
        best = ctypes.c_double()
        self._check(self.lib.xdrop_autotune(self.h, _ptr(recs), recs.size,
                                            cache_path.encode() if cache_path else None, ctypes.byref(best)))
        return self.tuning(), best.value

    def find_seeds(self, k: int = 31, stride: int = 1, lo: int = 20, hi: int = 30, x: int = 15,
                   weights=(1, -1, -1), max_records: int | None = None):
        """Seed records of the read pairs sharing a reliable k-mer (host array,
        order unspecified) and the call's statistics.  Without max_records the
        output starts at 64 records per read and grows once to the exact count."""
        ma, mi, g = weights
        prm = SeedParams(k, stride, lo, hi, x, ma, mi, g, 0)
        cap = max_records if max_records is not None else max(1024, 64 * self.n_reads)
        for _ in range(2):
            out = np.zeros(cap, RECORD_DTYPE)
            found = ctypes.c_size_t()
            st = SeedStats()
            rc = self.lib.xdrop_find_seeds(self.h, ctypes.byref(prm), _ptr(out) if cap else None, cap, 0,
                                           ctypes.byref(found), ctypes.byref(st))
            if rc == XDROP_E_NOMEM and max_records is None and found.value > cap:
                cap = found.value
                continue
            self._check(rc)
            return out[:found.value], st.as_dict()
        self._check(rc)

    def find_seeds_device(self, d_out, max_records: int, k: int = 31, stride: int = 1, lo: int = 20, hi: int = 30,
                          x: int = 15, weights=(1, -1, -1)):
        """Seed records written straight into device memory (d_out: a torch
        tensor or a device pointer with room for max_records 32-byte records);
        returns (records found, statistics).  Records beyond max_records are
        not written and the call raises XDROP_E_NOMEM."""
        ma, mi, g = weights
        prm = SeedParams(k, stride, lo, hi, x, ma, mi, g, 0)
        ptr = d_out.data_ptr() if hasattr(d_out, "data_ptr") else d_out
        found = ctypes.c_size_t()
        st = SeedStats()
        self._check(self.lib.xdrop_find_seeds(self.h, ctypes.byref(prm), ptr, max_records, 1,
                                              ctypes.byref(found), ctypes.byref(st)))
        return found.value, st.as_dict()

    def error(self) -> str:
        return self.lib.xdrop_last_error(self.h).decode()

    def _check(self, st):
        if st != XDROP_OK:
            raise XdropError(st, self.error() or self.lib.xdrop_status_string(st).decode())

    # -- host path ---------------------------------------------------------
    def submit(self, recs: np.ndarray, out: np.ndarray | None = None, cells: np.ndarray | None = None,
               count_cells: bool = False, admit_timeout_us: int = -1):
        recs = np.ascontiguousarray(recs, dtype=RECORD_DTYPE)
        n = recs.size
        if out is None:
            out = np.zeros(n, RESULT_DTYPE)
        if cells is None and count_cells:
            cells = np.zeros(n, np.uint64)
        t = ctypes.c_uint64()
        st = self.lib.xdrop_batch_submit(self.h, _ptr(recs) if n else None, n, _ptr(out) if n else None,
                                         _ptr(cells) if (cells is not None and n) else None,
                                         admit_timeout_us, ctypes.byref(t))
        self._check(st)
        self._pending[t.value] = (out, cells)
        return t.value, out, cells

    def wait(self, ticket: int, timeout_us: int = -1) -> dict:
        s = Stats()
        st = self.lib.xdrop_batch_wait(self.h, ticket, timeout_us, ctypes.byref(s))
        if st != XDROP_E_TIMEOUT:   # the ticket is consumed (done or failed)
            self._pending.pop(ticket, None)
        self._check(st)
        return s.as_dict()

    def run(self, recs: np.ndarray, count_cells: bool = False):
        """Submit one host batch and wait: (results, cells or None, stats)."""
        t, out, cells = self.submit(recs, count_cells=count_cells)
        stats = self.wait(t)
        return out, cells, stats

    # -- device path (torch tensors or raw device pointers) ----------------
    def submit_device(self, d_recs, n: int, d_out, d_cells=None, stream=None) -> int:
        t = ctypes.c_uint64()
        sp = None if stream is None else int(getattr(stream, "cuda_stream", stream))
        st = self.lib.xdrop_batch_submit_device(self.h, _ptr(d_recs), n, _ptr(d_out),
                                                _ptr(d_cells) if d_cells is not None else None, sp,
                                                ctypes.byref(t))
        self._check(st)
        self._pending[t.value] = (d_recs, d_out, d_cells)
        return t.value

    def run_noalloc(self, d_recs, n: int, d_out, d_cells=None, d_invalid=None, stream=None) -> None:
        """Enqueue one device batch on `stream` through the entry point that
        allocates nothing (xdrop_batch_run_noalloc); results are ready when the
        stream reaches the work.  Buffers: torch tensors or device pointers."""
        sp = None if stream is None else int(getattr(stream, "cuda_stream", stream))
        self._check(self.lib.xdrop_batch_run_noalloc(self.h, _ptr(d_recs), n, _ptr(d_out),
                                                     _ptr(d_cells) if d_cells is not None else None,
                                                     _ptr(d_invalid) if d_invalid is not None else None, sp))


def status_string(st: int) -> str:
    return load_library().xdrop_status_string(st).decode()
