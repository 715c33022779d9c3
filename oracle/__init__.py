"""CPU oracle for batched X-drop seed-and-extend (ctypes binding).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check in
``__graft_entry__.py`` and by the ``cpu_baseline`` leg of ``bench.py``.
The product library never imports, links or runs anything in this folder,
and this folder imports nothing from the product package.

The arithmetic lives in ``xdrop_oracle.c`` (a plain sequential
transcription of the X-drop reading stated in its header; paper: "Related
works", BELLA/LOGAN paragraphs, and "Results", where the aligner is
described as Needleman-Wunsch / Smith-Waterman with an X-drop).  This module
only marshals arguments.

Bases are handled as codes A=0, C=1, G=2, T=3.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xdrop_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

INF_X = 1 << 30  # the largest drop accepted; behaves as "no drop" for reads <= 100 kb


class Ext(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int64), ("i", ctypes.c_int64), ("j", ctypes.c_int64),
                ("cells", ctypes.c_uint64)]

    def tup(self):
        return (self.score, self.i, self.j, self.cells)


class Rec(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int64), ("left", ctypes.c_int64), ("right", ctypes.c_int64),
                ("seed", ctypes.c_int64), ("a_begin", ctypes.c_int64), ("a_end", ctypes.c_int64),
                ("b_begin", ctypes.c_int64), ("b_end", ctypes.c_int64),
                ("cells_left", ctypes.c_uint64), ("cells_right", ctypes.c_uint64)]


REC_DTYPE = np.dtype([("score", "<i8"), ("left", "<i8"), ("right", "<i8"), ("seed", "<i8"),
                      ("a_begin", "<i8"), ("a_end", "<i8"), ("b_begin", "<i8"), ("b_end", "<i8"),
                      ("cells_left", "<u8"), ("cells_right", "<u8")])
assert REC_DTYPE.itemsize == ctypes.sizeof(Rec)


def build(out_path: str = _LIB_PATH, mutation: int = 0) -> str:
    """Compile the oracle with gcc.  ``mutation`` > 0 plants a known mistake
    (used only by the tests that show the pins catch mistakes)."""
    # built beside the target and renamed over it, so that a process that has
    # the old library loaded keeps a valid mapping
    tmp = f"{out_path}.tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-shared", "-fPIC", "-pthread", f"-DOX_MUTATION={int(mutation)}",
           _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out_path)
    return out_path


def _bind(lib):
    P = ctypes.POINTER
    u8p, i64p = P(ctypes.c_uint8), P(ctypes.c_int64)
    i64 = ctypes.c_int64
    for name in ("ox_extend", "ox_extend_dense"):
        f = getattr(lib, name)
        f.argtypes = [u8p, i64, u8p, i64, i64, i64, i64, i64, P(Ext)]
        f.restype = ctypes.c_int
    lib.ox_extend_band.argtypes = [u8p, i64, u8p, i64, i64, i64, i64, i64, P(Ext), i64p]
    lib.ox_extend_band.restype = ctypes.c_int
    lib.ox_nw_best.argtypes = [u8p, i64, u8p, i64, i64, i64, i64, P(Ext)]
    lib.ox_nw_best.restype = ctypes.c_int
    lib.ox_record.argtypes = [u8p, i64, u8p, i64, i64, i64, i64, ctypes.c_int, i64, i64, i64, i64,
                              P(Rec)]
    lib.ox_record.restype = ctypes.c_int
    lib.ox_batch.argtypes = [u8p, i64p, i64p] + [i64p] * 10 + [i64, ctypes.c_int, ctypes.c_void_p,
                                                                 P(ctypes.c_int)]
    lib.ox_batch.restype = ctypes.c_int
    lib.ox_mutation.restype = ctypes.c_int
    return lib


def load(path: str | None = None):
    """Load the oracle library (building it with gcc when it is absent)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build()
            _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


_CODE = np.full(256, 255, dtype=np.uint8)
for _c, _v in zip(b"ACGTacgt", [0, 1, 2, 3, 0, 1, 2, 3]):
    _CODE[_c] = _v


def codes(seq) -> np.ndarray:
    """ASCII string/bytes (ACGT, any case) or a code array -> uint8 codes 0..3."""
    if isinstance(seq, np.ndarray):
        arr = np.ascontiguousarray(seq, dtype=np.uint8)
    else:
        if isinstance(seq, str):
            seq = seq.encode()
        arr = _CODE[np.frombuffer(seq, dtype=np.uint8)] if len(seq) else np.zeros(0, np.uint8)
    if arr.size and arr.max() > 3:
        raise ValueError("oracle: non-ACGT base")
    return np.ascontiguousarray(arr)


def _u8(arr):
    if arr.size == 0:
        arr = np.zeros(1, np.uint8)
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), arr


def extend(a, b, ma=1, mi=-1, g=-1, X=50, dense=False, lib=None):
    """One X-drop extension of a against b from cell (0,0): (T, i*, j*, cells)."""
    lib = lib or load()
    a, b = codes(a), codes(b)
    pa, ka = _u8(a)
    pb, kb = _u8(b)
    out = Ext()
    f = lib.ox_extend_dense if dense else lib.ox_extend
    rc = f(pa, a.size, pb, b.size, ma, mi, g, X, ctypes.byref(out))
    if rc != 0:
        raise MemoryError("oracle extend failed")
    return out.tup()


def extend_band(a, b, ma=1, mi=-1, g=-1, X=50, lib=None):
    """extend() plus the widest live range of any anti-diagonal:
    ((T, i*, j*, cells), max_width)."""
    lib = lib or load()
    a, b = codes(a), codes(b)
    pa, ka = _u8(a)
    pb, kb = _u8(b)
    out = Ext()
    w = ctypes.c_int64()
    if lib.ox_extend_band(pa, a.size, pb, b.size, ma, mi, g, X, ctypes.byref(out), ctypes.byref(w)) != 0:
        raise MemoryError("oracle extend failed")
    return out.tup(), int(w.value)


def nw_best(a, b, ma=1, mi=-1, g=-1, lib=None):
    """Full Needleman-Wunsch prefix table maximum: (H*, i*, j*, (m+1)(n+1)-1)."""
    lib = lib or load()
    a, b = codes(a), codes(b)
    pa, ka = _u8(a)
    pb, kb = _u8(b)
    out = Ext()
    if lib.ox_nw_best(pa, a.size, pb, b.size, ma, mi, g, ctypes.byref(out)) != 0:
        raise MemoryError("oracle nw failed")
    return out.tup()


def record(A, B, pos_a, pos_b, k, strand, X, ma=1, mi=-1, g=-1, lib=None) -> dict:
    """One seed-and-extend record; B span reported in the oriented frame B'."""
    lib = lib or load()
    A, B = codes(A), codes(B)
    pA, kA = _u8(A)
    pB, kB = _u8(B)
    out = Rec()
    rc = lib.ox_record(pA, A.size, pB, B.size, pos_a, pos_b, k, int(strand), X, ma, mi, g,
                       ctypes.byref(out))
    if rc == -2:
        raise ValueError("oracle: seed outside a read")
    if rc != 0:
        raise MemoryError("oracle record failed")
    return {name: getattr(out, name) for name, _ in Rec._fields_}


def default_threads() -> int:
    """Host threads for batch(): the CPUs this process may run on, at most
    16 (the host share of one GPU on a shared multi-GPU node)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def batch(read_codes: np.ndarray, read_off: np.ndarray, read_len: np.ndarray, recs,
          nthreads: int | None = None, lib=None):
    """Run ``ox_record`` over a record table on a pool of threads.

    ``read_codes`` is one uint8 code buffer holding every read, ``read_off`` /
    ``read_len`` index it.  ``recs`` is any mapping/structured array with the
    fields read_a, read_b, pos_a, pos_b, k, strand, x, match, mismatch, gap.
    Returns (structured array of REC_DTYPE, threads used).
    """
    lib = lib or load()
    n = len(recs["read_a"])
    if nthreads is None:
        nthreads = default_threads()
    cols = [np.ascontiguousarray(recs[f], dtype=np.int64) for f in
            ("read_a", "read_b", "pos_a", "pos_b", "k", "strand", "x", "match", "mismatch", "gap")]
    codes_arr = np.ascontiguousarray(read_codes, dtype=np.uint8)
    roff = np.ascontiguousarray(read_off, dtype=np.int64)
    rlen = np.ascontiguousarray(read_len, dtype=np.int64)
    out = np.zeros(n, dtype=REC_DTYPE)
    status = np.zeros(max(n, 1), dtype=np.int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    used = lib.ox_batch(codes_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                        roff.ctypes.data_as(i64p), rlen.ctypes.data_as(i64p),
                        *[c.ctypes.data_as(i64p) for c in cols], n, int(nthreads),
                        out.ctypes.data_as(ctypes.c_void_p),
                        status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if n and np.any(status[:n] != 0):
        bad = int(np.flatnonzero(status[:n])[0])
        raise ValueError(f"oracle batch: record {bad} failed with status {int(status[bad])}")
    return out, used
