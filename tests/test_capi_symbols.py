"""The C-ABI library loads and exports every entry point that include/xdrop.h
declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import numpy as np

from paper_2309_07270_amd import workload as W
from paper_2309_07270_amd import xdrop as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "xdrop.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(xdrop_\w+)\s*\(", text, re.M)))


def test_header_declares_the_batch_api():
    names = declared_functions()
    for f in ("xdrop_batch_create", "xdrop_batch_submit", "xdrop_batch_submit_device", "xdrop_batch_wait",
              "xdrop_batch_destroy"):
        assert f in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(X.LIB_PATH), "run __graft_entry__.build() first"
    lib = ctypes.CDLL(X.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", X.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (xdrop_\w+)", out))
    assert set(declared_functions()) <= exported


def test_struct_layouts_match_header():
    assert W.RECORD_DTYPE.itemsize == 32 and W.RESULT_DTYPE.itemsize == 32
    assert ctypes.sizeof(X.Stats) == 8 + 8 + 3 * 8 + 4 * 8 * X.NUM_STAGES
    # field offsets of xdrop_record as declared
    offs = {n: W.RECORD_DTYPE.fields[n][1] for n in W.RECORD_DTYPE.names}
    assert offs == {"read_a": 0, "read_b": 4, "pos_a": 8, "pos_b": 12, "k": 16, "strand": 18, "pad": 19,
                    "x": 20, "match": 24, "mismatch": 26, "gap": 28, "pad2": 30}


def test_status_strings_and_null_handles():
    lib = X.load_library()
    assert lib.xdrop_status_string(0) == b"ok"
    assert lib.xdrop_status_string(-5).startswith(b"admission")
    assert lib.xdrop_batch_destroy(None) == 0
    assert lib.xdrop_batch_create(None, None) == X.XDROP_E_INVALID
    t = ctypes.c_uint64()
    assert lib.xdrop_batch_submit(None, None, 0, None, None, 0, ctypes.byref(t)) == X.XDROP_E_INVALID
    assert lib.xdrop_batch_wait(None, 1, 0, None) == X.XDROP_E_INVALID


def test_create_rejects_bad_reads_before_touching_the_device():
    lib = X.load_library()
    for reads in ([b"ACGN"], [b""], [b"ACGT", b"AC-T"]):
        arr = (ctypes.c_char_p * len(reads))(*reads)
        lens = (ctypes.c_uint32 * len(reads))(*[len(r) for r in reads])
        cfg = X.Config(arr, lens, len(reads), 0, 0, 0, 0, None, 0)
        h = ctypes.c_void_p()
        assert lib.xdrop_batch_create(ctypes.byref(cfg), ctypes.byref(h)) == X.XDROP_E_INVALID
        assert not h.value


def test_binding_keeps_output_buffers_alive_until_wait():
    """The library writes results when a batch completes: the binding must hold
    the output arrays of an outstanding ticket even if the caller drops them."""
    import inspect
    src = inspect.getsource(X.Context)
    assert "_pending[t.value]" in src and "_pending.pop(ticket" in src
