"""The entry point that allocates nothing (xdrop_batch_run_noalloc), called
through the C ABI, against the existing device entry point
(xdrop_batch_submit_device) and the CPU oracle: every result field and every
per-record cell count equal (integers: the bar is equality).

Two no-alloc calls run back to back on one stream, the second with fewer
records, so the second runs on what the first left in the library's
per-GPU array.  The records include wide bands that climb through every
window class into the unbounded kernel, so the carry pool and the unbounded
kernel's scratch, both carved from that array, are used.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2309_07270_amd import workload as W

pytestmark = pytest.mark.gpu

FIELDS = (("score", "score"), ("left_score", "left"), ("right_score", "right"), ("seed_score", "seed"),
          ("a_begin", "a_begin"), ("a_end", "a_end"), ("b_begin", "b_begin"), ("b_end", "b_end"))


def note(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def xd():
    import torch
    assert torch.cuda.is_available()
    from paper_2309_07270_amd import xdrop
    xdrop.load_library()
    return xdrop


def assert_oracle(res, cells, ref):
    for fg, fr in FIELDS:
        g = res[fg].astype(np.int64)
        bad = np.flatnonzero(g != ref[fr].astype(np.int64))
        assert bad.size == 0, f"{fg}: record {int(bad[0])} gpu {int(g[bad[0]])} oracle {int(ref[fr][bad[0]])}"
    want = (ref["cells_left"] + ref["cells_right"]).astype(np.uint64)
    bad = np.flatnonzero(cells.astype(np.uint64) != want)
    assert bad.size == 0, f"cells: record {int(bad[0])}"


def test_noalloc_equals_submit_device_two_calls(xd):
    import torch
    rng = np.random.Generator(np.random.PCG64(71))
    store = W.random_store(rng, 40, 800, 3000, related=0.7)
    big = W.random_records(rng, store, 1500, x_choices=(20, 100, 500, 1500, 1 << 30))
    small = W.random_records(rng, store, 300, x_choices=(15, 50, 3000))
    refs = [oracle.batch(store.codes, store.off, store.length, r)[0] for r in (big, small)]
    stream = torch.cuda.current_stream()
    with xd.Context(store) as ctx:
        d_in, want = [], []
        for recs in (big, small):
            n = len(recs)
            note(f"submit_device: {n} records")
            d_recs = torch.from_numpy(recs.view(np.uint8).copy()).cuda()
            d_out = torch.zeros(n * 32, dtype=torch.uint8, device="cuda")
            d_cells = torch.zeros(n, dtype=torch.int64, device="cuda")
            ctx.wait(ctx.submit_device(d_recs, n, d_out, d_cells, stream=stream))
            torch.cuda.synchronize()
            d_in.append(d_recs)
            want.append((d_out.cpu().numpy().view(W.RESULT_DTYPE).copy(), d_cells.cpu().numpy().astype(np.uint64)))
        # the two no-alloc calls, back to back on the stream; outputs start
        # filled with garbage so that an unwritten row shows
        outs = []
        for recs, d_recs in zip((big, small), d_in):
            n = len(recs)
            note(f"run_noalloc: {n} records")
            d_out = torch.full((n * 32,), 0xA5, dtype=torch.uint8, device="cuda")
            d_cells = torch.full((n,), -7, dtype=torch.int64, device="cuda")
            d_inv = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
            ctx.run_noalloc(d_recs, n, d_out, d_cells, d_inv, stream=stream)
            outs.append((d_out, d_cells, d_inv))
        torch.cuda.synchronize()
        for (d_out, d_cells, d_inv), (res_w, cells_w), ref in zip(outs, want, refs):
            res = d_out.cpu().numpy().view(W.RESULT_DTYPE).copy()
            cells = d_cells.cpu().numpy().astype(np.uint64)
            assert int(d_inv.cpu().item()) == 0
            assert np.array_equal(res, res_w), "results differ from xdrop_batch_submit_device"
            assert np.array_equal(cells, cells_w), "cell counts differ from xdrop_batch_submit_device"
            assert_oracle(res, cells, ref)


def test_noalloc_invalid_records_and_limits(xd):
    import torch
    rng = np.random.Generator(np.random.PCG64(72))
    store = W.random_store(rng, 20, 300, 1200)
    recs = W.random_records(rng, store, 200, x_choices=(20, 50))
    recs[17]["read_a"] = store.n + 5          # read id out of range
    recs[90]["k"] = 0                          # empty seed
    ok = np.ones(len(recs), bool)
    ok[[17, 90]] = False
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs[ok])
    stream = torch.cuda.current_stream()
    with xd.Context(store) as ctx:
        n = len(recs)
        note(f"run_noalloc with 2 invalid records of {n}")
        d_recs = torch.from_numpy(recs.view(np.uint8).copy()).cuda()
        d_out = torch.full((n * 32,), 0x5A, dtype=torch.uint8, device="cuda")
        d_cells = torch.zeros(n, dtype=torch.int64, device="cuda")
        d_inv = torch.zeros(1, dtype=torch.int32, device="cuda")
        ctx.run_noalloc(d_recs, n, d_out, d_cells, d_inv, stream=stream)
        torch.cuda.synchronize()
        res = d_out.cpu().numpy().view(W.RESULT_DTYPE).copy()
        cells = d_cells.cpu().numpy().astype(np.uint64)
        assert int(d_inv.cpu().item()) == 2
        assert not res[~ok].view(np.uint8).any() and not cells[~ok].any()
        assert_oracle(res[ok], cells[ok], ref)
        # an empty batch: nothing computed, the invalid count is 0
        ctx.run_noalloc(d_recs, 0, d_out, None, d_inv, stream=stream)
        torch.cuda.synchronize()
        assert int(d_inv.cpu().item()) == 0
        # beyond the record limit: refused on the host before any launch
        with pytest.raises(xd.XdropError) as e:
            ctx.run_noalloc(d_recs, xd.NOALLOC_MAX_RECORDS + 1, d_out, None, None, stream=stream)
        assert e.value.status == xd.XDROP_E_INVALID and "limit" in ctx.error()
