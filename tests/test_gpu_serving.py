"""Serving loop on the GPU: many producer threads submit batches to one
context; admitted batches run concurrently on their own streams (continuous
batching).  Each batch's results must equal the CPU oracle's, field by field
and in cell counts, both alone and in the mix (integer path: tolerance 0),
and admission must apply back-pressure when the HBM budget is exhausted.
"""
import sys
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2309_07270_amd import workload as W

pytestmark = pytest.mark.gpu

FIELDS = (("score", "score"), ("left_score", "left"), ("right_score", "right"), ("seed_score", "seed"),
          ("a_begin", "a_begin"), ("a_end", "a_end"), ("b_begin", "b_begin"), ("b_end", "b_end"))


def note(msg):
    print(f"[gpu-serving] {msg}", flush=True)
    sys.stdout.flush()


def assert_oracle(res, cells, ref, what):
    """res / cells of one batch against the oracle rows of the same records."""
    for fg, fr in FIELDS:
        g = res[fg].astype(np.int64)
        r = ref[fr].astype(np.int64)
        bad = np.flatnonzero(g != r)
        assert bad.size == 0, f"{what}: {fg} differs at record {int(bad[0])}: gpu {int(g[bad[0]])} oracle {int(r[bad[0]])}"
    if cells is not None:
        want = (ref["cells_left"] + ref["cells_right"]).astype(np.uint64)
        bad = np.flatnonzero(cells.astype(np.uint64) != want)
        assert bad.size == 0, f"{what}: cells differ at record {int(bad[0])}"


def oracle_rows(wl, idx):
    """Oracle results of records wl.records[idx], computed once per distinct record."""
    uniq, inv = np.unique(idx, return_inverse=True)
    ref, _ = oracle.batch(wl.store.codes, wl.store.off, wl.store.length, wl.records[uniq])
    return ref[inv]


@pytest.fixture(scope="module")
def xd():
    import torch
    assert torch.cuda.is_available()
    from paper_2309_07270_amd import xdrop
    xdrop.load_library()
    return xdrop


@pytest.fixture(scope="module")
def wl():
    # c2-shaped reads (100x, mean 10 kb) on a smaller genome; X in {20,50,100}
    return W.make_workload("c2", pairs=60000, genome=1_000_000)


@pytest.fixture(scope="module")
def pool_ref(wl):
    # the oracle over the whole 60,000-record pool (every batch below is a slice of it)
    note("oracle over the 60,000-record pool")
    ref, _ = oracle.batch(wl.store.codes, wl.store.off, wl.store.length, wl.records)
    return ref


def test_alone_equals_mixed(xd, wl, pool_ref):
    rng = np.random.default_rng(0)
    n_prod, per = 25, 3
    sizes = rng.integers(1000, 4000, size=n_prod * per)
    starts = rng.integers(0, len(wl.records) - 4000, size=n_prod * per)
    batches = [wl.records[s:s + z] for s, z in zip(starts, sizes)]
    note(f"alone: {len(batches)} batches one at a time")
    alone = []
    with xd.Context(wl.store, max_inflight=1) as ctx:
        for b in batches:
            res, cells, _ = ctx.run(b, count_cells=True)
            alone.append((res, cells))
    note("mixed: 25 producer threads, 6 slots in flight")
    mixed = [None] * len(batches)
    errors = []
    with xd.Context(wl.store, max_inflight=6) as ctx:
        def producer(p):
            try:
                for k in range(per):
                    i = p * per + k
                    t, out, cells = ctx.submit(batches[i], count_cells=True)
                    ctx.wait(t)
                    mixed[i] = (out, cells)
            except Exception as e:  # pragma: no cover - reported below
                errors.append(e)
        th = [threading.Thread(target=producer, args=(p,)) for p in range(n_prod)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=120)
    assert not errors, errors
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert m is not None, f"batch {i} missing"
        ref = pool_ref[starts[i]:starts[i] + sizes[i]]
        assert_oracle(a[0], a[1], ref, f"batch {i} alone")
        assert_oracle(m[0], m[1], ref, f"batch {i} mixed")


def test_wide_bands_alone_equals_mixed(xd):
    # c4 stress mix (half unrelated pairs, X = 100, reads up to 100 kb): the
    # unrelated extensions climb through the wide classes and hand their
    # state over in each slot's own carry pool while other batches run
    wl4 = W.make_workload("c4", pairs=3000, genome=1_000_000, coverage=30)
    rng = np.random.default_rng(4)
    n_prod, per = 6, 2
    sizes = rng.integers(150, 300, size=n_prod * per)
    starts = rng.integers(0, len(wl4.records) - 300, size=n_prod * per)
    batches = [wl4.records[s:s + z] for s, z in zip(starts, sizes)]
    note(f"wide bands alone: {len(batches)} batches of the c4 mix one at a time")
    alone, wide_tasks = [], 0
    with xd.Context(wl4.store, max_inflight=1) as ctx:
        for b in batches:
            res, cells, st = ctx.run(b, count_cells=True)
            alone.append((res, cells))
            wide_tasks += int(st["stage_tasks"][xd.STAGE_NAMES.index("wide2048")]) + \
                int(st["stage_tasks"][xd.STAGE_NAMES.index("generic")])
    assert wide_tasks > 0   # extensions finished after a hand-over
    note("wide bands mixed: 6 producer threads, 4 slots in flight")
    mixed = [None] * len(batches)
    errors = []
    with xd.Context(wl4.store, max_inflight=4) as ctx:
        def producer(p):
            try:
                for k in range(per):
                    i = p * per + k
                    t, out, cells = ctx.submit(batches[i], count_cells=True)
                    ctx.wait(t)
                    mixed[i] = (out, cells)
            except Exception as e:  # pragma: no cover - reported below
                errors.append(e)
        th = [threading.Thread(target=producer, args=(p,)) for p in range(n_prod)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=120)
    assert not errors, errors
    note("oracle of the wide-band batches")
    idx = np.concatenate([np.arange(s, s + z) for s, z in zip(starts, sizes)])
    refs = oracle_rows(wl4, idx)
    off = 0
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert m is not None, f"batch {i} missing"
        ref = refs[off:off + sizes[i]]
        off += sizes[i]
        assert_oracle(a[0], a[1], ref, f"wide batch {i} alone")
        assert_oracle(m[0], m[1], ref, f"wide batch {i} mixed")


def test_admission_backpressure_and_timeouts(xd, wl, pool_ref):
    recs = wl.records[:20000]
    big = np.tile(wl.records, 20)[:1 << 20]
    with xd.Context(wl.store) as probe:
        one = probe.footprint(len(recs))
        assert probe.footprint(len(big)) > 1.5 * one
    note(f"HBM budget of 1.5 slots ({one * 1.5 / 2**20:.0f} MiB): one 20k batch fits, a second must wait")
    with xd.Context(wl.store, max_inflight=4, hbm_budget_bytes=int(one * 1.5)) as ctx:
        # the first batch (30k records, same slot size) keeps the GPU busy for tens of ms
        t1, out1, _ = ctx.submit(wl.records[:30000])
        with pytest.raises(xd.XdropError) as e:
            ctx.submit(recs, admit_timeout_us=0)
        assert e.value.status == xd.XDROP_E_BUSY
        # a blocking submit is admitted once the first batch completes
        t2, out2, _ = ctx.submit(recs, admit_timeout_us=-1)
        ctx.wait(t1)
        ctx.wait(t2)
        assert_oracle(out1, None, pool_ref[:30000], "first batch")
        assert_oracle(out2, None, pool_ref[:20000], "batch admitted after back-pressure")
        # a batch that can never fit is refused outright
        with pytest.raises(xd.XdropError) as e:
            ctx.submit(big)
        assert e.value.status == xd.XDROP_E_NOMEM
    note("wait(0) polls; unknown tickets are rejected; destroy drains")
    with xd.Context(wl.store) as ctx:
        t, out, _ = ctx.submit(wl.records[:30000])
        try:
            ctx.wait(t, timeout_us=0)
        except xd.XdropError as e:
            assert e.status == xd.XDROP_E_TIMEOUT
            ctx.wait(t)
        with pytest.raises(xd.XdropError) as e:
            ctx.wait(t)
        assert e.value.status == xd.XDROP_E_STATE
        # destroy with an outstanding ticket: drains, then frees
        ctx.submit(wl.records[:30000])
    assert out["score"].min() > 0


def test_overlap_on_device(xd, wl):
    """Batches admitted together overlap on the GPU: four concurrent batches
    finish in less wall time than four back to back."""
    recs = wl.records[:15000]
    with xd.Context(wl.store, max_inflight=4) as ctx:
        for _ in range(2):  # warm-up: four slots with their graphs
            ts = [ctx.submit(recs)[0] for _ in range(4)]
            for t in ts:
                ctx.wait(t)
        t0 = time.perf_counter()
        for _ in range(4):
            ctx.run(recs)
        serial = time.perf_counter() - t0
        t0 = time.perf_counter()
        ts = [ctx.submit(recs)[0] for _ in range(4)]
        for t in ts:
            ctx.wait(t)
        overlapped = time.perf_counter() - t0
    note(f"4 batches: serial {serial * 1e3:.1f} ms, overlapped {overlapped * 1e3:.1f} ms")
    assert overlapped < serial


def test_sub_batch_hand_off_equals_whole(xd, wl, pool_ref):
    """A producer batch handed over as sub-batches (submitted back to back,
    waited together) gives the oracle's results, as the whole batch does."""
    recs = wl.records[5000:17000]
    note("12,000 records whole vs 5 sub-batches of 2,500 (last 2,000)")
    with xd.Context(wl.store, max_inflight=4) as ctx:
        whole, cw, _ = ctx.run(recs, count_cells=True)
        parts = [ctx.submit(recs[o:o + 2500], count_cells=True) for o in range(0, len(recs), 2500)]
        for t, _, _ in parts:
            ctx.wait(t)
    split = np.concatenate([p[1] for p in parts])
    cs = np.concatenate([p[2] for p in parts])
    ref = pool_ref[5000:17000]
    assert_oracle(whole, cw, ref, "whole batch")
    assert_oracle(split, cs, ref, "sub-batches")
