"""GPU parity of the narrow class (two extensions per wavefront, one per
half of the lanes) against the CPU oracle, bit-exact in every result field
and in per-record cell counts.

The narrow class takes records with x <= narrow_x (20 by default) and weights
match 1, gap -1, mismatch 0 / -1 / -2 in the persistent form, in batches of at
least narrow_min_records records (the tests set it to 0).  Cases cover:
tiny reads and seeds at read ends (empty extensions); bands that need the
64-slot window and bands wider than it (the task restarts in the adaptive
class); batches with an odd number of extensions and batches of one record
(one half of a wavefront empty); mixes with records of other classes; and
the narrow class switched off, which must not change any result.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2309_07270_amd import workload as W

pytestmark = pytest.mark.gpu

FIELDS = (("score", "score"), ("left_score", "left"), ("right_score", "right"), ("seed_score", "seed"),
          ("a_begin", "a_begin"), ("a_end", "a_end"), ("b_begin", "b_begin"), ("b_end", "b_end"))
NARROW_WEIGHTS = ((1, -1, -1), (1, 0, -1), (1, -2, -1))


def note(msg):
    print(f"[gpu-narrow] {msg}", flush=True)
    sys.stdout.flush()


def assert_same(res, cells, ref):
    for fg, fr in FIELDS:
        g = res[fg].astype(np.int64)
        r = ref[fr].astype(np.int64)
        bad = np.flatnonzero(g != r)
        assert bad.size == 0, f"{fg}: {bad.size} records differ, first {int(bad[0])}: gpu {int(g[bad[0]])} " \
                              f"oracle {int(r[bad[0]])}"
    want = (ref["cells_left"] + ref["cells_right"]).astype(np.uint64)
    bad = np.flatnonzero(cells.astype(np.uint64) != want)
    assert bad.size == 0, f"cells: {bad.size} records differ, first {int(bad[0])}"


@pytest.fixture(scope="module")
def xd():
    import torch
    assert torch.cuda.is_available()
    from paper_2309_07270_amd import xdrop
    xdrop.load_library()
    return xdrop


def narrow_ctx(xd, store, **kw):
    """A context whose narrow class takes batches of any size."""
    ctx = xd.Context(store, **kw)
    ctx.set_tuning(narrow_min_records=0)
    return ctx


def stage(xd, st, name):
    return int(st["stage_tasks"][xd.STAGE_NAMES.index(name)])


def widest_bands(store, recs):
    """Widest live range of every extension (left, right) from the oracle."""
    out = []
    for R in recs:
        a = store.read(int(R["read_a"]))
        b = store.read(int(R["read_b"]))
        k = int(R["k"])
        pb = int(R["pos_b"])
        if R["strand"]:
            b = W.revcomp_codes(b)
            pb = b.size - pb - k
        pa = int(R["pos_a"])
        w = (int(R["match"]), int(R["mismatch"]), int(R["gap"]), int(R["x"]))
        out.append(oracle.extend_band(a[:pa][::-1].copy(), b[:pb][::-1].copy(), *w)[1])
        out.append(oracle.extend_band(a[pa + k:].copy(), b[pb + k:].copy(), *w)[1])
    return np.array(out)


@pytest.mark.parametrize("seed,lo,hi,related,n", [
    (201, 1, 40, 0.5, 3000),      # tiny reads: many empty extensions, seeds at read ends
    (202, 20, 400, 0.5, 3000),
    (203, 300, 1500, 0.7, 2000),
    (204, 800, 3000, 0.0, 600),   # unrelated reads: bands outgrow 64 slots, tasks go to the adaptive class
])
def test_narrow_random_bit_exact(xd, seed, lo, hi, related, n):
    rng = np.random.Generator(np.random.PCG64(seed))
    store = W.random_store(rng, 60, lo, hi, related=related)
    recs = W.random_records(rng, store, n, x_choices=tuple(range(0, 21)), weights=NARROW_WEIGHTS)
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    note(f"narrow random records seed={seed} len=[{lo},{hi}] related={related}")
    for mode in (0, 1):
        with narrow_ctx(xd, store, mode=mode) as ctx:
            res, cells, st = ctx.run(recs, count_cells=True)
        assert_same(res, cells, ref)
        if mode == 0:
            assert stage(xd, st, "narrow") > 0
            if related == 0.0:
                assert stage(xd, st, "adaptive") > 0   # bands wider than 64 slots restarted there


def test_narrow_c1_shaped_x20(xd):
    # 15 %-error reads at X = 20: the widest band of an extension is 29
    # cells at the median and 36 at the 99th percentile, so most extensions
    # need the 64-slot window at some point and none leaves the class
    wl = W.make_workload("c1", pairs=3000, x_choices=(20,), genome=1_000_000)
    ref, _ = oracle.batch(wl.store.codes, wl.store.off, wl.store.length, wl.records)
    widths = widest_bands(wl.store, wl.records[:600])
    assert np.mean((widths > 30) & (widths <= 56)) > 0.1, np.percentile(widths, [50, 90, 99])
    note("narrow class on c1-shaped records at X = 20")
    with narrow_ctx(xd, wl.store) as ctx:
        res, cells, st = ctx.run(wl.records, count_cells=True)
    assert_same(res, cells, ref)
    assert stage(xd, st, "narrow") == 2 * len(wl.records)


def test_narrow_mixed_with_other_classes(xd):
    # the 1M-pair workload's mix (X in {20, 50, 100}) on a smaller genome:
    # one third of the records run two per wavefront, the rest in the
    # adaptive windows, in one batch
    wl = W.make_workload("c2", pairs=4000, genome=1_000_000)
    ref, _ = oracle.batch(wl.store.codes, wl.store.off, wl.store.length, wl.records)
    note("c2-shaped mix: narrow and adaptive classes in one batch")
    with narrow_ctx(xd, wl.store) as ctx:
        res, cells, st = ctx.run(wl.records, count_cells=True)
    assert_same(res, cells, ref)
    assert stage(xd, st, "narrow") > 0 and stage(xd, st, "adaptive") > 0
    sc = np.array(st["stage_cells"], np.uint64)
    assert int(sc.sum()) == int(cells.sum())


def test_narrow_odd_and_tiny_batches(xd):
    # 1, 2, 3 and 7 records (2 to 14 extensions): wavefronts with one half empty
    rng = np.random.Generator(np.random.PCG64(205))
    store = W.random_store(rng, 20, 200, 900, related=0.8)
    recs = W.random_records(rng, store, 13, x_choices=(3, 10, 20), weights=NARROW_WEIGHTS)
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    note("narrow class: batches of 1, 2, 3 and 7 records")
    with narrow_ctx(xd, store) as ctx:
        off = 0
        for n in (1, 2, 3, 7):
            res, cells, st = ctx.run(recs[off:off + n], count_cells=True)
            assert_same(res, cells, ref[off:off + n])
            assert stage(xd, st, "narrow") + stage(xd, st, "adaptive") == 2 * n
            off += n


def test_narrow_off_gives_the_same_results(xd):
    wl = W.make_workload("c1", pairs=2000, x_choices=(5, 15, 20), genome=1_000_000)
    note("narrow class on and off: identical results and cell counts")
    with narrow_ctx(xd, wl.store) as ctx:
        res_on, cells_on, st_on = ctx.run(wl.records, count_cells=True)
        ctx.set_tuning(narrow_x=-1)
        assert ctx.tuning()["narrow_x"] == -1
        res_off, cells_off, st_off = ctx.run(wl.records, count_cells=True)
        ctx.set_tuning(narrow_x=1000)          # clamped to the class limit
        assert ctx.tuning()["narrow_x"] == 64
    assert np.array_equal(res_on, res_off) and np.array_equal(cells_on, cells_off)
    assert stage(xd, st_on, "narrow") > 0 and stage(xd, st_off, "narrow") == 0


def test_narrow_only_in_large_batches(xd):
    # a batch smaller than narrow_min_records runs every extension one per
    # wavefront; from that size on the narrow class takes its records
    wl = W.make_workload("c1", pairs=400, x_choices=(10, 20), genome=1_000_000)
    ref, _ = oracle.batch(wl.store.codes, wl.store.off, wl.store.length, wl.records)
    note("narrow class by batch size (narrow_min_records)")
    with xd.Context(wl.store) as ctx:
        assert ctx.tuning()["narrow_min_records"] == 100000
        res0, cells0, st0 = ctx.run(wl.records, count_cells=True)
        ctx.set_tuning(narrow_min_records=400)
        res1, cells1, st1 = ctx.run(wl.records, count_cells=True)
        res2, cells2, st2 = ctx.run(wl.records[:399], count_cells=True)
    for res, cells, r in ((res0, cells0, ref), (res1, cells1, ref), (res2, cells2, ref[:399])):
        assert_same(res, cells, r)
    assert stage(xd, st0, "narrow") == 0 and stage(xd, st0, "adaptive") == 800
    assert stage(xd, st1, "narrow") > 0
    assert stage(xd, st2, "narrow") == 0 and stage(xd, st2, "adaptive") == 798
