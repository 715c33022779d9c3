"""GPU parity: libxdrop.so (through its C ABI) against the CPU oracle, bit-exact.

Every compared field is an integer, so the bar is equality: scores, the four
span coordinates and the per-record cell counts.
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
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def assert_same(res, cells, ref, idx=None):
    idx = np.arange(len(res)) if idx is None else idx
    for fg, fr in FIELDS:
        g = res[fg].astype(np.int64)
        r = ref[fr].astype(np.int64)
        if not np.array_equal(g, r):
            bad = np.flatnonzero(g != r)
            raise AssertionError(f"{fg}: {bad.size} records differ, first record {int(idx[bad[0]])}: "
                                 f"gpu {int(g[bad[0]])} oracle {int(r[bad[0]])}")
    if cells is not None:
        want = (ref["cells_left"] + ref["cells_right"]).astype(np.uint64)
        if not np.array_equal(cells.astype(np.uint64), want):
            bad = np.flatnonzero(cells.astype(np.uint64) != want)
            raise AssertionError(f"cells: {bad.size} records differ, first {int(idx[bad[0]])}: "
                                 f"gpu {int(cells[bad[0]])} oracle {int(want[bad[0]])}")


@pytest.fixture(scope="module")
def xd():
    import torch
    assert torch.cuda.is_available()
    from paper_2309_07270_amd import xdrop
    xdrop.load_library()
    return xdrop


@pytest.fixture(scope="module")
def c0():
    wl = W.make_workload("c0")
    ref, _ = oracle.batch(wl.store.codes, wl.store.off, wl.store.length, wl.records)
    return wl, ref


@pytest.mark.parametrize("mode", [0, 1])
def test_c0_bit_exact(xd, c0, mode):
    wl, ref = c0
    note(f"c0 1000 records mode={mode}")
    with xd.Context(wl.store, mode=mode) as ctx:
        res, cells, st = ctx.run(wl.records, count_cells=True)
        res2, cells2, _ = ctx.run(wl.records, count_cells=False)
    assert_same(res, cells, ref)
    assert_same(res2, None, ref)
    assert st["cells"] == int(cells.sum())


def small_case(seed, n_reads, lo, hi, n_recs, x_choices):
    rng = np.random.Generator(np.random.PCG64(seed))
    store = W.random_store(rng, n_reads, lo, hi)
    recs = W.random_records(rng, store, n_recs, x_choices=x_choices)
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    return store, recs, ref


@pytest.mark.parametrize("seed,lo,hi,xs,related,n_recs", [
    (11, 1, 40, (0, 1, 2, 3, 5), 0.0, 3000),
    (12, 20, 400, (0, 5, 20, 50), 0.0, 3000),
    (13, 300, 1500, (10, 50, 100), 0.0, 3000),
    # wide bands: about two thirds of these extensions leave the adaptive
    # kernel, hundreds reach the 2048-slot class by hand-over, a few the
    # unbounded kernel
    (102, 800, 3000, (500, 1500, 1 << 30), 0.7, 1500),
    (103, 2000, 3000, (50, 1000, 3000), 0.7, 1500),
])
def test_random_records_bit_exact(xd, seed, lo, hi, xs, related, n_recs):
    rng = np.random.Generator(np.random.PCG64(seed))
    if related:
        store = W.random_store(rng, 40, lo, hi, related=related)
        recs = W.random_records(rng, store, n_recs, x_choices=xs)
        ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    else:
        store, recs, ref = small_case(seed, 60, lo, hi, n_recs, xs)
    note(f"random records seed={seed} len=[{lo},{hi}] X={xs}")
    for mode in (0, 1):
        with xd.Context(store, mode=mode) as ctx:
            res, cells, _ = ctx.run(recs, count_cells=True)
        assert_same(res, cells, ref)


def test_wide_bands_escalate(xd):
    # X = 2^30 never drops a cell: the band grows to the whole table and the
    # task has to climb through every window class into the unbounded kernel.
    rng = np.random.Generator(np.random.PCG64(21))
    store = W.random_store(rng, 12, 200, 2600, related=0.8)
    recs = W.random_records(rng, store, 40, x_choices=(W_INF := 1 << 30, 300, 1000), k_max=5)
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    note("wide bands: X up to 2^30, reads up to 2.6 kb")
    with xd.Context(store) as ctx:
        res, cells, _ = ctx.run(recs, count_cells=True)
    assert_same(res, cells, ref)


def test_unbounded_band_wider_than_lds_ring(xd):
    # X = 2^30 on 9-9.6 kb reads: the candidate range of the middle
    # anti-diagonals is about 9,000 cells, wider than the unbounded kernel's
    # 8,192-slot LDS ring, so the extension moves to global memory part way;
    # X = 4000 on the same reads stays in the ring
    rng = np.random.Generator(np.random.PCG64(33))
    a = rng.integers(0, 4, 9600).astype(np.uint8)
    b = a[200:9400].copy()
    flip = rng.random(b.size) < 0.1
    b[flip] = (b[flip] + rng.integers(1, 4, int(flip.sum()))) % 4
    c = rng.integers(0, 4, 9300).astype(np.uint8)
    store = W.ReadStore(np.concatenate([a, b, c]), np.array([0, 9600, 9600 + 9200]),
                        np.array([9600, 9200, 9300]))
    recs = np.zeros(4, W.RECORD_DTYPE)
    recs["read_a"] = [0, 0, 0, 1]
    recs["read_b"] = [1, 2, 2, 2]
    recs["pos_a"] = [0, 9590, 0, 4000]
    recs["pos_b"] = [0, 9290, 0, 4000]
    recs["k"] = [3, 3, 3, 5]
    recs["x"] = [1 << 30, 1 << 30, 4000, 4000]
    recs["match"], recs["mismatch"], recs["gap"] = 1, -1, -1
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    note("unbounded band wider than the LDS ring: 9-9.6 kb reads, X = 2^30 and 4000")
    with xd.Context(store) as ctx:
        res, cells, _ = ctx.run(recs, count_cells=True)
    assert_same(res, cells, ref)


def test_unbounded_resume_into_used_ring(xd):
    # Unrelated 70-95 kb reads at X = 100 (+1/-1/-1), seeds near the start:
    # the right extensions run the whole reads with ragged bands of 2,200-
    # 3,100 cells (dead cells inside the band), climb through both wide
    # classes with their state and resume in the unbounded kernel.  One
    # workgroup (generic_waves 16) runs those extensions one after another,
    # so every resumed band lands in a ring that holds the previous
    # extension's values; the dead cells inside a carried band must read as
    # dead there (the stress mix's long unrelated pairs hit this).
    rng = np.random.Generator(np.random.PCG64(92))
    lens = rng.integers(70000, 95001, size=12)
    codes = rng.integers(0, 4, int(lens.sum())).astype(np.uint8)
    store = W.ReadStore(codes, np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    n = 8
    recs = np.zeros(n, W.RECORD_DTYPE)
    recs["read_a"] = np.arange(n)
    recs["read_b"] = (np.arange(n) + 1 + rng.integers(0, 11, n)) % 12
    recs["pos_a"] = rng.integers(0, 50, n)
    recs["pos_b"] = rng.integers(0, 50, n)
    recs["k"] = 3
    recs["x"] = 100
    recs["match"], recs["mismatch"], recs["gap"] = 1, -1, -1
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    note("unbounded kernel: carried ragged bands resumed in a used ring (one workgroup, 70-95 kb, X = 100)")
    with xd.Context(store) as ctx:
        ctx.set_tuning(generic_waves=16)
        res, cells, st = ctx.run(recs, count_cells=True)
    assert int(st["stage_tasks"][xd.STAGE_NAMES.index("generic")]) >= 4
    assert_same(res, cells, ref)


def test_unbounded_window_then_ring(xd):
    # Unrelated 12-20 kb reads at X = 800-3000: widest bands of 3,300-8,400
    # cells with dead cells inside.  The unbounded class starts each
    # extension in its 4096-slot register window (resumed from the 2048-slot
    # class); bands past 4092 move into the LDS ring, those past 8192 on to
    # global memory.  One workgroup runs every task in turn, so each resume
    # lands in buffers an earlier task used.
    rng = np.random.Generator(np.random.PCG64(93))
    lens = rng.integers(12000, 20001, size=10)
    codes = rng.integers(0, 4, int(lens.sum())).astype(np.uint8)
    store = W.ReadStore(codes, np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    n = 6
    recs = np.zeros(n, W.RECORD_DTYPE)
    recs["read_a"] = np.arange(n)
    recs["read_b"] = np.arange(n) + 4
    recs["pos_a"] = rng.integers(0, 3000, n)
    recs["pos_b"] = rng.integers(0, 3000, n)
    recs["k"] = 5
    recs["strand"] = [0, 1, 0, 1, 0, 1]
    recs["x"] = [800, 1500, 3000, 800, 1500, 4000]
    order = np.argsort(-lens)   # the last record: the two longest reads, seeds at 0
    recs["read_a"][5], recs["read_b"][5], recs["pos_a"][5], recs["pos_b"][5], recs["strand"][5] = \
        order[0], order[1], 0, 0, 0
    recs["match"], recs["mismatch"], recs["gap"] = 1, -1, -1
    widths = []
    for R in recs:
        a, b = store.read(int(R["read_a"])), store.read(int(R["read_b"]))
        k, pa, pb = int(R["k"]), int(R["pos_a"]), int(R["pos_b"])
        if R["strand"]:
            b = W.revcomp_codes(b)
            pb = b.size - pb - k
        for u, v in ((a[:pa][::-1], b[:pb][::-1]), (a[pa + k:], b[pb + k:])):
            widths.append(oracle.extend_band(u.copy(), v.copy(), 1, -1, -1, int(R["x"]))[1])
    widths = np.array(widths)
    # the case holds bands for the window, the ring and global memory
    assert np.any((widths > 2175) & (widths < 3900)) and np.any((widths > 4300) & (widths < 7800)) \
        and np.any(widths > 8600), widths
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    note("unbounded class: register window, then LDS ring and global memory (12-20 kb, X = 800-4000)")
    for gw in (16, 4096):
        with xd.Context(store) as ctx:
            ctx.set_tuning(generic_waves=gw)
            res, cells, st = ctx.run(recs, count_cells=True)
        assert_same(res, cells, ref)
        assert int(st["stage_tasks"][xd.STAGE_NAMES.index("generic")]) == int(np.sum(widths > 2044))


@pytest.mark.parametrize("wide_waves", [1, 2, 4])
def test_class_hand_over_pool_overflow(xd, wide_waves):
    # Every right extension here outgrows the 1024- and 2048-slot windows
    # (X = 2^30, ~2.3 kb on both sides), so each record hands about 6,200
    # words of window state to wider classes: far more than a 1,024-record
    # batch's carry pool holds.  Early tasks resume from their carried
    # state, later ones restart; both must give the oracle's results, with
    # one, two or four wavefronts per extension in the 2048-slot class.
    rng = np.random.Generator(np.random.PCG64(44))
    base = rng.integers(0, 4, 2700).astype(np.uint8)
    reads, lens = [], []
    for _ in range(24):
        r = base[rng.integers(0, 150):].copy()
        r = r[:rng.integers(2300, r.size + 1)]
        flip = rng.random(r.size) < 0.12
        r[flip] = (r[flip] + rng.integers(1, 4, int(flip.sum()))) % 4
        reads.append(r)
        lens.append(r.size)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]])
    store = W.ReadStore(np.concatenate(reads), off, np.array(lens))
    n = 200
    recs = np.zeros(n, W.RECORD_DTYPE)
    recs["read_a"] = rng.integers(0, 24, n)
    recs["read_b"] = (recs["read_a"] + rng.integers(1, 24, n)) % 24
    recs["pos_a"] = rng.integers(0, 20, n)
    recs["pos_b"] = rng.integers(0, 20, n)
    recs["k"] = 1
    recs["x"] = np.where(rng.random(n) < 0.8, 1 << 30, 400)
    recs["match"], recs["mismatch"], recs["gap"] = 1, -1, -1
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    note(f"class hand-over beyond the carry pool: 200 records, X = 2^30 / 400, ~2.3 kb extensions, "
         f"wide_waves {wide_waves}")
    with xd.Context(store) as ctx:
        ctx.set_tuning(wide_waves=wide_waves)
        res, cells, stats = ctx.run(recs, count_cells=True)
    assert_same(res, cells, ref)
    assert int(stats["stage_tasks"][xd.STAGE_NAMES.index("generic")]) > 0   # the unbounded class ran


@pytest.mark.parametrize("weights", [(1, -1, -1), (1, -2, -1), (2, -3, -2)])
def test_group_window_random(xd, weights):
    # related 2-4 kb reads (20 % substitutions) at drops that take many bands
    # through the 1281-2048-cell class: the window shared by 2 and 4
    # wavefronts gives the oracle's results, as one wavefront does; seeds
    # anywhere, both strands, short reads among them
    rng = np.random.Generator(np.random.PCG64(300 + weights[1]))
    base = rng.integers(0, 4, 4200).astype(np.uint8)
    reads = []
    for q in range(16):
        r = base[rng.integers(0, 200):].copy()
        r = r[:rng.integers(300 if q < 2 else 2000, r.size + 1)]
        flip = rng.random(r.size) < 0.2
        r[flip] = (r[flip] + rng.integers(1, 4, int(flip.sum()))) % 4
        reads.append(r)
    lens = np.array([r.size for r in reads])
    store = W.ReadStore(np.concatenate(reads), np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    n = 160
    recs = np.zeros(n, W.RECORD_DTYPE)
    recs["read_a"] = rng.integers(0, 16, n)
    recs["read_b"] = (recs["read_a"] + rng.integers(1, 16, n)) % 16
    recs["k"] = rng.integers(1, 20, n)
    for i in range(n):
        la, lb = lens[recs["read_a"][i]], lens[recs["read_b"][i]]
        recs["pos_a"][i] = rng.integers(0, la - recs["k"][i] + 1)
        recs["pos_b"][i] = rng.integers(0, lb - recs["k"][i] + 1)
    recs["strand"] = rng.integers(0, 2, n)
    recs["x"] = rng.choice([300, 800, 1500, 3000, 1 << 30], n)
    recs["match"], recs["mismatch"], recs["gap"] = weights
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    note(f"group window, random related reads, weights {weights}")
    with xd.Context(store) as ctx:
        for ww in (2, 4, 1):
            ctx.set_tuning(wide_waves=ww)
            res, cells, st = ctx.run(recs, count_cells=True)
            assert_same(res, cells, ref)
            assert int(st["stage_tasks"][xd.STAGE_NAMES.index("wide2048")]) > 0
            sc = np.array(st["stage_cells"], np.uint64)
            assert int(sc.sum()) == int(cells.sum())


# Window classes by the widest live range of an extension (from the oracle):
# the adaptive windows hold bands up to 252 slots, the first wide class up to
# 1276, the second up to 2044; wider bands finish in the unbounded kernel.
# Each case below sits at least 6 % away from those limits.  Extensions of
# small drops with match 1, gap -1 (narrow class, two per wavefront) stay
# there while their band fits 60 slots.
CLASS_BRACKETS = ((0, 235), (275, 1195), (1360, 1915), (2175, 1 << 30))
NARROW_LIMIT = (56, 64)   # a narrow-class band at most the first completes there; none in between
NARROW_X = 20             # default drop bound of the narrow class


def narrow_eligible(weights, x):
    ma, mi, gap = weights
    return x <= NARROW_X and ma == 1 and gap == -1 and mi >= -2
WIDEN_NARROW_CASES = {
    # weights: (read a, read b, X) per record, one or two records per class
    (1, -1, -1): [(2, 1, 14), (0, 2, 25), (2, 3, 30), (2, 3, 300), (0, 1, 600), (2, 3, 1200), (0, 1, 1500)],
    (1, -2, -2): [(0, 1, 190), (0, 1, 400), (0, 1, 500), (0, 1, 2000), (0, 1, 2500), (0, 1, 4000)],
    (2, -3, -2): [(0, 2, 36), (1, 3, 50), (0, 1, 60), (2, 3, 500), (0, 1, 1100), (2, 3, 2000), (0, 1, 2400)],
}


@pytest.mark.parametrize("wide_waves", [1, 2, 4])
@pytest.mark.parametrize("weights", sorted(WIDEN_NARROW_CASES))
def test_bands_widen_then_narrow(xd, weights, wide_waves):
    # A random 2.5-3.2 kb prefix, then 6 kb shared by every read.  Through
    # the random part the band widens: the windows step up their ladders and
    # hand over to wider classes.  In the shared part the band collapses to
    # about X, so the windows step back down.  The three weight sets take the
    # three step variants (sigma in 2-bit fields; match 1 with a wider sigma;
    # general weights), and the 2048-slot class runs with one, two or four
    # wavefronts per extension.  Seeds sit at position 0, so every left extension is
    # empty and every right extension runs the whole reads.  For each weight
    # set the cases reach every class, and each class must complete exactly
    # the extensions whose widest band (from the oracle) it holds.
    rng = np.random.Generator(np.random.PCG64(55))
    shared = rng.integers(0, 4, 6000).astype(np.uint8)
    reads = [np.concatenate([rng.integers(0, 4, n).astype(np.uint8), shared]) for n in (2500, 2600, 3200, 3000)]
    lens = [r.size for r in reads]
    store = W.ReadStore(np.concatenate(reads), np.concatenate([[0], np.cumsum(lens)[:-1]]), np.array(lens))
    cases = WIDEN_NARROW_CASES[weights]
    recs = np.zeros(len(cases), W.RECORD_DTYPE)
    recs["read_a"] = [c[0] for c in cases]
    recs["read_b"] = [c[1] for c in cases]
    recs["k"] = 1
    recs["x"] = [c[2] for c in cases]
    recs["match"], recs["mismatch"], recs["gap"] = weights
    want = [0] * 5           # narrow, adaptive, 1280-slot, 2048-slot, unbounded
    for a, b, x in cases:
        _, width = oracle.extend_band(reads[a][1:], reads[b][1:], *weights, x)
        cls = [k for k, (lo, hi) in enumerate(CLASS_BRACKETS) if lo <= width <= hi]
        assert len(cls) == 1, f"case {(a, b, x)}: widest band {width} too near a class limit"
        if narrow_eligible(weights, x):
            assert not NARROW_LIMIT[0] < width < NARROW_LIMIT[1], f"case {(a, b, x)}: band {width} near 60"
            if width <= NARROW_LIMIT[0]:
                want[0] += 1
                continue
        want[1 + cls[0]] += 1
    assert all(want[1:]), want   # every window class is reached
    for a, b, x in cases:        # the empty left extensions end in the first class they enter
        want[0 if narrow_eligible(weights, x) else 1] += 1
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    note(f"bands that widen through every window class, then narrow; weights {weights}")
    with xd.Context(store) as ctx:
        assert ctx.tuning()["narrow_x"] == NARROW_X
        ctx.set_tuning(narrow_min_records=0, wide_waves=wide_waves)   # narrow class for a batch this small
        assert ctx.tuning()["wide_waves"] == wide_waves
        res, cells, st = ctx.run(recs, count_cells=True)
    assert_same(res, cells, ref)
    tasks = [int(v) for v in st["stage_tasks"][1:6]]
    assert tasks == want, (tasks, want)
    # each stage reports the cells it computed, also for extensions it
    # handed to a wider class: the sums add up to the per-record counts,
    # every window stage holds at least its cells in lane-steps, and every
    # class that ran reports work
    sc = np.array(st["stage_cells"], np.uint64)
    ss = np.array(st["stage_slots"], np.uint64)
    assert int(sc.sum()) == int(cells.sum())
    assert np.all(ss >= sc) and np.all(sc[2:6] > 0), (sc, ss)


def test_identical_reads_full_length(xd):
    rng = np.random.Generator(np.random.PCG64(5))
    seq = rng.integers(0, 4, 3000).astype(np.uint8)
    store = W.ReadStore(np.concatenate([seq, seq]), np.array([0, 3000]), np.array([3000, 3000]))
    recs = np.zeros(6, W.RECORD_DTYPE)
    recs["read_a"], recs["read_b"] = 0, 1
    recs["pos_a"] = recs["pos_b"] = [0, 1000, 2983, 5, 1500, 0]
    recs["k"] = 17
    recs["x"] = [0, 1, 20, 50, 100, 1 << 30]
    recs["match"], recs["mismatch"], recs["gap"] = 1, -1, -1
    note("identical reads")
    with xd.Context(store) as ctx:
        res, cells, _ = ctx.run(recs, count_cells=True)
    assert np.all(res["score"] == 3000)
    assert np.all(res["a_begin"] == 0) and np.all(res["a_end"] == 3000)
    ref, _ = oracle.batch(store.codes, store.off, store.length, recs)
    assert_same(res, cells, ref)


def test_device_path(xd, c0):
    import torch
    wl, ref = c0
    note("device path (torch tensors)")
    d_recs = torch.from_numpy(wl.records.view(np.uint8)).cuda()
    d_out = torch.zeros(len(wl.records) * 32, dtype=torch.uint8, device="cuda")
    d_cells = torch.zeros(len(wl.records), dtype=torch.int64, device="cuda")
    with xd.Context(wl.store) as ctx:
        stream = torch.cuda.current_stream()
        t = ctx.submit_device(d_recs, len(wl.records), d_out, d_cells, stream=stream)
        ctx.wait(t)
        torch.cuda.synchronize()
    res = d_out.cpu().numpy().view(W.RESULT_DTYPE)
    assert_same(res, d_cells.cpu().numpy().astype(np.uint64), ref)


def test_invalid_and_empty(xd, c0):
    wl, _ = c0
    note("invalid records and empty batch")
    with xd.Context(wl.store) as ctx:
        out, _, st = ctx.run(wl.records[:0])
        assert out.size == 0 and st["records"] == 0
        for field, val in (("read_a", 10 ** 6), ("k", 0), ("x", -1), ("gap", 0), ("pos_a", 10 ** 6)):
            bad = wl.records[:5].copy()
            bad[field][2] = val
            with pytest.raises(xd.XdropError) as e:
                ctx.submit(bad)
            assert e.value.status == xd.XDROP_E_INVALID
        # the device path validates on the GPU: the ticket reports the error
        import torch
        bad = wl.records[:300].copy()
        bad["read_b"][7] = 10 ** 7
        d_recs = torch.from_numpy(bad.view(np.uint8)).cuda()
        d_out = torch.zeros(300 * 32, dtype=torch.uint8, device="cuda")
        t = ctx.submit_device(d_recs, 300, d_out)
        with pytest.raises(xd.XdropError) as e:
            ctx.wait(t)
        assert e.value.status == xd.XDROP_E_INVALID
        res, _, _ = ctx.run(wl.records[:10])
        assert np.all(res["score"] > 0)


def test_autotune_and_tuning_cache(xd, c0, tmp_path):
    wl, ref = c0
    note("autotune on c0 (sweep of launch parameters)")
    cache = str(tmp_path / "tune.txt")
    with xd.Context(wl.store) as ctx:
        tuning, best_ms = ctx.autotune(wl.records, cache_path=cache)
        assert best_ms > 0 and tuning["shrink_margin"] >= 1
        res, cells, _ = ctx.run(wl.records, count_cells=True)
    assert_same(res, cells, ref)
    with xd.Context(wl.store, tuning_cache=cache) as ctx2:
        assert ctx2.tuning() == tuning
        # every setting gives the same results
        ctx2.set_tuning(waves_per_cu=4, buckets=0, grow_margin=2, shrink_margin=1, generic_waves=8)
        res2, cells2, _ = ctx2.run(wl.records, count_cells=True)
    assert_same(res2, cells2, ref)


def test_paper_settings_k31_x15(xd):
    # the paper's own runs use k = 31 and an X-drop of 15 ("Results",
    # experimental setup); c1-shaped reads on a smaller genome
    wl = W.make_workload("c1", pairs=3000, k=31, x_choices=(15,), genome=1_000_000)
    ref, _ = oracle.batch(wl.store.codes, wl.store.off, wl.store.length, wl.records)
    note("paper settings: k=31, X=15, 3000 c1-shaped records")
    for mode, narrow_min in ((0, 0), (0, 100000), (1, 0)):
        with xd.Context(wl.store, mode=mode) as ctx:
            ctx.set_tuning(narrow_min_records=narrow_min)   # 0: two extensions per wavefront
            res, cells, _ = ctx.run(wl.records, count_cells=True)
        assert_same(res, cells, ref)
    assert np.all(res["seed_score"] == 31)


def test_stage_counters_and_lane_occupancy(xd, c0):
    # per-stage totals of a counting pass: cells and tasks add up to the
    # per-record counts, and each stage's window lane-steps bound its cells
    wl, ref = c0
    note("stage counters (cells, tasks, lane-steps)")
    with xd.Context(wl.store) as ctx:
        _, cells, st = ctx.run(wl.records, count_cells=True)
    sc = np.array(st["stage_cells"], np.uint64)
    stt = np.array(st["stage_tasks"], np.uint64)
    ss = np.array(st["stage_slots"], np.uint64)
    assert int(sc.sum()) == int(cells.sum())
    assert int(stt.sum()) == 2 * len(wl.records)
    assert np.all(ss >= sc)
    k = xd.STAGE_NAMES.index("adaptive")   # c0: X = 50, all in the adaptive windows
    occ = float(sc[k]) / float(ss[k])
    assert 0.2 < occ <= 1.0, occ
