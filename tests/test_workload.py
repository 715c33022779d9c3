"""The seeded generator: shapes, determinism and planted exact seeds."""
import numpy as np

from paper_2309_07270_amd import workload as W


def _oriented(wl, t):
    r = wl.records[t]
    A, B = wl.store.read(r["read_a"]), wl.store.read(r["read_b"])
    k = int(r["k"])
    if r["strand"]:
        Bp, pb = W.revcomp_codes(B), len(B) - int(r["pos_b"]) - k
    else:
        Bp, pb = B, int(r["pos_b"])
    return A, Bp, int(r["pos_a"]), pb, k


def test_c0_shape_and_exact_seeds():
    wl = W.make_workload("c0")
    assert len(wl.records) == 1000 and wl.records.dtype == W.RECORD_DTYPE
    assert wl.store.length.min() >= 900 and wl.store.length.max() <= 2200
    for t in range(len(wl.records)):
        A, Bp, pa, pb, k = _oriented(wl, t)
        assert np.array_equal(A[pa:pa + k], Bp[pb:pb + k])
    assert set(np.unique(wl.records["x"])) == {50}
    assert 0.4 < wl.records["strand"].mean() < 0.6


def test_determinism_and_scaling():
    a = W.make_workload("c1", pairs=500, genome=300_000)
    b = W.make_workload("c1", pairs=500, genome=300_000)
    assert np.array_equal(a.records, b.records) and np.array_equal(a.store.codes, b.store.codes)
    assert 5000 < a.store.length.mean() < 11000


def test_error_mix_rates():
    # read vs its template: the length grows by about ins - del = +1 %
    wl = W.make_workload("c0")
    ratio = wl.store.length.sum() / (1500 * len(wl.store.length))
    assert 0.97 < ratio < 1.05


def test_overlapping_pairs_enumeration():
    start = np.array([0, 100, 700, 5000])
    end = np.array([1000, 900, 1800, 6000])
    i, j = W.overlapping_pairs(start, end, 500)
    got = sorted(tuple(sorted(p)) for p in zip(i.tolist(), j.tolist()))
    # (0,1): 800 bp; (0,2): 300 < 500; (1,2): 200
    assert got == [(0, 1)]


def test_decoy_mix():
    wl = W.make_workload("c4", pairs=2000, genome=200_000, coverage=20)
    assert wl.meta["decoy_pairs"] == 1000
    assert wl.records["read_b"].max() >= wl.meta["reads"] - 50_000
