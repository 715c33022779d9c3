"""GPU seed discovery (xdrop_find_seeds) against the seed oracle.

The record set is unique, its order is not: both sides are compared as sets
of (read_a, read_b, pos_a, pos_b, strand), integer-exact.
"""
import os
import sys

import numpy as np
import pytest

from oracle import seeds as S
from paper_2309_07270_amd import workload as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
BASES = "ACGT"


def note(msg):
    print(f"[gpu-seeds] {msg}", flush=True)
    sys.stdout.flush()


def tuples(recs):
    return sorted((int(r["read_a"]), int(r["read_b"]), int(r["pos_a"]), int(r["pos_b"]), int(r["strand"]))
                  for r in recs)


@pytest.fixture(scope="module")
def xd():
    import torch
    assert torch.cuda.is_available()
    from paper_2309_07270_amd import xdrop
    xdrop.load_library()
    return xdrop


def test_hand_vectors(xd):
    note("hand-derived seed vectors")
    for line in open(os.path.join(HERE, "golden", "seed_hand.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        reads_s, par_s, rec_s = [t.strip() for t in line.split("|")]
        reads = reads_s.split()
        k, lo, hi = map(int, par_s.split())
        want = sorted(tuple(map(int, r.split())) for r in rec_s.split(";"))
        codes = np.array([BASES.index(c) for r in reads for c in r], np.uint8)
        length = np.array([len(r) for r in reads])
        store = W.ReadStore(codes, np.concatenate([[0], np.cumsum(length)[:-1]]), length)
        with xd.Context(store) as ctx:
            recs, st = ctx.find_seeds(k=k, lo=lo, hi=hi, x=7)
        assert tuples(recs) == want
        assert np.all(recs["k"] == k) and np.all(recs["x"] == 7)


@pytest.mark.parametrize("k,stride,lo,hi,err", [(31, 1, 10, 40, 0.01), (15, 2, 3, 25, 0.02),
                                                 (21, 1, 2, 8, 0.05), (9, 3, 1, 4, 0.1)])
def test_parity_small(xd, k, stride, lo, hi, err):
    st = W.make_readset("c0", error=err, genome=15_000, coverage=20, seed=77 + k)
    want = S.find_seeds(st.codes, st.off, st.length, k=k, stride=stride, lo=lo, hi=hi)
    note(f"k={k} stride={stride} window [{lo},{hi}] error {err}: {st.n} reads, {len(want)} pairs")
    with xd.Context(st) as ctx:
        recs, stats = ctx.find_seeds(k=k, stride=stride, lo=lo, hi=hi)
    assert stats["pairs"] == len(want)
    assert tuples(recs) == tuples(want)


def test_c1_shaped_sampled(xd):
    # 29x reads of a 1 Mb genome, 1 % error, the paper's k = 31 and window [20, 30]
    st = W.make_readset("c1", error=0.01, genome=1_000_000)
    note(f"c1-shaped read set: {st.n} reads, {int(st.length.sum())} bases")
    with xd.Context(st) as ctx:
        recs, stats = ctx.find_seeds(k=31, lo=20, hi=30)
    keys, reads, poss, revs = S.kmer_occurrences(st.codes, st.off, st.length, 31)
    rel = S.reliable_kmers(keys, 20, 30)
    assert stats["kmers"] == keys.size and stats["reliable"] == rel.size
    assert stats["distinct"] == np.unique(keys).size
    assert len(recs) == stats["pairs"] > 1000
    pairs = set(zip(recs["read_a"].tolist(), recs["read_b"].tolist()))
    assert len(pairs) == len(recs) and np.all(recs["read_a"] < recs["read_b"])
    # sampled pairs: the smallest candidate over the two reads' reliable occurrences
    sel = np.isin(keys, rel)
    keys, reads, poss, revs = keys[sel], reads[sel], poss[sel], revs[sel]
    rng = np.random.default_rng(3)
    for t in rng.choice(len(recs), size=60, replace=False):
        a, b = int(recs[t]["read_a"]), int(recs[t]["read_b"])
        ia, ib = np.flatnonzero(reads == a), np.flatnonzero(reads == b)
        common = np.intersect1d(keys[ia], keys[ib])
        best = None
        for kk in common:
            for i in ia[keys[ia] == kk]:
                for j in ib[keys[ib] == kk]:
                    cand = (int(poss[i]), int(poss[j]), int(revs[i] != revs[j]))
                    best = cand if best is None or cand < best else best
        assert best == (int(recs[t]["pos_a"]), int(recs[t]["pos_b"]), int(recs[t]["strand"])), (a, b)


def test_edge_cases(xd):
    st = W.make_readset("c0", error=0.01, genome=10_000, coverage=15, seed=5)
    with xd.Context(st) as ctx:
        note("empty window, too small an output, k longer than every read")
        recs, stats = ctx.find_seeds(k=31, lo=1000, hi=2000)
        assert len(recs) == 0 and stats["reliable"] == 0
        full, _ = ctx.find_seeds(k=21, lo=2, hi=30)
        assert len(full) > 10
        with pytest.raises(xd.XdropError) as e:
            ctx.find_seeds(k=21, lo=2, hi=30, max_records=len(full) // 2)
        assert e.value.status == xd.XDROP_E_NOMEM
        for bad in (dict(k=0), dict(k=32), dict(stride=0), dict(lo=5, hi=4), dict(x=-1)):
            with pytest.raises(xd.XdropError) as e:
                ctx.find_seeds(**bad)
            assert e.value.status == xd.XDROP_E_INVALID
    short = W.ReadStore(np.zeros(20, np.uint8), np.array([0, 10]), np.array([10, 10]))
    with xd.Context(short) as ctx:
        recs, stats = ctx.find_seeds(k=11, lo=1, hi=5)
        assert len(recs) == 0 and stats["kmers"] == 0


def test_device_output_equals_host_output(xd):
    import torch
    st = W.make_readset("c0", error=0.01, genome=15_000, coverage=20, seed=91)
    note("device output of xdrop_find_seeds")
    with xd.Context(st) as ctx:
        host, _ = ctx.find_seeds(k=21, lo=3, hi=30)
        d_out = torch.zeros(len(host) * 32, dtype=torch.uint8, device="cuda")
        n, stats = ctx.find_seeds_device(d_out, len(host), k=21, lo=3, hi=30)
        torch.cuda.synchronize()
    dev = d_out.cpu().numpy().view(W.RECORD_DTYPE)
    assert n == len(host) == stats["pairs"]
    assert tuples(dev) == tuples(host)
