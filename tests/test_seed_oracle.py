"""Pins of the seed-discovery oracle (oracle/seeds.py), on the CPU.

* hand-derived vectors (tests/golden/seed_hand.txt);
* brute force with strings: k-mers, reverse complements and canonical forms
  taken as Python strings (no base-4 encoding), counted in a dict;
* properties: every seed is an exact match of a reliable k-mer in the
  stated orientation; the pair set does not change when a read is stored
  reverse-complemented; stride s keeps exactly the positions p = 0 mod s.
"""
import os
from collections import Counter

import numpy as np
import pytest

from oracle import seeds as S
from paper_2309_07270_amd import workload as W

HERE = os.path.dirname(os.path.abspath(__file__))
BASES = "ACGT"
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def store_of(reads):
    codes = np.array([BASES.index(c) for r in reads for c in r], np.uint8)
    length = np.array([len(r) for r in reads], np.int64)
    off = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.int64)
    return codes, off, length


def as_tuples(recs):
    return sorted((int(r["read_a"]), int(r["read_b"]), int(r["pos_a"]), int(r["pos_b"]), int(r["strand"]))
                  for r in recs)


def brute_force(reads, k, lo, hi, stride=1):
    rc = lambda s: "".join(COMP[c] for c in reversed(s))
    occ = []
    for r, s in enumerate(reads):
        for p in range(0, len(s) - k + 1, stride):
            km = s[p:p + k]
            can = min(km, rc(km))
            occ.append((can, r, p, km != can))
    freq = Counter(o[0] for o in occ)
    best = {}
    for x in occ:
        for y in occ:
            if x[0] != y[0] or not lo <= freq[x[0]] <= hi or x[1] >= y[1]:
                continue
            cand = (x[2], y[2], int(x[3] != y[3]))
            if (x[1], y[1]) not in best or cand < best[(x[1], y[1])]:
                best[(x[1], y[1])] = cand
    return sorted((a, b) + c for (a, b), c in best.items())


def test_hand_vectors():
    rows = 0
    for line in open(os.path.join(HERE, "golden", "seed_hand.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        reads_s, par_s, rec_s = [t.strip() for t in line.split("|")]
        reads = reads_s.split()
        k, lo, hi = map(int, par_s.split())
        want = sorted(tuple(map(int, r.split())) for r in rec_s.split(";"))
        got = as_tuples(S.find_seeds(*store_of(reads), k=k, lo=lo, hi=hi))
        assert got == want, (reads, k, lo, hi)
        rows += 1
    assert rows == 2


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_strings(seed):
    rng = np.random.default_rng(seed)
    tmpl = "".join(rng.choice(list(BASES), 60))
    reads = []
    for _ in range(int(rng.integers(3, 7))):
        s0 = int(rng.integers(0, 40))
        r = list(tmpl[s0:s0 + int(rng.integers(8, 20))])
        for i in range(len(r)):
            if rng.random() < 0.05:
                r[i] = BASES[int(rng.integers(0, 4))]
        r = "".join(r)
        if rng.random() < 0.5:
            r = "".join(COMP[c] for c in reversed(r))
        reads.append(r)
    k = int(rng.choice([3, 4, 5, 7]))
    lo, hi = int(rng.integers(1, 3)), int(rng.integers(3, 12))
    stride = int(rng.choice([1, 1, 2, 3]))
    got = as_tuples(S.find_seeds(*store_of(reads), k=k, stride=stride, lo=lo, hi=hi))
    assert got == brute_force(reads, k, lo, hi, stride)


def test_seeds_exact_and_reliable():
    st = W.make_readset("c0", error=0.01, genome=20_000, coverage=25)
    recs = S.find_seeds(st.codes, st.off, st.length, k=31, lo=10, hi=40)
    assert len(recs) > 50
    keys, _, _, _ = S.kmer_occurrences(st.codes, st.off, st.length, 31)
    freq = Counter(keys.tolist())
    w = 4 ** np.arange(30, -1, -1)
    for r in recs[:300]:
        a = st.read(int(r["read_a"]))[r["pos_a"]:r["pos_a"] + 31]
        b = st.read(int(r["read_b"]))
        b = b[r["pos_b"]:r["pos_b"] + 31]
        if r["strand"]:
            b = W.revcomp_codes(b)
        assert np.array_equal(a, b)
        code = int(a.astype(np.int64) @ w)
        rcode = int(W.revcomp_codes(a).astype(np.int64) @ w)
        assert 10 <= freq[min(code, rcode)] <= 40


def test_pair_set_unchanged_by_storing_a_read_reverse_complemented():
    st = W.make_readset("c0", error=0.005, genome=8_000, coverage=20)
    base = S.find_seeds(st.codes, st.off, st.length, k=15, lo=3, hi=30)
    codes = st.codes.copy()
    for r in (0, 3, 5):
        o, n = int(st.off[r]), int(st.length[r])
        codes[o:o + n] = W.revcomp_codes(codes[o:o + n])
    flipped = S.find_seeds(codes, st.off, st.length, k=15, lo=3, hi=30)
    assert len(base) > 20
    assert set(zip(base["read_a"], base["read_b"])) == set(zip(flipped["read_a"], flipped["read_b"]))


def test_oracle_imports_nothing_from_the_product():
    # the oracle modules load and run in a process that never imports the
    # product package, and the seed records use the C ABI's record layout
    import subprocess
    import sys
    root = os.path.dirname(HERE)
    code = ("import sys, numpy as np; import oracle, oracle.seeds as S; oracle.load();"
            "c = np.array([0,1,2,3,0,1,2,3,0,1,2,3], np.uint8);"
            "r = S.find_seeds(c, np.array([0, 6]), np.array([6, 6]), k=3, lo=1, hi=9);"
            "assert len(r) == 1;"
            "bad = [m for m in sys.modules if m.startswith('paper_2309_07270_amd')];"
            "assert not bad, bad")
    subprocess.run([sys.executable, "-c", code], cwd=root, check=True)
    assert S.SEED_RECORD_DTYPE == W.RECORD_DTYPE
