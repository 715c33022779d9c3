"""Seed discovery oracle: shared reliable k-mers -> one seed record per read pair.

TEST INFRASTRUCTURE ONLY.  Only tests/ and bench.py's cpu_baseline leg use
it; nothing in the product path imports it, and it shares no code with the
HIP path.

What it computes (paper: "Related works", BELLA detects overlaps with a
seed-based approach over reliable k-mers and extends each seed with an
X-drop; "Method", the runs use k-mers of length 31 at stride 1 and keep
k-mers whose frequency lies in [LOWER_KMER_FREQ, UPPER_KMER_FREQ], 20..30
for the 29x set and 20..50 for the 100x set).  The paper fixes nothing
else; the reading implemented here, step by step:

1. Every read contributes the k-mer starting at each position p = 0, s, 2s,
   ... with p + k <= length (k <= 31, stride s).
2. A k-mer and its reverse complement are the same k-mer; it is represented
   by the lexicographically smaller of the two strings (A < C < G < T), its
   canonical form.  An occurrence is "forward" when the read holds the
   canonical string itself, "reverse" when it holds its reverse complement.
3. The frequency of a canonical k-mer is its number of occurrences over all
   reads and positions.  It is reliable when lo <= frequency <= hi.
4. Two different reads a < b are a candidate pair when they share a reliable
   k-mer.  Every pair of occurrences (a, p_a, o_a), (b, p_b, o_b) of one
   reliable k-mer is a candidate seed: strand 0 when o_a == o_b, else 1
   (B is then aligned reverse-complemented), pos_a = p_a and pos_b = p_b,
   both in the reads' stored (forward) coordinates.  With strand 1 the seed
   sits at |B| - p_b - k in the reverse complement of B, where it equals
   A[p_a, p_a + k).
5. The pair's seed is the candidate with the smallest (pos_a, pos_b, strand).
6. Output: one record per candidate pair with that seed, k, and the given
   drop and weights, ordered by (read_a, read_b).
"""
from __future__ import annotations

import numpy as np

__all__ = ["kmer_occurrences", "reliable_kmers", "find_seeds", "SEED_RECORD_DTYPE"]

# Layout of one output record: the 32-byte seed-and-extend record of the
# library's C ABI (read ids, seed start in both reads' stored coordinates,
# seed length, strand, drop and weights), restated here so that this module
# depends on nothing outside oracle/.
SEED_RECORD_DTYPE = np.dtype([
    ("read_a", "<u4"), ("read_b", "<u4"), ("pos_a", "<u4"), ("pos_b", "<u4"),
    ("k", "<u2"), ("strand", "u1"), ("pad", "u1"), ("x", "<i4"),
    ("match", "<i2"), ("mismatch", "<i2"), ("gap", "<i2"), ("pad2", "<i2"),
])
assert SEED_RECORD_DTYPE.itemsize == 32


def kmer_occurrences(codes: np.ndarray, off: np.ndarray, length: np.ndarray, k: int, stride: int = 1):
    """Steps 1-2: (canonical code, read, position, reverse) of every k-mer.

    The canonical code is the base-4 number of the canonical string, first
    base most significant, so numeric order is lexicographic order."""
    if not 1 <= k <= 31:
        raise ValueError("k must be in 1..31")
    weights = 4 ** np.arange(k - 1, -1, -1, dtype=np.int64)   # first base most significant
    keys, reads, poss, revs = [], [], [], []
    for r in range(len(length)):
        n = int(length[r])
        if n < k:
            continue
        seq = codes[int(off[r]):int(off[r]) + n].astype(np.int64)
        win = np.lib.stride_tricks.sliding_window_view(seq, k)[::stride]
        fwd = win @ weights
        rc = (3 - win[:, ::-1]) @ weights                        # reverse complement string
        keys.append(np.minimum(fwd, rc))
        revs.append(rc < fwd)
        poss.append(np.arange(0, n - k + 1, stride, dtype=np.int64))
        reads.append(np.full(win.shape[0], r, np.int64))
    if not keys:
        z = np.zeros(0, np.int64)
        return z, z, z, np.zeros(0, bool)
    return np.concatenate(keys), np.concatenate(reads), np.concatenate(poss), np.concatenate(revs)


def reliable_kmers(keys: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Step 3: the canonical codes whose frequency lies in [lo, hi]."""
    uniq, cnt = np.unique(keys, return_counts=True)
    return uniq[(cnt >= lo) & (cnt <= hi)]


def find_seeds(codes, off, length, k: int = 31, stride: int = 1, lo: int = 20, hi: int = 30,
               x: int = 15, weights=(1, -1, -1)) -> np.ndarray:
    """Steps 1-6: seed records (SEED_RECORD_DTYPE) ordered by (read_a, read_b)."""
    keys, reads, poss, revs = kmer_occurrences(codes, off, length, k, stride)
    rel = reliable_kmers(keys, lo, hi)
    sel = np.isin(keys, rel)
    keys, reads, poss, revs = keys[sel], reads[sel], poss[sel], revs[sel]
    order = np.argsort(keys, kind="stable")
    keys, reads, poss, revs = keys[order], reads[order], poss[order], revs[order]
    bounds = np.flatnonzero(np.diff(keys)) + 1
    best: dict = {}
    for grp in np.split(np.arange(keys.size), bounds):
        for ii in range(grp.size):
            i = grp[ii]
            for jj in range(ii + 1, grp.size):
                j = grp[jj]
                if reads[i] == reads[j]:
                    continue
                a, b = (i, j) if reads[i] < reads[j] else (j, i)
                cand = (int(poss[a]), int(poss[b]), int(revs[a] != revs[b]))
                pair = (int(reads[a]), int(reads[b]))
                if pair not in best or cand < best[pair]:
                    best[pair] = cand
    out = np.zeros(len(best), SEED_RECORD_DTYPE)
    for t, (pair, (pa, pb, st)) in enumerate(sorted(best.items())):
        out[t]["read_a"], out[t]["read_b"] = pair
        out[t]["pos_a"], out[t]["pos_b"], out[t]["strand"] = pa, pb, st
    out["k"] = k
    out["x"] = x
    out["match"], out["mismatch"], out["gap"] = weights
    return out
