"""Seeded synthetic workloads for batched X-drop seed-and-extend.

This module only draws inputs: a random genome, long reads sampled from it
with a PacBio-CLR-like error mix, overlapping read pairs, and one planted
exact k-mer seed per pair.  It holds none of the alignment arithmetic, and
both the HIP path and the CPU oracle take their inputs from it.

The E. coli read sets of the paper (section "Results", experimental setup:
29X with 8,605 reads and 100X with 91,394 reads) are not available here; the
presets below stand in for them with the same shape (4.6 Mb genome, 29x and
100x coverage, long reads of several kb, 15 % error).

Recipe (all numpy PCG64, seed = 230907270 + preset index unless given):
  * genome: i.i.d. uniform ACGT;
  * read templates: uniform start, length from the preset's law, strand
    '+'/'-' with probability 1/2; '-' reads are stored reverse-complemented;
  * errors per template base: substitution 8 % (uniform over the 3 other
    bases), insertion 4 % (base kept, then one random base), deletion 3 %,
    unchanged 85 %;
  * pairs: reads whose template intervals overlap by >= 500 bp, sampled
    without replacement; A/B order random;
  * seed: one k-mer (k = 17) at a uniform genome position inside the
    overlap; errors are suppressed in that k-mer in both reads, so the seed is
    exact; strand = 1 when the two reads lie on different strands, pos_b is in
    the stored coordinates of read B.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 230907270

# xdrop_record (32 bytes) -- field order and widths of the C ABI record.
RECORD_DTYPE = np.dtype([
    ("read_a", "<u4"), ("read_b", "<u4"), ("pos_a", "<u4"), ("pos_b", "<u4"),
    ("k", "<u2"), ("strand", "u1"), ("pad", "u1"), ("x", "<i4"),
    ("match", "<i2"), ("mismatch", "<i2"), ("gap", "<i2"), ("pad2", "<i2"),
])
assert RECORD_DTYPE.itemsize == 32

# xdrop_result (32 bytes).
RESULT_DTYPE = np.dtype([
    ("score", "<i4"), ("left_score", "<i4"), ("right_score", "<i4"), ("seed_score", "<i4"),
    ("a_begin", "<u4"), ("a_end", "<u4"), ("b_begin", "<u4"), ("b_end", "<u4"),
])
assert RESULT_DTYPE.itemsize == 32

ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)


@dataclasses.dataclass
class ReadStore:
    codes: np.ndarray      # uint8 codes 0..3, all reads concatenated
    off: np.ndarray        # int64 offset of each read in ``codes``
    length: np.ndarray     # int64 length of each read

    @property
    def n(self) -> int:
        return int(self.length.size)

    def read(self, r: int) -> np.ndarray:
        o = int(self.off[r])
        return self.codes[o:o + int(self.length[r])]

    def ascii(self, r: int) -> bytes:
        return ASCII[self.read(r)].tobytes()

    def ascii_list(self) -> list:
        return [self.ascii(r) for r in range(self.n)]


@dataclasses.dataclass
class Workload:
    name: str
    store: ReadStore
    records: np.ndarray    # RECORD_DTYPE
    meta: dict


@dataclasses.dataclass(frozen=True)
class Preset:
    genome: int
    coverage: float
    length_law: str        # "uniform" or "lognormal"
    len_a: float           # uniform: low;  lognormal: mean
    len_b: float           # uniform: high; lognormal: sd
    clip_lo: int
    clip_hi: int
    pairs: int
    x_choices: tuple
    weights: tuple = (1, -1, -1)
    decoy_fraction: float = 0.0
    decoy_reads: int = 0


PRESETS = {
    # 1,000 pairs, 200 kb genome, reads U[1,2] kb, 30x (our choice), X=50.
    "c0": Preset(200_000, 30.0, "uniform", 1000, 2000, 1000, 2000, 1000, (50,)),
    # 100,000 pairs, 29x of a 4.6 Mb genome, lognormal mean 8 kb sd 4 kb, [1, 30] kb, X=50.
    "c1": Preset(4_600_000, 29.0, "lognormal", 8000, 4000, 1000, 30000, 100_000, (50,)),
    # 1,000,000 pairs, 100x, lognormal mean 10 kb (sd 5 kb assumed), [1, 40] kb, X in {20,50,100}.
    "c2": Preset(4_600_000, 100.0, "lognormal", 10000, 5000, 1000, 40000, 1_000_000, (20, 50, 100)),
    # stress mix: 2M pairs, half true overlaps (100x, mean 20 kb, sd 10 kb assumed, [1, 100] kb),
    # half unrelated pairs against a 50k-read random decoy pool; X=100.
    "c4": Preset(4_600_000, 100.0, "lognormal", 20000, 10000, 1000, 100000, 2_000_000, (100,),
                 decoy_fraction=0.5, decoy_reads=50_000),
    # c4 with weights (+1, -2, -2): unrelated pairs stop early.
    "c4b": Preset(4_600_000, 100.0, "lognormal", 20000, 10000, 1000, 100000, 2_000_000, (100,),
                  weights=(1, -2, -2), decoy_fraction=0.5, decoy_reads=50_000),
}
PRESET_INDEX = {"c0": 0, "c1": 1, "c2": 2, "c3": 3, "c4": 4, "c4b": 5}


def _lengths(rng, p: Preset, n: int) -> np.ndarray:
    if p.length_law == "uniform":
        ln = rng.integers(int(p.len_a), int(p.len_b) + 1, size=n)
    else:
        s2 = math.log(1.0 + (p.len_b / p.len_a) ** 2)
        mu = math.log(p.len_a) - s2 / 2.0
        ln = np.rint(rng.lognormal(mu, math.sqrt(s2), size=n)).astype(np.int64)
    return np.clip(ln, p.clip_lo, p.clip_hi).astype(np.int64)


def revcomp_codes(x: np.ndarray) -> np.ndarray:
    return (3 - x[::-1]).astype(np.uint8)


def overlapping_pairs(start: np.ndarray, end: np.ndarray, min_overlap: int = 500):
    """All unordered pairs of intervals [start, end) overlapping by >= min_overlap."""
    order = np.argsort(start, kind="stable")
    s, e = start[order], end[order]
    hi = np.searchsorted(s, e - min_overlap, side="right")
    cnt = np.maximum(hi - np.arange(s.size) - 1, 0)
    i_idx = np.repeat(np.arange(s.size), cnt)
    first = np.cumsum(cnt) - cnt
    j_idx = i_idx + 1 + (np.arange(i_idx.size) - np.repeat(first, cnt))
    ov = np.minimum(e[i_idx], e[j_idx]) - s[j_idx]
    keep = ov >= min_overlap
    return order[i_idx[keep]], order[j_idx[keep]]


def _apply_errors(rng, genome, t_start, t_len, protect_off, protect_read, k, chunk=1 << 24,
                  rates=(0.08, 0.04, 0.03)):
    """Apply the substitution / insertion / deletion mix (default 8/4/3 %) to
    every template; returns forward-frame reads (concatenated), their
    offsets/lengths and, for each protected k-mer, its position in its read's
    forward frame."""
    p_sub, p_ins, p_del = rates
    n = t_len.size
    out_parts, out_len = [], np.zeros(n, np.int64)
    prot_pos = np.zeros(protect_off.size, np.int64)
    # group protected k-mers by read
    order = np.argsort(protect_read, kind="stable")
    pr_sorted = protect_read[order]
    bounds = np.searchsorted(pr_sorted, np.arange(n + 1))
    r0 = 0
    while r0 < n:
        r1 = r0
        tot = 0
        while r1 < n and (tot == 0 or tot + t_len[r1] <= chunk):
            tot += int(t_len[r1])
            r1 += 1
        lens = t_len[r0:r1]
        toff = np.concatenate([[0], np.cumsum(lens)[:-1]])
        idx = np.repeat(t_start[r0:r1] - toff, lens) + np.arange(tot)
        tmpl = genome[idx]
        # protected bases (planted seeds) keep their template base
        diff = np.zeros(tot + 1, np.int32)
        sel = order[bounds[r0]:bounds[r1]]
        if sel.size:
            g0 = toff[protect_read[sel] - r0] + protect_off[sel]
            np.add.at(diff, g0, 1)
            np.add.at(diff, g0 + k, -1)
        prot = np.cumsum(diff[:-1]) > 0
        u = rng.random(tot)
        sub = (u < p_sub) & ~prot
        ins = (u >= p_sub) & (u < p_sub + p_ins) & ~prot
        dele = (u >= p_sub + p_ins) & (u < p_sub + p_ins + p_del) & ~prot
        base = tmpl.copy()
        base[sub] = (base[sub] + rng.integers(1, 4, size=int(sub.sum()))) % 4
        cnt = np.ones(tot, np.int64) + ins - dele
        pos = np.cumsum(cnt) - cnt                     # output index of each template base
        out = np.empty(int(cnt.sum()), np.uint8)
        kept = ~dele
        out[pos[kept]] = base[kept]
        out[pos[ins] + 1] = rng.integers(0, 4, size=int(ins.sum())).astype(np.uint8)
        starts_out = pos[toff]
        ends_out = np.concatenate([starts_out[1:], [out.size]])
        out_len[r0:r1] = ends_out - starts_out
        out_parts.append(out)
        if sel.size:
            prot_pos[sel] = pos[g0] - starts_out[protect_read[sel] - r0]
        r0 = r1
    codes = np.concatenate(out_parts) if out_parts else np.zeros(0, np.uint8)
    off = np.concatenate([[0], np.cumsum(out_len)[:-1]]).astype(np.int64)
    return codes, off, out_len, prot_pos


def make_workload(name: str, seed: int | None = None, pairs: int | None = None,
                  x_choices: tuple | None = None, weights: tuple | None = None,
                  k: int = 17, min_overlap: int = 500, genome: int | None = None,
                  coverage: float | None = None) -> Workload:
    """Build one preset (``c0`` .. ``c4b``), optionally scaled down.

    ``pairs``/``genome``/``coverage`` shrink a preset for quick tests; the
    defaults are the full sizes.
    """
    p = PRESETS[name]
    if seed is None:
        seed = SEED_BASE + PRESET_INDEX[name]
    rng = np.random.Generator(np.random.PCG64(seed))
    G = genome or p.genome
    cov = coverage or p.coverage
    n_pairs = pairs if pairs is not None else p.pairs
    xs = tuple(x_choices or p.x_choices)
    ma, mi, g = weights or p.weights
    n_true = n_pairs - int(round(n_pairs * p.decoy_fraction))
    n_decoy_pairs = n_pairs - n_true

    gen = rng.integers(0, 4, size=G, dtype=np.uint8)
    mean_len = p.len_a if p.length_law == "lognormal" else (p.len_a + p.len_b) / 2
    n_reads = max(2, int(round(cov * G / mean_len)))
    t_len = np.minimum(_lengths(rng, p, n_reads), G)
    t_start = (rng.random(n_reads) * (G - t_len + 1)).astype(np.int64)
    t_strand = rng.integers(0, 2, size=n_reads).astype(np.int64)

    ia, ib = overlapping_pairs(t_start, t_start + t_len, min_overlap)
    if ia.size < n_true:
        raise ValueError(f"{name}: only {ia.size} overlapping pairs for {n_true} requested")
    pick = rng.choice(ia.size, size=n_true, replace=False)
    ra, rb = ia[pick], ib[pick]
    swap = rng.integers(0, 2, size=n_true).astype(bool)
    ra, rb = np.where(swap, rb, ra), np.where(swap, ra, rb)
    ov_s = np.maximum(t_start[ra], t_start[rb])
    ov_e = np.minimum(t_start[ra] + t_len[ra], t_start[rb] + t_len[rb])
    sp = ov_s + (rng.random(n_true) * (ov_e - ov_s - k + 1)).astype(np.int64)

    prot_read = np.concatenate([ra, rb])
    prot_off = np.concatenate([sp - t_start[ra], sp - t_start[rb]])
    codes, off, length, ppos = _apply_errors(rng, gen, t_start, t_len, prot_off, prot_read, k)
    # '-' reads are stored reverse-complemented
    minus = np.flatnonzero(t_strand == 1)
    for r in minus:
        o, ln = int(off[r]), int(length[r])
        codes[o:o + ln] = revcomp_codes(codes[o:o + ln])
    fwd_a, fwd_b = ppos[:n_true], ppos[n_true:]
    pos_a = np.where(t_strand[ra] == 1, length[ra] - fwd_a - k, fwd_a)
    pos_b = np.where(t_strand[rb] == 1, length[rb] - fwd_b - k, fwd_b)
    strand = (t_strand[ra] != t_strand[rb]).astype(np.int64)

    n_store = n_reads
    if n_decoy_pairs:
        d_len = np.minimum(_lengths(rng, p, p.decoy_reads), G)
        d_codes = rng.integers(0, 4, size=int(d_len.sum()), dtype=np.uint8)
        d_off = off[-1] + length[-1] + np.concatenate([[0], np.cumsum(d_len)[:-1]])
        codes = np.concatenate([codes, d_codes])
        off = np.concatenate([off, d_off])
        length = np.concatenate([length, d_len])
        da = rng.integers(0, n_reads, size=n_decoy_pairs)
        db = n_reads + rng.integers(0, p.decoy_reads, size=n_decoy_pairs)
        dpa = (rng.random(n_decoy_pairs) * (length[da] - k + 1)).astype(np.int64)
        dpb = (rng.random(n_decoy_pairs) * (length[db] - k + 1)).astype(np.int64)
        dst = rng.integers(0, 2, size=n_decoy_pairs)
        ra = np.concatenate([ra, da]); rb = np.concatenate([rb, db])
        pos_a = np.concatenate([pos_a, dpa]); pos_b = np.concatenate([pos_b, dpb])
        strand = np.concatenate([strand, dst])
        n_store += p.decoy_reads

    n_all = ra.size
    rec = np.zeros(n_all, RECORD_DTYPE)
    rec["read_a"], rec["read_b"] = ra, rb
    rec["pos_a"], rec["pos_b"] = pos_a, pos_b
    rec["k"], rec["strand"] = k, strand
    rec["x"] = np.asarray(xs, np.int64)[rng.integers(0, len(xs), size=n_all)]
    rec["match"], rec["mismatch"], rec["gap"] = ma, mi, g
    if n_decoy_pairs:
        perm = rng.permutation(n_all)
        rec = rec[perm]
    meta = dict(name=name, seed=seed, genome=G, coverage=cov, reads=n_store, pairs=n_all,
                true_pairs=n_true, decoy_pairs=n_decoy_pairs, x_choices=list(xs),
                weights=[ma, mi, g], k=k, min_overlap=min_overlap,
                mean_read_len=float(length.mean()), total_bases=int(length.sum()))
    return Workload(name, ReadStore(codes, off.astype(np.int64), length.astype(np.int64)), rec, meta)


def random_records(rng, store: ReadStore, n: int, x_choices=(0, 1, 5, 20, 50), k_max: int = 20,
                   weights=((1, -1, -1), (2, -3, -2), (1, -2, -2), (3, -1, -4))) -> np.ndarray:
    """Records with seeds anywhere in the reads (not necessarily exact), mixed
    strands, drops and weights -- for edge-case and brute-force parity tests."""
    rec = np.zeros(n, RECORD_DTYPE)
    ra = rng.integers(0, store.n, size=n)
    rb = rng.integers(0, store.n, size=n)
    la, lb = store.length[ra], store.length[rb]
    kk = np.minimum(rng.integers(1, k_max + 1, size=n), np.minimum(la, lb))
    rec["read_a"], rec["read_b"] = ra, rb
    rec["k"] = kk
    rec["pos_a"] = (rng.random(n) * (la - kk + 1)).astype(np.int64)
    rec["pos_b"] = (rng.random(n) * (lb - kk + 1)).astype(np.int64)
    rec["strand"] = rng.integers(0, 2, size=n)
    rec["x"] = np.asarray(x_choices)[rng.integers(0, len(x_choices), size=n)]
    w = np.asarray(weights)[rng.integers(0, len(weights), size=n)]
    rec["match"], rec["mismatch"], rec["gap"] = w[:, 0], w[:, 1], w[:, 2]
    return rec


def random_store(rng, n_reads: int, lo: int, hi: int, related: float = 0.5) -> ReadStore:
    """Small reads: half unrelated random sequences, half mutated copies of a
    shared random template (so that some pairs align)."""
    lens = rng.integers(lo, hi + 1, size=n_reads)
    tmpl = rng.integers(0, 4, size=max(hi, 1) * 2, dtype=np.uint8)
    parts = []
    for ln in lens:
        if rng.random() < related:
            s = int(rng.integers(0, tmpl.size - ln + 1))
            x = tmpl[s:s + ln].copy()
            flip = rng.random(ln) < 0.1
            x[flip] = rng.integers(0, 4, size=int(flip.sum()))
        else:
            x = rng.integers(0, 4, size=ln, dtype=np.uint8)
        parts.append(x.astype(np.uint8))
    codes = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    return ReadStore(codes, off, lens.astype(np.int64))


def make_readset(name: str = "c1", error: float = 0.01, seed: int | None = None, genome: int | None = None,
                 coverage: float | None = None) -> ReadStore:
    """Reads only (no records), for seed discovery: the preset's genome size,
    coverage and length law, strands +/- with p = 1/2 ('-' stored reverse-
    complemented), and a total error rate split 8:4:3 into substitutions,
    insertions and deletions.  A shared 31-mer survives in ~(1-error)^31 of
    the reads that cover it, so the paper's frequency windows ([20, 30] at
    29x, [20, 50] at 100x) only select k-mers of near error-free reads."""
    p = PRESETS[name]
    if seed is None:
        seed = SEED_BASE + 100 + PRESET_INDEX[name]
    rng = np.random.Generator(np.random.PCG64(seed))
    G = genome or p.genome
    cov = coverage or p.coverage
    gen = rng.integers(0, 4, size=G, dtype=np.uint8)
    mean_len = p.len_a if p.length_law == "lognormal" else (p.len_a + p.len_b) / 2
    n_reads = max(2, int(round(cov * G / mean_len)))
    t_len = np.minimum(_lengths(rng, p, n_reads), G)
    t_start = (rng.random(n_reads) * (G - t_len + 1)).astype(np.int64)
    t_strand = rng.integers(0, 2, size=n_reads).astype(np.int64)
    rates = (error * 8 / 15, error * 4 / 15, error * 3 / 15)
    codes, off, length, _ = _apply_errors(rng, gen, t_start, t_len, np.zeros(0, np.int64),
                                          np.zeros(0, np.int64), 1, rates=rates)
    for r in np.flatnonzero(t_strand == 1):
        o, ln = int(off[r]), int(length[r])
        codes[o:o + ln] = revcomp_codes(codes[o:o + ln])
    return ReadStore(codes, off, length)
