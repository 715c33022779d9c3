"""Pins of the CPU oracle against things other than itself.

* hand-traced extensions (tests/golden/hand_traces.txt);
* worked extensions and a worked record from an implementation of the
  reading written independently of the oracle, including vectors on which
  other readings of X-drop differ and the non-monotone-in-X example
  (tests/golden/reading_vectors.txt, tests/golden/worked_record.txt);
* brute force: with a drop so large that nothing is ever pruned, the X-drop
  result must be the best cell of the full Needleman-Wunsch prefix table with
  the tie-break (max score, min i+j, min i); that table is itself checked
  against an enumeration of every alignment path on tiny inputs;
* closed form: with no pruning every cell but (0,0) is evaluated, so
  cells = (m+1)(n+1) - 1;
* invariants that hold for any X: identical prefixes extend to the end with
  score match*|a|; 0 <= T <= NW optimum; T and cells are symmetric in (a, b)
  and invariant under complementing both; an extension that stopped on two
  dead anti-diagonals ignores anything appended after the point it reached;
* record level: a strand-'-' record equals the '+' record on the explicit
  reverse complement of B; score = left + seed + right;
* mutation check: each planted mistake (OX_MUTATION=1..7) fails at least one
  of the pins above.
Paper context: "Related works" (BELLA: seed-and-extend with X-drop; LOGAN:
anti-diagonal X-drop) and "Results" (NW/SW with X-drop).
"""
import itertools
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

INF = oracle.INF_X
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_traces.txt")
WEIGHTS = [(1, -1, -1), (2, -3, -2), (1, -2, -2), (3, -1, -4), (5, -4, -3)]
ALPHA = "ACGT"


def read_golden():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        lhs, rhs = line.split("->")
        a, b, ma, mi, g, X = lhs.split()
        a = "" if a == "-" else a
        b = "" if b == "-" else b
        rows.append((a, b, int(ma), int(mi), int(g), int(X), tuple(int(v) for v in rhs.split())))
    return rows


VECTORS = os.path.join(os.path.dirname(__file__), "golden", "reading_vectors.txt")
RECORD = os.path.join(os.path.dirname(__file__), "golden", "worked_record.txt")


def read_vectors():
    """(a, b, ma, mi, g, X, (T, i, j, cells or None)) rows of reading_vectors.txt."""
    rows = []
    for line in open(VECTORS):
        line = line.split("#")[0].strip()
        if not line:
            continue
        lhs, rhs = line.split("->")
        a, b, ma, mi, g, X = lhs.split()
        T, i, j, cells = rhs.split()
        rows.append(("" if a == "-" else a, "" if b == "-" else b, int(ma), int(mi), int(g), int(X),
                     (int(T), int(i), int(j), None if cells == "*" else int(cells))))
    return rows


def read_records():
    rows = []
    for line in open(RECORD):
        line = line.split("#")[0].strip()
        if not line:
            continue
        lhs, rhs = line.split("->")
        A, B, *nums = lhs.split()
        rows.append((A, B, [int(v) for v in nums], [int(v) for v in rhs.split()]))
    return rows


def rand_seq(rng, lo, hi):
    return "".join(rng.choice(list(ALPHA), int(rng.integers(lo, hi + 1))))


def related_pair(rng, lo, hi, err=0.15):
    a = rand_seq(rng, lo, hi)
    b = []
    for ch in a:
        u = rng.random()
        if u < err / 3:
            continue
        if u < 2 * err / 3:
            b.append(rng.choice(list(ALPHA)))
        b.append(ch if u >= err else rng.choice(list(ALPHA)))
    return a, "".join(b)


# ---------------------------------------------------------------- the pins
def pin_hand_traces(lib):
    bad = []
    for a, b, ma, mi, g, X, want in read_golden():
        got = oracle.extend(a, b, ma, mi, g, X, lib=lib)
        if got != want:
            bad.append((a, b, X, got, want))
    return bad


def pin_reading_vectors(lib):
    bad = []
    for a, b, ma, mi, g, X, want in read_vectors():
        got = oracle.extend(a, b, ma, mi, g, X, lib=lib)
        if got[:3] != want[:3] or (want[3] is not None and got[3] != want[3]):
            bad.append((a, b, X, got, want))
    return bad


def pin_worked_record(lib):
    keys = ("score", "left", "right", "seed", "a_begin", "a_end", "b_begin", "b_end", "cells_left", "cells_right")
    bad = []
    for A, B, (pa, pb, k, strand, X, ma, mi, g), want in read_records():
        r = oracle.record(A, B, pa, pb, k, strand, X, ma, mi, g, lib=lib)
        got = [r[key] for key in keys]
        if got != want:
            bad.append((A, B, strand, got, want))
    return bad


def pin_nw_at_infinite_x(lib, trials=1500, seed=1):
    """No pruning: X-drop result == NW table best (brute-force table) and
    cells == (m+1)(n+1)-1."""
    ref = oracle.load()
    rng = np.random.default_rng(seed)
    bad = []
    for _ in range(trials):
        a, b = rand_seq(rng, 0, 10), rand_seq(rng, 0, 10)
        ma, mi, g = WEIGHTS[int(rng.integers(len(WEIGHTS)))]
        got = oracle.extend(a, b, ma, mi, g, INF, lib=lib)
        want = oracle.nw_best(a, b, ma, mi, g, lib=ref)
        if got != want or got[3] != (len(a) + 1) * (len(b) + 1) - 1:
            bad.append((a, b, (ma, mi, g), got, want))
    return bad


def pin_identical_prefix(lib, trials=300, seed=2):
    rng = np.random.default_rng(seed)
    bad = []
    for _ in range(trials):
        a = rand_seq(rng, 0, 30)
        b = a + rand_seq(rng, 0, 6)
        ma, mi, g = WEIGHTS[int(rng.integers(len(WEIGHTS)))]
        for X in (0, 1, 2, 3, 5, 8):
            T, i, j, _ = oracle.extend(a, b, ma, mi, g, X, lib=lib)
            if (T, i, j) != (ma * len(a), len(a), len(a)):
                bad.append((a, b, X, (T, i, j)))
    return bad


def pin_invariants(lib, trials=600, seed=3):
    """bounds 0 <= T <= NW optimum, (a,b) symmetry of T and cells,
    invariance under complementing both sequences."""
    ref = oracle.load()
    rng = np.random.default_rng(seed)
    comp = str.maketrans("ACGT", "TGCA")
    bad = []
    for t in range(trials):
        a, b = related_pair(rng, 0, 40) if t % 2 else (rand_seq(rng, 0, 30), rand_seq(rng, 0, 30))
        ma, mi, g = WEIGHTS[int(rng.integers(len(WEIGHTS)))]
        X = int(rng.integers(0, 12))
        r = oracle.extend(a, b, ma, mi, g, X, lib=lib)
        full = oracle.nw_best(a, b, ma, mi, g, lib=ref)
        if not (0 <= r[0] <= full[0]):
            bad.append(("bounds", a, b, X, r, full))
        s = oracle.extend(b, a, ma, mi, g, X, lib=lib)
        if (s[0], s[3]) != (r[0], r[3]):
            bad.append(("symmetry", a, b, X, r, s))
        c = oracle.extend(a.translate(comp), b.translate(comp), ma, mi, g, X, lib=lib)
        if c != r:
            bad.append(("complement", a, b, X, r, c))
    return bad


def pin_suffix_independence(lib, trials=400, seed=4):
    """Every anti-diagonal up to the stop holds at least one candidate, so a
    run with cells < min(m, n) stopped before leaving the square
    min(m,n) x min(m,n): appending any bases to either sequence must leave
    the result unchanged."""
    rng = np.random.default_rng(seed)
    bad = []
    checked = 0
    for _ in range(trials):
        a, b = rand_seq(rng, 20, 60), rand_seq(rng, 20, 60)
        ma, mi, g = WEIGHTS[int(rng.integers(len(WEIGHTS)))]
        X = int(rng.integers(0, 4))
        r = oracle.extend(a, b, ma, mi, g, X, lib=lib)
        if r[3] >= min(len(a), len(b)):
            continue
        checked += 1
        r2 = oracle.extend(a + rand_seq(rng, 1, 30), b + rand_seq(rng, 1, 30), ma, mi, g, X, lib=lib)
        if r2 != r:
            bad.append(("suffix", a, b, X, r, r2))
    if checked < trials // 4:
        bad.append(("too few early stops", checked))
    return bad


def pin_dense_agrees(lib, trials=800, seed=5):
    """The live-range form agrees with the whole-table form on every output."""
    ref = oracle.load()
    rng = np.random.default_rng(seed)
    bad = []
    for t in range(trials):
        a, b = related_pair(rng, 0, 60) if t % 3 else (rand_seq(rng, 0, 40), rand_seq(rng, 0, 40))
        ma, mi, g = WEIGHTS[int(rng.integers(len(WEIGHTS)))]
        X = int(rng.integers(0, 25))
        r = oracle.extend(a, b, ma, mi, g, X, lib=lib)
        d = oracle.extend(a, b, ma, mi, g, X, dense=True, lib=ref)
        if r != d:
            bad.append((a, b, (ma, mi, g), X, r, d))
    return bad


ALL_PINS = [pin_hand_traces, pin_reading_vectors, pin_worked_record, pin_nw_at_infinite_x, pin_identical_prefix,
            pin_invariants, pin_suffix_independence, pin_dense_agrees]


# ---------------------------------------------------------------- tests
def test_golden_file_parses():
    rows = read_golden()
    assert len(rows) >= 9
    assert len(read_vectors()) == 18 and len(read_records()) == 2


def test_reading_vectors_show_non_monotone_score_in_x():
    # the stored example itself: T(X=2) = 12 > T(X=3) = 5 < T(X=4) = 16
    rows = [r for r in read_vectors() if len(r[0]) == 43]
    by_x = {X: want[0] for _, _, _, _, _, X, want in rows}
    assert by_x[2] > by_x[3] < by_x[4]


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin, oracle_lib):
    bad = pin(oracle_lib)
    assert not bad, f"{pin.__name__}: {len(bad)} failures, first {bad[0]}"


def _all_paths_best(a, b, ma, mi, g):
    """Enumerate every alignment path from (0,0) (steps: diagonal, down,
    right) to every cell; return (best, i, j) with ties to min i+j, min i."""
    best = (0, 0, 0)

    def rec(i, j, s):
        nonlocal best
        if (s > best[0]) or (s == best[0] and (i + j, i) < (best[1] + best[2], best[1])):
            best = (s, i, j)
        if i < len(a) and j < len(b):
            rec(i + 1, j + 1, s + (ma if a[i] == b[j] else mi))
        if i < len(a):
            rec(i + 1, j, s + g)
        if j < len(b):
            rec(i, j + 1, s + g)

    rec(0, 0, 0)
    return best


def test_nw_table_against_path_enumeration():
    """The NW prefix table used as reference is itself pinned by enumerating
    every path on tiny inputs (exhaustive over lengths <= 3, random up to 5)."""
    lib = oracle.load()
    cases = []
    for la in range(4):
        for lb in range(4):
            for a in itertools.product(ALPHA, repeat=la):
                for b in itertools.product(ALPHA, repeat=lb):
                    if (la + lb) <= 4 or (hash(a + b) % 7 == 0):
                        cases.append(("".join(a), "".join(b)))
    rng = np.random.default_rng(9)
    cases += [(rand_seq(rng, 0, 5), rand_seq(rng, 0, 5)) for _ in range(300)]
    for a, b in cases:
        for ma, mi, g in WEIGHTS[:3]:
            got = oracle.nw_best(a, b, ma, mi, g, lib=lib)[:3]
            want = _all_paths_best(a, b, ma, mi, g)
            assert got == want, (a, b, (ma, mi, g), got, want)


def test_no_prune_threshold():
    """X at least ma*min(m,n) + |g|*(m+n) never prunes: result == NW."""
    lib = oracle.load()
    rng = np.random.default_rng(6)
    for _ in range(200):
        a, b = related_pair(rng, 0, 50)
        ma, mi, g = WEIGHTS[int(rng.integers(len(WEIGHTS)))]
        xsafe = ma * min(len(a), len(b)) + (-g) * (len(a) + len(b)) + (-mi) * (len(a) + len(b))
        assert oracle.extend(a, b, ma, mi, g, xsafe, lib=lib) == oracle.nw_best(a, b, ma, mi, g, lib=lib)


def _revcomp(s):
    return s[::-1].translate(str.maketrans("ACGT", "TGCA"))


def test_record_strand_and_decomposition():
    lib = oracle.load()
    rng = np.random.default_rng(7)
    for t in range(300):
        A, B = related_pair(rng, 20, 200)
        if len(B) < 5:
            continue
        k = int(rng.integers(1, min(len(A), len(B), 20) + 1))
        pa = int(rng.integers(0, len(A) - k + 1))
        pb = int(rng.integers(0, len(B) - k + 1))
        X = int(rng.integers(0, 30))
        ma, mi, g = WEIGHTS[int(rng.integers(len(WEIGHTS)))]
        plus = oracle.record(A, B, pa, pb, k, 0, X, ma, mi, g, lib=lib)
        # B stored reverse-complemented, strand '-': same alignment
        minus = oracle.record(A, _revcomp(B), pa, len(B) - pb - k, k, 1, X, ma, mi, g, lib=lib)
        assert plus == minus
        assert plus["score"] == plus["left"] + plus["seed"] + plus["right"]
        L = oracle.extend(A[:pa][::-1], B[:pb][::-1], ma, mi, g, X, lib=lib)
        R = oracle.extend(A[pa + k:], B[pb + k:], ma, mi, g, X, lib=lib)
        assert (plus["left"], plus["right"]) == (L[0], R[0])
        assert (plus["a_begin"], plus["a_end"]) == (pa - L[1], pa + k + R[1])
        assert (plus["b_begin"], plus["b_end"]) == (pb - L[2], pb + k + R[2])
        assert plus["seed"] == sum(ma if A[pa + u] == B[pb + u] else mi for u in range(k))


def test_record_identical_reads_score_equals_length():
    lib = oracle.load()
    rng = np.random.default_rng(8)
    for _ in range(50):
        A = rand_seq(rng, 30, 300)
        k = int(rng.integers(1, 20))
        p = int(rng.integers(0, len(A) - k + 1))
        for X in (0, 1, 10, 50):
            r = oracle.record(A, A, p, p, k, 0, X, lib=lib)
            assert r["score"] == len(A) and (r["a_begin"], r["a_end"]) == (0, len(A))


def test_monotonicity_in_x_is_reported_not_asserted(capsys):
    """Score is not monotone in X under this reading (a larger X can let an
    early branch raise T and prune the path that would score more).  Count
    and report violations on related pairs."""
    lib = oracle.load()
    rng = np.random.default_rng(10)
    viol = steps = 0
    for _ in range(300):
        a, b = related_pair(rng, 20, 70)
        prev = None
        for X in range(0, 16):
            T = oracle.extend(a, b, 1, -1, -1, X, lib=lib)[0]
            if prev is not None:
                steps += 1
                viol += T < prev
            prev = T
    print(f"monotonicity: {viol} decreases in {steps} X-steps")


@pytest.fixture(scope="module")
def mutants():
    d = tempfile.mkdtemp(prefix="oxmut")
    libs = {}
    for m in range(1, 8):
        path = os.path.join(d, f"liboracle_mut{m}.so")
        oracle.build(path, mutation=m)
        libs[m] = oracle.load(path)
        assert libs[m].ox_mutation() == m
    return libs


@pytest.mark.parametrize("m", range(1, 8))
def test_each_planted_mistake_is_caught(mutants, m):
    lib = mutants[m]
    caught = [p.__name__ for p in ALL_PINS if p(lib)]
    assert caught, f"mutation {m} passed every pin"
