#!/usr/bin/env python3
"""Write the stored oracle digests of the full-size workloads.

For each named workload (c1, c2, c4, c4b at their full sizes) the seeded
generator builds the records, the CPU oracle computes every record, and one
line per block of 10,000 records is written:

    <first record> <records> <oracle cells of the block> <sha256 of the rows>

(rows as in digest.py).  Calls only the generator and ``oracle/``; nothing of
the HIP path is involved.  Blocks already present in the output are kept, so
an interrupted run resumes where it stopped.

    python tests/golden/make_oracle_digests.py c2 c4b c4 [--threads N]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import digest  # noqa: E402
import oracle  # noqa: E402
from paper_2309_07270_amd import workload as W  # noqa: E402


def run(name: str, threads: int) -> None:
    t0 = time.time()
    wl = W.make_workload(name)
    n = len(wl.records)
    print(f"{name}: {n} records generated in {time.time() - t0:.1f} s", flush=True)
    path = digest.path_for(name)
    done = {}
    if os.path.exists(path):
        done, _ = digest.read_digests(name)
    header = (f"# workload: {name} (seed {wl.meta['seed']}), {n} records, {wl.meta['reads']} reads\n"
              f"# block: {digest.BLOCK}\n"
              f"# columns: {' '.join(digest.COLUMNS)} (little-endian int64 per record)\n"
              f"# written by: python tests/golden/make_oracle_digests.py {name}\n"
              f"# line: first_record records oracle_cells sha256\n")
    lines = {s: f"{s} {c} {cl} {h}\n" for s, (c, cl, h) in done.items()}
    lib = oracle.load()
    for s in range(0, n, digest.BLOCK):
        if s in lines:
            continue
        t1 = time.time()
        recs = wl.records[s:s + digest.BLOCK]
        ref, _ = oracle.batch(wl.store.codes, wl.store.off, wl.store.length, recs, nthreads=threads, lib=lib)
        r = digest.rows_from_oracle(ref)
        lines[s] = f"{s} {len(recs)} {int(r[:, 8].sum())} {digest.block_digest(r)}\n"
        with open(path + ".tmp", "w") as f:
            f.write(header)
            for k in sorted(lines):
                f.write(lines[k])
        os.replace(path + ".tmp", path)
        print(f"{name}: block {s // digest.BLOCK + 1}/{(n + digest.BLOCK - 1) // digest.BLOCK} "
              f"{int(r[:, 8].sum())} cells in {time.time() - t1:.1f} s", flush=True)
    print(f"{name}: done in {time.time() - t0:.1f} s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for name in a.names:
        run(name, a.threads)


if __name__ == "__main__":
    main()
