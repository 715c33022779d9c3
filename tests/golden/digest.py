"""Canonical digests of per-record X-drop results (test infrastructure).

A block of records is reduced to one SHA-256 over little-endian int64 rows
(score, left score, right score, seed score, a_begin, a_end, b_begin, b_end,
left + right candidate cells).  The stored digests of the full-size workloads
are written from the CPU oracle by ``make_oracle_digests.py``; the GPU tests
compute the same digest of the library's results and compare block by block.
This module holds no alignment arithmetic: it only lays out and hashes rows.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

BLOCK = 10_000
HERE = os.path.dirname(os.path.abspath(__file__))
COLUMNS = ("score", "left", "right", "seed", "a_begin", "a_end", "b_begin", "b_end", "cells")


def rows(score, left, right, seed, a_begin, a_end, b_begin, b_end, cells) -> np.ndarray:
    """(n, 9) little-endian int64 rows in COLUMNS order."""
    cols = [np.asarray(c).astype("<i8") for c in (score, left, right, seed, a_begin, a_end, b_begin, b_end, cells)]
    return np.ascontiguousarray(np.stack(cols, axis=1))


def rows_from_oracle(ref) -> np.ndarray:
    return rows(ref["score"], ref["left"], ref["right"], ref["seed"], ref["a_begin"], ref["a_end"],
                ref["b_begin"], ref["b_end"], ref["cells_left"].astype(np.int64) + ref["cells_right"].astype(np.int64))


def rows_from_results(res, cells) -> np.ndarray:
    """Rows of library results (xdrop_result array) and per-record cells."""
    return rows(res["score"], res["left_score"], res["right_score"], res["seed_score"], res["a_begin"],
                res["a_end"], res["b_begin"], res["b_end"], np.asarray(cells).astype(np.int64))


def block_digest(r: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(r, dtype="<i8").tobytes()).hexdigest()


def path_for(name: str) -> str:
    return os.path.join(HERE, f"oracle_digests_{name}.txt")


def read_digests(name: str):
    """{block start: (count, cells, sha256)} and the header fields of a stored digest file."""
    blocks, head = {}, {}
    with open(path_for(name)) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                if ":" in line:
                    k, v = line[1:].split(":", 1)
                    head[k.strip()] = v.strip()
                continue
            start, count, cells, sha = line.split()
            blocks[int(start)] = (int(count), int(cells), sha)
    return blocks, head
