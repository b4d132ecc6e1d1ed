"""Small test-side builders: hand-shaped patterns and dense expansions.

These feed both sides of a comparison; they hold no solver arithmetic.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np


def dense_pattern(n):
    rowptr = np.arange(0, n * n + 1, n, dtype=np.int32)
    colidx = np.tile(np.arange(n, dtype=np.int32), n)
    return rowptr, colidx


def chain_pattern(n):
    """Block tridiagonal (1D chain): ILU0 drops no fill on it."""
    rows, cols = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
    rowptr = np.zeros(n + 1, np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return rowptr, np.asarray(cols, np.int32)


def pattern_from_pairs(n, pairs, symmetric=True):
    s = set((i, i) for i in range(n))
    for i, j in pairs:
        s.add((i, j))
        if symmetric:
            s.add((j, i))
    ent = sorted(s)
    rowptr = np.zeros(n + 1, np.int32)
    np.cumsum(np.bincount([i for i, _ in ent], minlength=n), out=rowptr[1:])
    return rowptr, np.asarray([j for _, j in ent], np.int32)


def random_values(rowptr, colidx, seed=0, diag_boost=4.0):
    """Non-symmetric blocks with a dominant diagonal (so no zero pivots)."""
    rng = np.random.default_rng(seed)
    n = len(rowptr) - 1
    vals = rng.uniform(-1.0, 1.0, size=(len(colidx), 3, 3))
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            if colidx[p] == i:
                vals[p] += diag_boost * (rowptr[i + 1] - rowptr[i]) * np.eye(3)
    return vals


def to_dense(rowptr, colidx, vals):
    n = len(rowptr) - 1
    a = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            j = colidx[p]
            a[3 * i:3 * i + 3, 3 * j:3 * j + 3] = vals[p]
    return a


def split_lu(rowptr, colidx, lu):
    """Expand in-place factors into dense unit-lower L and upper U."""
    n = len(rowptr) - 1
    L = np.eye(3 * n)
    U = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            j = colidx[p]
            blk = slice(3 * i, 3 * i + 3), slice(3 * j, 3 * j + 3)
            if j < i:
                L[blk] = lu[p]
            else:
                U[blk] = lu[p]
    return L, U


def pattern_set(rowptr, colidx):
    n = len(rowptr) - 1
    return {(i, int(colidx[p])) for i in range(n) for p in range(rowptr[i], rowptr[i + 1])}


def read_golden(path):
    """Parse a ``NAME = a b c ; d e f ; ...`` fixture of exact rationals."""
    out = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = (t.strip() for t in line.split("=", 1))
            rows = [[float(Fraction(t)) for t in r.split()] for r in val.split(";")]
            out[key] = np.asarray(rows if len(rows) > 1 else rows[0])
    return out
