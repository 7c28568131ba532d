"""Sparsity statistics used by NeutronSparse (TEST INFRASTRUCTURE ONLY).

* Table 2 (Sec. 8.1): AvgL = NNZ / rows; Dens = NNZ / (rows * cols), printed
  scaled by 1e-3; Skew = fraction of NNZ held by the top 10% of rows ranked by
  row NNZ; "Empty" = fraction of empty 16x16 tiles.
* Table 1 (Sec. 3.2): tile a matrix into t x t tiles, call a tile active if it
  holds at least one nonzero, and report the fraction of zeros over all
  active tiles.
* Sec. 8.4 density of the matrix-engine workload: nnz / (tile area) over the
  tiles handed to it.
"""
from __future__ import annotations

import math

import numpy as np


def avg_len(nnz, rows):
    return nnz / rows


def density(nnz, rows, cols):
    return nnz / (rows * cols)


def row_skew(rowptr, top_frac=0.10):
    """Fraction of NNZ in the top ``top_frac`` of rows by row length
    (ceil of the row count; ties among equal lengths do not matter)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    lens = np.sort(rowptr[1:] - rowptr[:-1])[::-1]
    top = int(math.ceil(top_frac * lens.size))
    total = int(lens.sum())
    return float(lens[:top].sum()) / total if total else 0.0


def _tile_counts(rowptr, colidx, m, k, t):
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), rowptr[1:] - rowptr[:-1])
    nbc = (k + t - 1) // t
    # duplicates of one (row, col) are one nonzero position
    pos = np.unique(rows * k + colidx)
    key = (pos // k // t) * nbc + (pos % k) // t
    uniq, cnt = np.unique(key, return_counts=True)
    return uniq, cnt, (m + t - 1) // t, nbc


def active_tile_zero_fraction(rowptr, colidx, m, k, t):
    """Table 1 measure for tile size t.  Edge tiles count their full t x t
    area, as the kernel processes whole tiles."""
    uniq, cnt, _, _ = _tile_counts(rowptr, colidx, m, k, t)
    if uniq.size == 0:
        return 0.0
    area = uniq.size * t * t
    return 1.0 - cnt.sum() / area


def empty_tile_fraction(rowptr, colidx, m, k, t=16):
    """Fraction of all t x t grid tiles that hold no nonzero."""
    uniq, _, nbr, nbc = _tile_counts(rowptr, colidx, m, k, t)
    return 1.0 - uniq.size / (nbr * nbc)
