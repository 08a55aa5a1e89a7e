"""Pins of the oracle's LDS bank-pass count (the layout's bank model: aligned
runs of 32 entries per tile-pair block, passes = most frequent row offset mod
32 + most frequent column offset mod 32), by closed forms on hand-built
matrices given in their final numbering."""
from types import SimpleNamespace

import numpy as np

import oracle


def lower(n, entries):
    entries = sorted(entries)
    rp = np.zeros(n + 1, np.int32)
    for i, _ in entries:
        rp[i + 1] += 1
    return SimpleNamespace(n=n, rowptr=np.cumsum(rp).astype(np.int32), col=np.array([j for _, j in entries], np.int32),
                           val=np.ones(len(entries)), nnz=len(entries))


def test_path_graph():
    """Entries (i, i-1), n = 256 k, 256-row tiles: all outer (beta = 1, so
    t_out = 0).  Tile t holds one block (t, t) with the 255 entries of rows
    1..255 on one diagonal (8 runs of consecutive rows, 1 + 1 passes each)
    and, for t > 0, a block (t, t-1) with one entry (1 run, 2 passes)."""
    for k in (1, 3):
        n = 256 * k
        runs, passes = oracle.lds_passes_sorted(lower(n, [(i, i - 1) for i in range(1, n)]))
        assert runs == 8 * k + (k - 1)
        assert passes == 2 * runs


def test_one_column():
    """Entries (r, 0) for r = 33..63 in one 64-row tile: distinct row classes
    1..31, one column class.  With everything in the middle part one run of 31
    entries: 1 + 31 passes.  With the default split (beta = 63, t_out = 60)
    rows 61..63 form an outer block of their own: 1 + 28 and 1 + 3 passes."""
    L = lower(64, [(r, 0) for r in range(33, 64)])
    assert oracle.lds_passes_sorted(L, 64, 0, 1000) == (1, 32)
    assert oracle.lds_passes_sorted(L, 64) == (2, 33)


def test_two_diagonals_in_diagonal_order():
    """Entries (i, i-1), i = 1..63, and (i, i-2), i = 2..63, one 64-row tile,
    all outer.  Sorted by block diagonal (63 - 1 for d = 2 comes first) then
    row: run 0 = rows 2..33 of d = 2 (distinct classes: 2 passes); run 1 =
    rows 34..63 of d = 2 and rows 1, 2 of d = 1 (row class 2 and column
    classes 0 and 1 twice: 4 passes); runs 2 and 3 = rows 3..34 and 35..63 of
    d = 1 (2 passes each).  A row-major order would pair the two entries of
    every row instead."""
    L = lower(64, [(i, i - 1) for i in range(1, 64)] + [(i, i - 2) for i in range(2, 64)])
    assert oracle.lds_passes_sorted(L, 64) == (4, 10)


def test_inner_band_is_not_counted():
    """With w_in = 2 both diagonals of the previous matrix are inner."""
    L = lower(64, [(i, i - 1) for i in range(1, 64)] + [(i, i - 2) for i in range(2, 64)])
    assert oracle.lds_passes_sorted(L, 64, 2, 10) == (0, 0)
    assert oracle.lds_passes_sorted(L, 64, 1, 10) == (2, 4)
