"""Pins of the oracle's LDS bank-pass count (the layout's bank model: aligned
runs of 16 entries per tile-pair block, one quarter of a wavefront's add;
passes = most frequent row offset mod 32 + most frequent column offset mod
32), by closed forms on hand-built matrices given in their final numbering."""
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
    1..255 on one diagonal (16 runs of consecutive rows, 1 + 1 passes each)
    and, for t > 0, a block (t, t-1) with one entry (1 run, 2 passes)."""
    for k in (1, 3):
        n = 256 * k
        runs, passes = oracle.lds_passes_sorted(lower(n, [(i, i - 1) for i in range(1, n)]))
        assert runs == 16 * k + (k - 1)
        assert passes == 2 * runs


def test_one_column():
    """Entries (r, 0) for r = 33..63 in one 64-row tile: distinct row classes
    1..31, one column class.  With everything in the middle part: runs of 16
    and 15 entries, 1 + 16 and 1 + 15 passes.  With the default split (beta =
    63, t_out = 60) rows 61..63 form an outer block of their own: the middle
    block's runs of 16 and 12 entries take 17 and 13 passes, the outer one 4."""
    L = lower(64, [(r, 0) for r in range(33, 64)])
    assert oracle.lds_passes_sorted(L, 64, 0, 1000) == (2, 33)
    assert oracle.lds_passes_sorted(L, 64) == (3, 34)


def test_runs_of_32_count_halves():
    """The same matrix with runs of 32 (one run of 31 entries: 1 + 31)."""
    L = lower(64, [(r, 0) for r in range(33, 64)])
    assert oracle.lds_passes_sorted(L, 64, 0, 1000, run=32) == (1, 32)


def test_diagonal_order_keeps_runs_conflict_free():
    """Entries (i, i-1), i = 1..63, and (i, i-33), i = 33..63, one 64-row
    tile, all outer.  Sorted by block diagonal, the 31 entries of d = 33
    (block diagonal 31) come first, then the 63 of d = 1 (block diagonal 63):
    runs of 16 consecutive rows of one diagonal, or the tail of d = 33 (rows
    49..63, columns 16..30) with the first entry of d = 1 (row 1, column 0),
    all with distinct classes: 6 runs at 2 passes.  A row-major order would
    put the two entries of rows 33..63 next to each other (2 passes per side
    in those runs)."""
    L = lower(64, [(i, i - 1) for i in range(1, 64)] + [(i, i - 33) for i in range(33, 64)])
    assert oracle.lds_passes_sorted(L, 64) == (6, 12)


def test_inner_band_is_not_counted():
    """With w_in = 2 both diagonals of the next matrix are inner; with w_in = 1
    only d = 2 is left: 62 consecutive rows, 4 runs at 2 passes."""
    L = lower(64, [(i, i - 1) for i in range(1, 64)] + [(i, i - 2) for i in range(2, 64)])
    assert oracle.lds_passes_sorted(L, 64, 2, 10) == (0, 0)
    assert oracle.lds_passes_sorted(L, 64, 1, 10) == (4, 8)


def test_rows_sharing_a_class_collide():
    """Entries (i, 0) for i in {1, 33} and (i, 1) for i in {2, 34}, one
    64-row tile, everything middle: block diagonals 63, 31, 63, 31 for the
    entries (1,0), (33,0), (2,1), (34,1); sorted: (33,0), (34,1) (diagonal
    31), then (1,0), (2,1) (diagonal 63).  One run: row classes 1, 2, 1, 2
    (2 passes), column classes 0, 1, 0, 1 (2 passes)."""
    L = lower(64, [(1, 0), (33, 0), (2, 1), (34, 1)])
    assert oracle.lds_passes_sorted(L, 64, 0, 1000) == (1, 4)
