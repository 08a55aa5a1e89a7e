"""Pins of the oracle's conflict map (Section 3, Fig. 2): block-row
ownership, safe (R1) and conflicting (R2) entries, halo columns and partner
blocks, checked against brute force with Python sets, the two extreme
distributions, the block-0 property and the band bound."""
import numpy as np
import pytest

import oracle
import synth


def brute(L, part, bounds):
    """The same counts from their definitions, with Python sets."""
    nb = len(bounds) - 1
    owner = {}
    for p in range(nb):
        for i in range(bounds[p], bounds[p + 1]):
            owner[i] = p
    rows_of = np.repeat(np.arange(L.n), np.diff(L.rowptr))
    out = []
    for p in range(nb):
        lo, hi = bounds[p], bounds[p + 1]
        safe, conf = [0, 0, 0], [0, 0, 0]
        cols = set()
        for e in np.flatnonzero((rows_of >= lo) & (rows_of < hi)):
            j = int(L.col[e])
            if j >= lo:
                safe[part[e]] += 1
            else:
                conf[part[e]] += 1
                cols.add(j)
        out.append([lo, hi - lo, *safe, *conf, min(cols) if cols else lo, len({owner[j] for j in cols}), len(cols)])
    return np.array(out, np.int64).reshape(nb, 11)


def random_bounds(n, nb, rng):
    cuts = np.sort(rng.integers(0, n + 1, nb - 1))
    return np.concatenate([[0], cuts, [n]]).astype(np.int64)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force(seed):
    rng = np.random.default_rng(seed)
    L = synth.rgg2d(300, 6.0, seed)
    B = oracle.permute(L, oracle.rcm(L))
    part, _, _ = oracle.split(B, int(rng.integers(0, 3)), -1)
    nb = int(rng.integers(1, 12))
    bounds = random_bounds(B.n, nb, rng)  # empty blocks included
    assert np.array_equal(oracle.conflict_map(B, part, nb, bounds), brute(B, part, bounds))
    balanced = (np.arange(nb + 1) * B.n) // nb
    assert np.array_equal(oracle.conflict_map(B, part, nb), brute(B, part, balanced))


def test_single_block_has_no_conflicts():
    L = synth.grid2d(12, 2)
    part, cnt, _ = oracle.split(L)
    m = oracle.conflict_map(L, part, 1)
    assert m[0, 1] == L.n and m[0, 2:5].tolist() == cnt.tolist() and not m[0, 5:8].any()
    assert m[0, 8] == 0 and m[0, 9] == 0 and m[0, 10] == 0


def test_one_row_per_block_makes_every_entry_conflicting():
    L = synth.rgg2d(200, 5.0, 3)
    part, cnt, _ = oracle.split(L)
    m = oracle.conflict_map(L, part, L.n, np.arange(L.n + 1))
    lens = np.diff(L.rowptr)
    assert not m[:, 2:5].any()
    assert m[:, 5:8].sum(0).tolist() == cnt.tolist()
    assert np.array_equal(m[:, 10], lens) and np.array_equal(m[:, 9], lens)
    first = np.array([L.col[L.rowptr[i]] if lens[i] else i for i in range(L.n)])
    assert np.array_equal(m[:, 8], first)


@pytest.mark.parametrize("nb", [2, 7, 64])
def test_block_zero_safe_and_totals(nb):
    L = synth.chung_lu(2000, 8.0, 2.5, 4)
    part, cnt, _ = oracle.split(L, 1, -1)
    m = oracle.conflict_map(L, part, nb)
    assert not m[0, 5:8].any() and m[0, 9] == 0 and m[0, 10] == 0
    assert (m[:, 2:5] + m[:, 5:8]).sum(0).tolist() == cnt.tolist()
    assert m[:, 1].sum() == L.n
    assert np.all(m[:, 10] <= m[:, 5:8].sum(1)) and np.all(m[:, 9] <= np.arange(nb))


def test_band_bound():
    """Blocks longer than the bandwidth beta: every conflicting column lies in
    the previous block and within beta rows of the boundary."""
    L = synth.grid2d(60, 5)
    B = oracle.permute(L, oracle.rcm(L))
    part, _, (_, _, beta) = oracle.split(B)
    nb = B.n // (2 * beta)
    m = oracle.conflict_map(B, part, nb)
    assert np.all(m[1:, 9] == 1)
    assert np.all(m[:, 0] - m[:, 8] <= beta) and np.all(m[:, 10] <= beta)


def test_bad_bounds():
    L = synth.grid2d(5, 1)
    part, _, _ = oracle.split(L)
    for nb, b in ((0, None), (2, [0, 3, 24]), (2, [1, 3, 25]), (3, [0, 5, 4, 25])):
        with pytest.raises(ValueError):
            oracle.conflict_map(L, part, nb, b)


# ---- conflict features over balanced blocks (the selector's inputs 33-35)
def brute_features(L, nb):
    """The three ratios from their definitions, with Python sets."""
    n = L.n
    bounds = [(p * n) // nb for p in range(nb + 1)]
    rows_of = np.repeat(np.arange(n), np.diff(L.rowptr))
    conf, halo, reach = 0, 0.0, 0.0
    for p in range(nb):
        lo, hi = bounds[p], bounds[p + 1]
        rows = max(hi - lo, 1)
        cols = [int(L.col[e]) for e in np.flatnonzero((rows_of >= lo) & (rows_of < hi)) if L.col[e] < lo]
        conf += len(cols)
        halo = max(halo, len(set(cols)) / rows)
        reach = max(reach, (lo - min(cols)) / rows if cols else 0.0)
    return np.array([conf / L.nnz if L.nnz else 0.0, halo, reach])


def test_features_path_graph_closed_form():
    """A path of 80 nodes in 8 blocks of 10 rows: each block but the first
    has one conflicting entry, the edge into the block before it, with one
    halo column one row back."""
    L = synth.from_edges(80, [(i, i + 1) for i in range(79)])
    f = oracle.conflict_features(L, 8)
    assert f[0] == 7 / 79 and f[1] == 1 / 10 and f[2] == 1 / 10


def test_features_complete_graph_closed_form():
    """K_16 in 8 blocks of 2 rows: block p has 4p conflicting entries over
    2p halo columns reaching back to column 0, so the largest halo and reach
    per row are both 14 / 2 = 7 and 112 of the 120 entries conflict."""
    L = synth.from_edges(16, [(i, j) for i in range(16) for j in range(i + 1, 16)])
    f = oracle.conflict_features(L, 8)
    assert f[0] == 112 / 120 and f[1] == 7.0 and f[2] == 7.0


def test_features_empty_and_single_block():
    L = synth.from_edges(40, [])
    assert np.array_equal(oracle.conflict_features(L, 8), np.zeros(3))
    G = synth.grid2d(12, 3)
    assert np.array_equal(oracle.conflict_features(G, 1), np.zeros(3))


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("nb", [3, 8])
def test_features_brute_force(seed, nb):
    for L in (synth.rgg2d(600, 8.0, seed), synth.chung_lu(500, 6.0, 2.5, seed), synth.grid2d(20, seed)):
        assert np.allclose(oracle.conflict_features(L, nb), brute_features(L, nb), rtol=0, atol=0)


def test_features_bad_block_count():
    with pytest.raises(ValueError):
        oracle.conflict_features(synth.grid2d(5, 1), 0)
