"""Conflict map of a block-row distribution (Section 3, Fig. 2) on the GPU,
bit-exact against the oracle on the oracle's own reordering and split."""
import numpy as np
import pytest

import oracle
import paper_2407_17651_amd as p3
import synth

pytestmark = pytest.mark.gpu


def oracle_map(L, nb, bounds=None, w_in=-1, t_out=-1, permute=True):
    B = oracle.permute(L, oracle.rcm(L)) if permute else L
    part, _, _ = oracle.split(B, w_in, t_out)
    return oracle.conflict_map(B, part, nb, bounds)


@pytest.mark.parametrize("name,maker", [
    ("rgg_20000", lambda: synth.rgg2d(20000, 12.0, 8)),
    ("grid3d_24", lambda: synth.grid3d(24, 3, "normal")),
    ("chung_lu_8000", lambda: synth.chung_lu(8000, 10.0, 2.5, 5)),
    ("pieces", lambda: synth.from_edges(40, [(i, i + 1) for i in range(0, 38, 3)], relabel=True, seed=3)),
])
@pytest.mark.parametrize("nb", [1, 2, 8, 61, 512])
def test_balanced_blocks(name, maker, nb):
    L = maker()
    print(f"[gpu] conflict map {name} nb={nb}", flush=True)
    M = p3.Matrix(L).reorder()
    assert np.array_equal(M.conflict_map(nb), oracle_map(L, nb))


@pytest.mark.parametrize("params", [dict(w_in=3), dict(w_in=0, t_out=0), dict(t_out=20)])
def test_parts_follow_the_split(params):
    L = synth.rgg2d(15000, 10.0, 2)
    M = p3.Matrix(L).reorder(**params)
    assert np.array_equal(M.conflict_map(16), oracle_map(L, 16, None, params.get("w_in", -1),
                                                         params.get("t_out", -1)))


def test_tiles_as_blocks_and_random_bounds():
    L = synth.rgg2d(30000, 16.0, 4)
    M = p3.Matrix(L).reorder(tile_rows=256)
    T = 256
    nt = -(-L.n // T)
    tiles = np.minimum(np.arange(nt + 1) * T, L.n)
    assert np.array_equal(M.conflict_map(nt, tiles), oracle_map(L, nt, tiles))
    rng = np.random.default_rng(3)
    for nb in (3, 17, 200):
        b = np.concatenate([[0], np.sort(rng.integers(0, L.n + 1, nb - 1)), [L.n]])
        assert np.array_equal(M.conflict_map(nb, b), oracle_map(L, nb, b))


def test_one_row_per_block():
    L = synth.grid2d(40, 6)
    M = p3.Matrix(L).reorder()
    b = np.arange(L.n + 1)
    assert np.array_equal(M.conflict_map(L.n, b), oracle_map(L, L.n, b))


def test_given_numbering():
    L = synth.rgg2d(5000, 8.0, 9)
    M = p3.Matrix(L).reorder(permute=0)
    assert np.array_equal(M.conflict_map(8), oracle_map(L, 8, permute=False))


def test_empty_and_errors():
    M0 = p3.Matrix(synth.from_edges(0, [], seed=0)).reorder()
    m0 = M0.conflict_map(3)
    assert m0.shape == (3, 11) and not m0.any()
    L = synth.grid2d(10, 1)
    M = p3.Matrix(L)
    with pytest.raises(p3.Pars3Error) as e:
        M.conflict_map(2)
    assert e.value.status == p3.ESTATE
    M.reorder()
    for nb, b in ((0, None), (2, [0, 3, 99]), (2, [1, 3, 100]), (3, [0, 50, 40, 100])):
        with pytest.raises(p3.Pars3Error) as e:
            M.conflict_map(nb, b)
        assert e.value.status == p3.EINVAL


def test_workload1_full_size():
    """The 3D 128^3 matrix: 8 equal row blocks (one per GPU of a node) and
    its 256-row tiles."""
    L = synth.workload(1)
    print("[gpu] conflict map workload1", flush=True)
    M = p3.Matrix(L).reorder(tile_rows=256)
    B = oracle.permute(L, oracle.rcm(L))
    part, _, _ = oracle.split(B)
    assert np.array_equal(M.conflict_map(8), oracle.conflict_map(B, part, 8))
    nt = -(-L.n // 256)
    tiles = np.minimum(np.arange(nt + 1) * 256, L.n)
    assert np.array_equal(M.conflict_map(nt, tiles), oracle.conflict_map(B, part, nt, tiles))


@pytest.mark.parametrize("name,maker", [
    ("rgg_20000", lambda: synth.rgg2d(20000, 12.0, 8)),
    ("grid3d_24", lambda: synth.grid3d(24, 3, "normal")),
    ("chung_lu_8000", lambda: synth.chung_lu(8000, 10.0, 2.5, 5)),
    ("path_80", lambda: synth.from_edges(80, [(i, i + 1) for i in range(79)], relabel=True, seed=2)),
    ("no_edges", lambda: synth.from_edges(50, [])),
])
@pytest.mark.parametrize("nb", [1, 8, 37])
def test_conflict_features_bit_exact(name, maker, nb):
    """The selector's conflict features equal the oracle's on the oracle's
    reordering, bit for bit (ratios of equal integer counts)."""
    L = maker()
    print(f"[gpu] conflict features {name} nb={nb}", flush=True)
    M = p3.Matrix(L).reorder()
    want = oracle.conflict_features(oracle.permute(L, oracle.rcm(L)), nb)
    assert np.array_equal(M.conflict_features(nb), want)


def test_conflict_features_errors():
    L = synth.grid2d(10, 1)
    M = p3.Matrix(L)
    with pytest.raises(p3.Pars3Error) as e:
        M.conflict_features(8)
    assert e.value.status == p3.ESTATE
    M.reorder()
    with pytest.raises(p3.Pars3Error) as e:
        M.conflict_features(0)
    assert e.value.status == p3.EINVAL
