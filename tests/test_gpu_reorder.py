"""GPU reverse Cuthill-McKee, sign-fixing permutation, three-way split and the
precision conversion against the oracle: bit-exact (integer and byte work)."""
import numpy as np
import pytest

import oracle
import paper_2407_17651_amd as p3
import synth

pytestmark = pytest.mark.gpu

GRAPHS = {
    "grid2d_12": lambda: synth.grid2d(12, 5),
    "grid3d_6": lambda: synth.grid3d(6, 6, "normal"),
    "rgg_2000": lambda: synth.rgg2d(2000, 8.0, 7),
    "chung_lu_3000": lambda: synth.chung_lu(3000, 6.0, 2.5, 8),
    "pieces": lambda: synth.from_edges(12, [(0, 1), (2, 3), (3, 4), (7, 9), (9, 11), (11, 7)], relabel=True, seed=3),
    "no_edges": lambda: synth.from_edges(5, [], seed=1),
    "single": lambda: synth.from_edges(1, [], seed=1),
    "pair": lambda: synth.from_edges(2, [(0, 1)], seed=1),
    "star": lambda: synth.from_edges(7, [(0, i) for i in range(1, 7)], seed=2),
    "grid3x3": lambda: synth.from_edges(9, [(0, 1), (1, 2), (3, 4), (4, 5), (6, 7), (7, 8), (0, 3), (3, 6), (1, 4),
                                            (4, 7), (2, 5), (5, 8)], seed=0),
    "workload0": lambda: synth.workload(0),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_rcm_and_permutation_bit_exact(name):
    L = GRAPHS[name]()
    print(f"[gpu] reorder {name} n={L.n} nnz={L.nnz}", flush=True)
    M = p3.Matrix(L).reorder()
    perm_o = oracle.rcm(L)
    assert np.array_equal(M.perm(), perm_o)
    B = oracle.permute(L, perm_o)
    rp, col, val, part = M.permuted_lower()
    assert np.array_equal(rp, B.rowptr)
    assert np.array_equal(col, B.col)
    assert np.array_equal(val.view(np.uint64), B.val.view(np.uint64))
    po, cnt, (w, t, beta) = oracle.split(B)
    assert np.array_equal(part, po)
    info = M.info()
    assert (info["beta"], info["w_in"], info["t_out"]) == (beta, w, t)
    assert [info["nnz_inner"], info["nnz_middle"], info["nnz_outer"]] == cnt.tolist()
    assert info["n_tiles"] == (L.n + 255) // 256
    assert (info["n_blocks"] > 0) == (cnt[1] + cnt[2] > 0)


def test_random_small_graphs_bit_exact():
    rng = np.random.default_rng(123)
    for trial in range(60):
        n = int(rng.integers(1, 200))
        dens = float(rng.uniform(0.0, 0.08))
        m = int(dens * n * (n - 1) / 2)
        pairs = set()
        while len(pairs) < m:
            a, b = rng.integers(0, n, 2)
            if a != b:
                pairs.add((int(max(a, b)), int(min(a, b))))
        L = synth.from_edges(n, sorted(pairs), seed=trial, relabel=True)
        print(f"[gpu] random graph trial={trial} n={n} nnz={L.nnz}", flush=True)
        M = p3.Matrix(L).reorder()
        assert np.array_equal(M.perm(), oracle.rcm(L)), trial


@pytest.mark.parametrize("w_in,t_out", [(0, -1), (2, -1), (3, 8), (0, 0), (1, 10 ** 6)])
def test_split_parameters(w_in, t_out):
    L = synth.rgg2d(5000, 10.0, 4)
    print(f"[gpu] split w_in={w_in} t_out={t_out}", flush=True)
    M = p3.Matrix(L).reorder(w_in=w_in, t_out=t_out)
    B = oracle.permute(L, oracle.rcm(L))
    po, cnt, (w, t, beta) = oracle.split(B, w_in, t_out)
    _, _, _, part = M.permuted_lower()
    assert np.array_equal(part, po)
    info = M.info()
    assert (info["w_in"], info["t_out"]) == (w, t)


def test_split_rejects_inverted_bounds():
    M = p3.Matrix(synth.grid2d(6, 1))
    with pytest.raises(p3.Pars3Error) as e:
        M.reorder(w_in=5, t_out=2)
    assert e.value.status == p3.EINVAL


@pytest.mark.parametrize("dtype", [p3.F64, p3.F32, p3.BF16])
def test_stored_values_bit_exact(dtype):
    L = synth.rgg2d(4000, 12.0, 9, "normal")
    print(f"[gpu] stored values dtype={dtype}", flush=True)
    M = p3.Matrix(L).reorder(value_dtype=dtype, w_in=2)
    B = oracle.permute(L, oracle.rcm(L))
    got = M.values(dtype)
    if dtype == p3.F64:
        assert np.array_equal(got.view(np.uint64), B.val.view(np.uint64))
    elif dtype == p3.F32:
        assert np.array_equal(got.view(np.uint32), oracle.round_f32(B.val).view(np.uint32))
    else:
        assert np.array_equal(got, oracle.round_bf16(oracle.round_f32(B.val)))


def test_identity_order_keeps_input():
    L = synth.grid2d(9, 3)
    M = p3.Matrix(L).reorder(permute=0)
    assert np.array_equal(M.perm(), np.arange(L.n))
    rp, col, val, _ = M.permuted_lower()
    assert np.array_equal(rp, L.rowptr) and np.array_equal(col, L.col) and np.array_equal(val, L.val)


def test_reorder_workload1_bit_exact():
    """The full 3D 128^3 workload: permutation, permuted matrix and split."""
    L = synth.workload(1)
    print(f"[gpu] reorder workload1 n={L.n}", flush=True)
    M = p3.Matrix(L).reorder()
    perm_o = oracle.rcm(L)
    assert np.array_equal(M.perm(), perm_o)
    B = oracle.permute(L, perm_o)
    rp, col, val, part = M.permuted_lower()
    assert np.array_equal(rp, B.rowptr) and np.array_equal(col, B.col)
    assert np.array_equal(val, B.val)
    po, cnt, (w, t, beta) = oracle.split(B)
    assert np.array_equal(part, po)
    assert M.info()["beta"] == beta
