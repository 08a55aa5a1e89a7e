"""Pins of the oracle's sign-fixing permutation and three-way split."""
import numpy as np
import pytest

import oracle
import synth


def dense_S(L):
    S = np.zeros((L.n, L.n))
    rows = np.repeat(np.arange(L.n), np.diff(L.rowptr))
    S[rows, L.col] = L.val
    S[L.col, rows] = -np.asarray(L.val)
    return S


@pytest.mark.parametrize("maker", [
    lambda: synth.grid2d(7, 1, values="int4"),
    lambda: synth.rgg2d(120, 7.0, 2, values="int4"),
    lambda: synth.chung_lu(150, 5.0, 2.5, 3, values="int4"),
])
def test_permutation_is_PAPt(maker):
    L = maker()
    perm = oracle.rcm(L)
    B = oracle.permute(L, perm)
    assert oracle.validate(B.n, B.col.shape[0], B.rowptr, B.col) == 0
    S = dense_S(L)
    SB = dense_S(B)
    assert np.array_equal(SB, S[np.ix_(perm, perm)])
    assert np.array_equal(SB, -SB.T)
    x = np.floor(synth.values(L.n, 5) * 4.99)
    # B (P x) = P (S x) exactly for integer data
    assert np.array_equal(oracle.spmv(B, 0.0, x[perm]), oracle.spmv(L, 0.0, x)[perm])


def test_permutation_random_order_sign_rule():
    L = synth.from_edges(3, [(1, 0)], seed=0, values="ones")  # S[1,0] = 1
    B = oracle.permute(L, np.array([1, 0, 2], np.int32))      # swap nodes 0 and 1
    # new (0,1) = old (1,0) = 1 -> stored lower entry (1,0) = S_new[1,0] = old S[0,1] = -1
    assert B.rowptr.tolist() == [0, 0, 1, 1] and B.col.tolist() == [0] and B.val.tolist() == [-1.0]


@pytest.mark.parametrize("w_in,t_out", [(-1, -1), (0, 5), (2, 9), (4, 4), (0, 10 ** 6)])
def test_split_partition(w_in, t_out):
    L = synth.rgg2d(2000, 10.0, 4)
    B = oracle.permute(L, oracle.rcm(L))
    part, cnt, (w, t, beta) = oracle.split(B, w_in, t_out)
    rows = np.repeat(np.arange(B.n), np.diff(B.rowptr))
    d = rows - B.col
    assert beta == int(d.max())
    if w_in < 0:
        assert w == 0
    if t_out < 0:
        assert t == max(beta - 3, 0)
    want = np.where(d <= w, 0, np.where(d <= t, 1, 2))
    assert np.array_equal(part, want)
    assert cnt.sum() == B.nnz and list(cnt) == [int((want == k).sum()) for k in range(3)]
    if w == 0:
        assert cnt[0] == 0
    if t >= beta:
        assert cnt[2] == 0


def test_split_rejects_inverted_bounds():
    L = synth.grid2d(5, 1)
    with pytest.raises(ValueError):
        oracle.split(L, 5, 3)


def test_split_default_outer_is_three_outermost_diagonals():
    L = synth.grid2d(30, 2)
    B = oracle.permute(L, oracle.rcm(L))
    part, cnt, (w, t, beta) = oracle.split(B)
    rows = np.repeat(np.arange(B.n), np.diff(B.rowptr))
    d = rows - B.col
    assert cnt[2] == int((d > beta - 3).sum()) and cnt[2] > 0
    assert cnt[1] > cnt[2]  # the middle holds most of the entries


def test_validation_codes():
    rp = np.array([0, 0, 1, 3], np.int32)
    assert oracle.validate(3, 3, rp, np.array([0, 0, 1], np.int32)) == 0
    assert oracle.validate(3, 3, rp, np.array([0, 1, 0], np.int32)) == 3  # unsorted
    assert oracle.validate(3, 3, rp, np.array([0, 1, 1], np.int32)) == 3  # duplicate
    assert oracle.validate(3, 3, rp, np.array([1, 0, 1], np.int32)) == 2  # col >= row
    assert oracle.validate(3, 3, rp, np.array([0, 0, 2], np.int32)) == 2  # diagonal
    assert oracle.validate(3, 3, rp, np.array([-1, 0, 1], np.int32)) == 2
    assert oracle.validate(3, 2, rp, np.array([0, 0, 1], np.int32)) == 1  # nnz mismatch
    assert oracle.validate(3, 3, np.array([0, 2, 1, 3], np.int32), np.array([0, 0, 1], np.int32)) == 1
    assert oracle.validate(-1, 0, np.array([0], np.int32), None) == 1
    assert oracle.validate(0, 0, np.array([0], np.int32), None) == 0
    assert oracle.validate(1, 0, np.array([0, 0], np.int32), None) == 0
