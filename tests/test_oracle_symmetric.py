"""Pins of the oracle's symmetric variant and diagonal array: the product
alpha*I + D + S with S = L + L^T (symmetric) or L - L^T (skew), in its
full-CSR and serial SSS forms, and the sign-free permutation of a symmetric
matrix.  Checked against dense products written with numpy indexing, exact
integer arithmetic, a hand-derived 4x4 example, the symmetry identity
z^T A x = x^T A z and a brute-force quadratic form."""
import json
import os

import numpy as np
import pytest

import oracle
import synth


def dense(L, sign):
    S = np.zeros((L.n, L.n))
    rows = np.repeat(np.arange(L.n), np.diff(L.rowptr))
    S[rows, L.col] = L.val
    S[L.col, rows] = sign * np.asarray(L.val)
    return S


def small_random(n, density, seed, values="uniform"):
    rng = np.random.default_rng(seed)
    edges = [(i, j) for i in range(n) for j in range(i) if rng.random() < density]
    return synth.from_edges(n, edges, seed=seed, values=values)


def test_symmetric_worked_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "symmetric_example.json")))
    L = synth.Lower(g["n"], np.array(g["rowptr"], np.int32), np.array(g["col"], np.int32), np.array(g["val"]))
    x, d, a = np.array(g["x"]), np.array(g["diag"]), g["alpha"]
    want = np.array(g["y_expected"])
    assert np.array_equal(oracle.spmv(L, a, x, diag=d, symmetric=True), want)
    assert np.array_equal(oracle.sss_spmv(L, a, x, diag=d, symmetric=True), want)


@pytest.mark.parametrize("n,density,seed", [(1, 0.0, 1), (2, 1.0, 2), (9, 0.5, 3), (40, 0.2, 4)])
@pytest.mark.parametrize("symmetric", [False, True])
@pytest.mark.parametrize("with_diag", [False, True])
def test_dense_product(n, density, seed, symmetric, with_diag):
    L = small_random(n, density, seed)
    x = synth.values(n, seed + 100)
    d = synth.values(n, seed + 200) if with_diag else None
    alpha = -0.37
    A = dense(L, 1.0 if symmetric else -1.0) + alpha * np.eye(n) + (np.diag(d) if with_diag else 0.0)
    want = A @ x
    scale = max(np.abs(want).max(), 1e-300)
    for got in (oracle.spmv(L, alpha, x, diag=d, symmetric=symmetric),
                oracle.sss_spmv(L, alpha, x, diag=d, symmetric=symmetric)):
        assert np.abs(got - want).max() / scale <= 1e-14


def test_integer_inputs_exact():
    L = small_random(60, 0.3, 9, values="int4")
    x = np.floor(synth.values(60, 77) * 4.999)
    d = np.floor(synth.values(60, 78) * 3.999)
    want = dense(L, 1.0) @ x + 2.0 * x + d * x
    assert np.array_equal(oracle.spmv(L, 2.0, x, diag=d, symmetric=True), want)
    assert np.array_equal(oracle.sss_spmv(L, 2.0, x, diag=d, symmetric=True), want)


def test_symmetry_identity():
    L = synth.rgg2d(500, 8.0, 11)
    d = synth.values(L.n, 3)
    x, z = synth.values(L.n, 1), synth.values(L.n, 2)
    Ax = oracle.spmv(L, 0.5, x, diag=d, symmetric=True)
    Az = oracle.spmv(L, 0.5, z, diag=d, symmetric=True)
    assert abs(z @ Ax - x @ Az) <= 1e-12 * (np.linalg.norm(z) * np.linalg.norm(Ax) + 1)


def test_quadratic_form_brute_force():
    """x^T (L + L^T) x = 2 * sum over stored l_ij of l_ij x_i x_j, summed by
    plain loops over the triangle."""
    L = small_random(30, 0.4, 12)
    x = synth.values(30, 13)
    want = 0.0
    for i in range(L.n):
        for e in range(L.rowptr[i], L.rowptr[i + 1]):
            want += 2.0 * L.val[e] * x[i] * x[L.col[e]]
    got = float(x @ oracle.spmv(L, 0.0, x, symmetric=True))
    assert abs(got - want) <= 1e-13 * max(1.0, abs(want))


def test_constant_diagonal_equals_shift():
    L = synth.grid2d(9, 4)
    x = synth.values(L.n, 6)
    for sym in (False, True):
        a = oracle.spmv(L, 0.0, x, diag=np.full(L.n, 0.75), symmetric=sym)
        b = oracle.spmv(L, 0.75, x, symmetric=sym)
        assert np.array_equal(a, b)


def test_skew_default_unchanged_by_zero_diagonal():
    L = synth.rgg2d(300, 7.0, 5)
    x = synth.values(L.n, 8)
    assert np.array_equal(oracle.spmv(L, 1.0, x, diag=np.zeros(L.n)), oracle.spmv(L, 1.0, x))
    assert np.array_equal(oracle.sss_spmv(L, 1.0, x, diag=np.zeros(L.n)), oracle.sss_spmv(L, 1.0, x))


@pytest.mark.parametrize("maker", [
    lambda: synth.grid2d(7, 1, values="int4"),
    lambda: synth.chung_lu(150, 5.0, 2.5, 3, values="int4"),
])
def test_symmetric_permutation_is_PAPt(maker):
    L = maker()
    perm = oracle.rcm(L)
    B = oracle.permute(L, perm, symmetric=True)
    assert oracle.validate(B.n, B.col.shape[0], B.rowptr, B.col) == 0
    S = dense(L, 1.0)
    SB = dense(B, 1.0)
    assert np.array_equal(SB, S[np.ix_(perm, perm)])
    assert np.array_equal(SB, SB.T)
    x = np.floor(synth.values(L.n, 5) * 4.99)
    d = np.floor(synth.values(L.n, 6) * 3.99)
    assert np.array_equal(oracle.spmv(B, 0.0, x[perm], diag=d[perm], symmetric=True),
                          oracle.spmv(L, 0.0, x, diag=d, symmetric=True)[perm])


def test_symmetric_permutation_keeps_sign():
    L = synth.from_edges(3, [(1, 0)], seed=0, values="ones")
    B = oracle.permute(L, np.array([1, 0, 2], np.int32), symmetric=True)
    assert B.rowptr.tolist() == [0, 0, 1, 1] and B.col.tolist() == [0] and B.val.tolist() == [1.0]


def test_full_csr_diagonal_entries():
    L = synth.grid2d(5, 8)
    d = np.zeros(L.n)
    d[3] = -1.5  # alpha + d_3 = 0: no diagonal entry in row 3
    d[4] = 2.0
    frow, fcol, fval = oracle.full_csr(L, 1.5, diag=d, symmetric=True)
    assert frow[-1] == 2 * L.nnz + L.n - 1
    for i in range(L.n):
        c = fcol[frow[i]:frow[i + 1]]
        assert np.all(np.diff(c) > 0)
        on = np.flatnonzero(c == i)
        if i == 3:
            assert on.size == 0
        else:
            assert fval[frow[i] + on[0]] == 1.5 + d[i]
    # every off-diagonal value appears twice with the same sign
    off = fcol != np.repeat(np.arange(L.n), np.diff(frow))
    assert np.isclose(fval[off].sum(), 2 * L.val.sum())
