"""Pins of the oracle's products (full-CSR definition and serial SSS kernel)
against the worked example of eqs. (2)-(6), dense products, exact integer
arithmetic and the skew-symmetry invariants."""
import json
import os

import numpy as np
import pytest

import oracle
import synth


def dense_S(L):
    """Dense S from its stored lower triangle, written with numpy indexing."""
    S = np.zeros((L.n, L.n))
    rows = np.repeat(np.arange(L.n), np.diff(L.rowptr))
    S[rows, L.col] = L.val
    S[L.col, rows] = -np.asarray(L.val)
    return S


def small_random(n, density, seed, values="uniform"):
    rng = np.random.default_rng(seed)
    edges = [(i, j) for i in range(n) for j in range(i) if rng.random() < density]
    return synth.from_edges(n, edges, seed=seed, values=values)


def test_worked_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "worked_example.json")))
    L = synth.Lower(g["n"], np.array(g["rowptr"], np.int32), np.array(g["col"], np.int32), np.array(g["val"]))
    x = np.array(g["x"])
    want = np.array(g["y_expected"])
    assert np.array_equal(oracle.spmv(L, 0.0, x), want)
    assert np.array_equal(oracle.sss_spmv(L, 0.0, x), want)


@pytest.mark.parametrize("n,density,seed", [(1, 0.0, 1), (2, 1.0, 2), (7, 0.5, 3), (33, 0.2, 4), (64, 0.1, 5)])
@pytest.mark.parametrize("alpha", [0.0, 1.0, -0.37])
def test_dense_product(n, density, seed, alpha):
    L = small_random(n, density, seed)
    x = synth.values(n, seed + 100)
    want = (dense_S(L) + alpha * np.eye(n)) @ x
    scale = max(np.abs(want).max(), 1e-300)
    for got in (oracle.spmv(L, alpha, x), oracle.sss_spmv(L, alpha, x)):
        assert np.abs(got - want).max() / scale <= 1e-14


def test_integer_inputs_exact():
    """Integer values in [-4, 4] and integer x: every partial sum is an exact
    integer, so all summation orders agree bit for bit."""
    L = small_random(50, 0.3, 9, values="int4")
    x = np.floor(synth.values(50, 77) * 4.999)
    want = dense_S(L) @ x + 2.0 * x
    assert np.array_equal(oracle.spmv(L, 2.0, x), want)
    assert np.array_equal(oracle.sss_spmv(L, 2.0, x), want)


def test_quadratic_form_vanishes():
    L = synth.grid2d(20, 3)
    x = synth.values(L.n, 5)
    y = oracle.spmv(L, 0.0, x)
    bound = 4 * L.nnz * np.finfo(float).eps * np.abs(L.val).max() * np.abs(x).max() ** 2
    assert abs(float(x @ y)) <= bound


def test_skew_adjoint_and_linearity():
    L = synth.rgg2d(500, 8.0, 11)
    x, z = synth.values(L.n, 1), synth.values(L.n, 2)
    Sx, Sz = oracle.spmv(L, 0.0, x), oracle.spmv(L, 0.0, z)
    assert abs(z @ Sx + x @ Sz) <= 1e-12 * (np.linalg.norm(z) * np.linalg.norm(Sx) + 1)
    comb = oracle.spmv(L, 0.0, 2.0 * x - 3.0 * z)
    assert np.abs(comb - (2.0 * Sx - 3.0 * Sz)).max() <= 1e-13 * np.abs(comb).max()


def test_shift_is_diagonal_only():
    L = synth.grid2d(8, 4)
    x = synth.values(L.n, 6)
    a = 0.75
    d = oracle.spmv(L, a, x) - oracle.spmv(L, 0.0, x)
    assert np.abs(d - a * x).max() <= 1e-15 * 4


def test_sss_matches_full_csr_on_workload0():
    L = synth.workload(0)
    x = synth.vector(L.n, 2000)
    y1, y2 = oracle.spmv(L, 1.0, x), oracle.sss_spmv(L, 1.0, x)
    assert np.abs(y1 - y2).max() / np.abs(y1).max() <= 1e-14


def test_full_csr_layout():
    L = synth.grid2d(5, 8)
    frow, fcol, fval = oracle.full_csr(L, 0.0)
    assert frow[-1] == 2 * L.nnz
    for i in range(L.n):
        c = fcol[frow[i]:frow[i + 1]]
        assert np.all(np.diff(c) > 0)
    frow_a, fcol_a, _ = oracle.full_csr(L, 1.5)
    assert frow_a[-1] == 2 * L.nnz + L.n


def test_parallel_full_csr_product_equals_serial():
    """The all-core baseline shares rows among threads; each row is summed
    alone in the same order, so the result is the serial one bit for bit."""
    L = synth.grid3d(30, 4, "normal")
    frow, fcol, fval = oracle.full_csr(L, 0.5)
    x = synth.vector(L.n, 9)
    assert np.array_equal(oracle.csr_spmv_par(frow, fcol, fval, x), oracle.csr_spmv(frow, fcol, fval, x))
    assert oracle.num_threads() >= 1
