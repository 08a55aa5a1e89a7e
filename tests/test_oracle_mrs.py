"""Pins of the oracle's MRS iteration: closed forms, brute-force Krylov least
squares, monotone residuals, agreement with a dense LU solve."""
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


def test_two_by_two_closed_form():
    s, a = 1.7, 0.4
    L = synth.Lower(2, np.array([0, 0, 1], np.int32), np.array([0], np.int32), np.array([s]))
    b = np.array([0.3, -1.1])
    x, info, _ = oracle.mrs(L, a, b, tol=1e-15, maxit=10)
    # S = [[0, -s], [s, 0]];  (aI + S)^-1 b = (a b0 + s b1, a b1 - s b0) / (a^2 + s^2)
    want = np.array([a * b[0] + s * b[1], a * b[1] - s * b[0]]) / (a * a + s * s)
    assert info["iters"] <= 2
    assert np.abs(x - want).max() <= 1e-15 * 8


def test_zero_matrix_one_step():
    L = synth.Lower(5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    b = synth.values(5, 1)
    x, info, _ = oracle.mrs(L, 2.0, b, tol=1e-14, maxit=10)
    assert info["iters"] == 1 and info["status"] == 0
    assert np.array_equal(x, b / 2.0)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_krylov_least_squares(seed):
    """x_k minimises ||b - A x|| over x0 + K_k(S, r0): explicit basis,
    Householder QR least squares, compared for every k."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 13))
    edges = [(i, j) for i in range(n) for j in range(i) if rng.random() < 0.5]
    L = synth.from_edges(n, edges, seed=seed)
    S = dense_S(L)
    a = float(rng.uniform(0.1, 2.0))
    A = a * np.eye(n) + S
    b = rng.uniform(-1, 1, n)
    x0 = rng.uniform(-1, 1, n)
    r0 = b - A @ x0
    K = []
    q = r0.copy()
    for k in range(1, n + 1):
        K.append(q)
        q = S @ q
        Q, _ = np.linalg.qr(np.array(K).T)
        Q, _ = np.linalg.qr(Q)  # orthonormalise twice
        y = np.linalg.lstsq(A @ Q, r0, rcond=None)[0]
        x_want = x0 + Q @ y
        if np.linalg.matrix_rank(np.array(K).T, tol=1e-9) < k:
            break
        x, info, _ = oracle.mrs(L, a, b, x0=x0, tol=0.0, maxit=k)
        if info["status"] != 1 and info["iters"] < k:  # exact solution reached early
            break
        assert np.abs(x - x_want).max() <= 1e-9 * max(1.0, np.abs(x_want).max()), k


def test_residual_history_monotone_and_exact():
    L = synth.rgg2d(300, 6.0, 2)
    b = oracle.spmv(L, 0.8, np.ones(L.n))
    x, info, hist = oracle.mrs(L, 0.8, b, tol=1e-12, maxit=400)
    assert info["status"] == 0
    assert np.all(np.diff(hist) <= 1e-15)
    # |eta| equals the true residual
    assert abs(info["eta"] - info["relres"]) <= 1e-10 * max(info["relres"], 1e-12) + 1e-13
    A = 0.8 * np.eye(L.n) + dense_S(L)
    assert np.abs(x - np.linalg.solve(A, b)).max() <= 1e-9


def test_eta_tracks_true_residual_each_step():
    L = synth.grid2d(10, 3)
    b = oracle.spmv(L, 1.0, np.ones(L.n))
    for k in (1, 3, 7, 15):
        x, info, hist = oracle.mrs(L, 1.0, b, tol=0.0, maxit=k)
        assert abs(hist[-1] - oracle.residual(L, 1.0, b, x)) <= 1e-10 * hist[-1] + 1e-15


def test_workload0_fifty_iterations():
    """Workload 0: alpha = 1, b = A 1, x0 = 0, 50 iterations."""
    L = synth.workload(0)
    b = oracle.spmv(L, 1.0, np.ones(L.n))
    x, info, hist = oracle.mrs(L, 1.0, b, tol=0.0, maxit=50)
    assert info["iters"] == 50
    assert hist[-1] <= 1e-8
    assert np.abs(x - 1.0).max() <= 1e-7


def test_singular_alpha_zero_odd_n():
    """alpha = 0 and odd n: S is singular; b outside its range cannot be solved."""
    L = synth.grid2d(3, 1)
    b = np.ones(L.n)
    x, info, _ = oracle.mrs(L, 0.0, b, tol=1e-12, maxit=50)
    assert info["status"] in (1, 2)
    assert info["relres"] > 1e-6


def test_exit_residual_is_the_full_csr_definition():
    """info['relres'] of the oracle's MRS is ||b - A x|| / ||b|| with A x from
    the full CSR of alpha*I + S (recomputed here by a dense product)."""
    L = synth.rgg2d(300, 8.0, 5)
    alpha = 0.3
    b = synth.vector(L.n, 2)
    x, info, _ = oracle.mrs(L, alpha, b, tol=1e-6, maxit=40)
    A = alpha * np.eye(L.n)
    for i in range(L.n):
        for e in range(L.rowptr[i], L.rowptr[i + 1]):
            j = L.col[e]
            A[i, j] += L.val[e]
            A[j, i] -= L.val[e]
    r = b - A @ x
    assert abs(info["relres"] - np.linalg.norm(r) / np.linalg.norm(b)) <= 1e-12 * info["relres"] + 1e-300
