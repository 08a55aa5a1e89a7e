"""Pins of the oracle's shifted skew-symmetric form of A = J + S with a
diagonal positive definite J = alpha*I + D (Section 1) and of MRS through it:
the dense scaling identity, dense solves, the residual bound, and the case
D = 0 that reduces to plain MRS on alpha*I + S."""
import numpy as np
import pytest

import oracle
import synth


def dense(L, sign=-1.0):
    S = np.zeros((L.n, L.n))
    rows = np.repeat(np.arange(L.n), np.diff(L.rowptr))
    S[rows, L.col] = L.val
    S[L.col, rows] = sign * np.asarray(L.val)
    return S


def test_scaling_identity():
    L = synth.rgg2d(120, 6.0, 3)
    d = np.abs(synth.values(L.n, 4)) * 5.0
    alpha = 0.3
    Lt, ds = oracle.skew_form(L, alpha, d)
    A = dense(L) + np.diag(alpha + d)
    want = np.diag(ds) @ A @ np.diag(ds)
    got = np.eye(L.n) + dense(Lt)
    assert np.abs(got - want).max() <= 1e-15 * np.abs(want).max()
    assert np.array_equal(dense(Lt), -dense(Lt).T)
    assert np.array_equal(Lt.rowptr, L.rowptr) and np.array_equal(Lt.col, L.col)


@pytest.mark.parametrize("seed", range(4))
def test_dense_solve(seed):
    rng = np.random.default_rng(seed)
    L = synth.rgg2d(80, 5.0, seed)
    d = rng.uniform(0.0, 10.0 ** rng.uniform(0, 3), L.n)
    alpha = float(rng.uniform(0.05, 1.0))
    b = synth.values(L.n, seed + 9)
    x, info, _ = oracle.mrs_shifted(L, alpha, d, b, tol=1e-12, maxit=2000)
    A = dense(L) + np.diag(alpha + d)
    xs = np.linalg.solve(A, b)
    r = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert info["status"] == 0 and r <= 1e-12 and abs(r - info["relres"]) <= 1e-14
    assert np.abs(x - xs).max() <= 1e-9 * np.abs(xs).max()


def test_residual_bound_with_wide_diagonal():
    L = synth.grid2d(30, 2)
    d = np.geomspace(1e-2, 1e3, L.n)[np.random.default_rng(3).permutation(L.n)]
    for tol in (1e-6, 1e-10):
        x, info, _ = oracle.mrs_shifted(L, 0.0, d, synth.values(L.n, 1), tol=tol, maxit=5000)
        assert info["status"] == 0 and info["relres"] <= tol


def test_zero_diagonal_is_plain_mrs():
    """D = 0: I + S/alpha spans the same Krylov spaces as alpha*I + S."""
    L = synth.workload(0)
    b = oracle.spmv(L, 1.0, np.ones(L.n))
    x1, i1, _ = oracle.mrs_shifted(L, 0.7, np.zeros(L.n), b, tol=1e-10, maxit=2000)
    x2, i2, _ = oracle.mrs(L, 0.7, b, tol=1e-10, maxit=2000)
    assert abs(i1["iters"] - i2["iters"]) <= 1
    assert np.abs(x1 - x2).max() <= 1e-9 * np.abs(x2).max()


def test_rejects_indefinite_diagonal():
    L = synth.grid2d(5, 1)
    d = np.zeros(L.n)
    d[3] = -1.0
    with pytest.raises(ValueError):
        oracle.skew_form(L, 0.5, d)
    with pytest.raises(ValueError):
        oracle.skew_form(L, 0.0, np.zeros(L.n))
