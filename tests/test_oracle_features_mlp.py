"""Pins of the oracle's sparsity features (hand-computed cases) and of the MLP
(finite differences, closed forms)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp


def path_lower(n):
    return synth.Lower(n, np.concatenate([[0], np.arange(n)]).astype(np.int32),
                       np.arange(n - 1, dtype=np.int32), np.ones(n - 1))


def test_path_features():
    n = 1000
    f = oracle.features(path_lower(n))
    assert f[0] == np.log2(n) and f[1] == np.log2(n - 1)
    assert f[2] == (n - 1) / n and f[3] == 1 / n and f[4] == 1.0
    # b_i = 1 except b_0 = 0: p10..max quantiles are all 1 (rank >= 2)
    assert list(f[5:10]) == [1.0] * 5
    assert f[10] == 1.0
    assert list(f[11:19]) == [1.0] * 8
    assert list(f[19:22]) == [1.0] * 3
    assert f[22] == 1 / n and f[23] == (n - 1) / n and sum(f[24:29]) == 0
    assert f[29] == n / (n - 1)
    assert f[30] == np.sqrt(n * (n - 1) - (n - 1) ** 2) / (n - 1)
    assert f[31] == 1.0


def test_hand_built_small():
    # n = 4: row 3 holds columns 0 and 2 (d = 3, 1); row 2 holds column 1 (d = 1)
    L = synth.Lower(4, np.array([0, 0, 0, 1, 3], np.int32), np.array([1, 0, 2], np.int32), np.ones(3))
    f = oracle.features(L)
    # b = [0, 0, 1, 3], beta = 3; ranks ceil(0.1*4)=1 -> 0, ceil(0.5*4)=2 -> 0, ceil(0.9*4)=4 -> 3
    assert list(f[5:10]) == [0.0, 0.0, 1.0, 1.0, 1.0]
    assert f[10] == 3 / 4
    assert f[11] == 2 / 3 and f[12] == 2 / 3 and f[13] == 1.0
    assert f[19] == 1 / 3  # only d = 3 exceeds beta / 2
    assert list(f[22:25]) == [0.5, 0.25, 0.25]
    assert f[29] == 2 * 4 / 3


def test_empty_matrix_features():
    f = oracle.features(synth.Lower(3, np.zeros(4, np.int32), np.zeros(0, np.int32), np.zeros(0)))
    assert f[0] == np.log2(3) and f[22] == 1.0 and f[31] == 1.0
    assert np.count_nonzero(f) == 3


def _params(rng, sizes=(32, 64, 64, 6)):
    p = {}
    for k, (a, b) in enumerate(zip(sizes[:-1], sizes[1:]), 1):
        p[f"W{k}"] = rng.normal(0, 1 / np.sqrt(a), (a, b))
        p[f"b{k}"] = rng.normal(0, 0.1, b)
    return p


def test_mlp_finite_differences():
    rng = np.random.default_rng(0)
    p = _params(rng)
    X = rng.normal(size=(9, 32))
    T = rng.normal(size=(9, 6))
    M = (rng.random((9, 6)) < 0.8).astype(float)
    out, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, out, T, M)
    h = 1e-6
    for k in mlp.NAMES:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(p, X)[0], T, M)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(p, X)[0], T, M)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_mlp_output_bias_gradient_closed_form():
    rng = np.random.default_rng(1)
    p = _params(rng)
    X = rng.normal(size=(5, 32))
    T = rng.normal(size=(5, 6))
    M = np.ones((5, 6))
    out, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, out, T, M)
    assert np.allclose(g["b3"], 2 * (out - T).sum(0) / M.sum(), rtol=1e-14, atol=1e-15)


def test_adam_first_step_is_signed_learning_rate():
    rng = np.random.default_rng(2)
    p = _params(rng)
    g = {k: rng.normal(size=v.shape) for k, v in p.items()}
    z = {k: np.zeros_like(v) for k, v in p.items()}
    P, m, v = mlp.adam_step(p, g, z, z, 1, lr=1e-2, eps=0.0)
    for k in mlp.NAMES:
        assert np.allclose(P[k] - p[k], -1e-2 * np.sign(g[k]), rtol=1e-12, atol=1e-15)


def test_window_fit_boundary_cases():
    """f[31] where its boundary decides: 256-row tiles, n = 20600 (the last
    tile holds 120 rows).  Tile 40 (rows 10240..10495) has one entry in
    column 256: window 10496 - 256 = 10240 rows = exactly 160 KiB at 16
    bytes a row, so it fits.  Tile 60 (rows 15360..15615) has one entry in
    column 15616 - 10241: window 10241 rows, 16 bytes over, so it does not.
    The last tile has one entry in column 20600 - 10240: its window, with
    the tile's end clipped to n, is exactly 160 KiB (unclipped it would not
    fit).  Every other tile is empty and fits.  So f[31] = 80/81; a row size
    of 8 bytes would give 81/81, '<' for '<=' 78/81 and an unclipped last
    tile 79/81."""
    n = 20600
    rows = [10300, 15400, 20590]
    cols = [256, 15616 - 10241, 20600 - 10240]
    rowptr = np.zeros(n + 1, np.int32)
    for r in rows:
        rowptr[r + 1:] += 1
    L = synth.Lower(n, rowptr, np.array(cols, np.int32), np.ones(3))
    f = oracle.features(L)
    assert f[31] == 80 / 81


def test_distance_shares_at_their_thresholds():
    """f[19..21] (shares with d/beta > 1/2, 3/4, 9/10) where d sits exactly at
    each threshold: beta = 20 and d in {20, 10, 15, 18, 11, 16, 19}, one
    entry per row.  d = 10, 15 and 18 equal beta/2, 3 beta/4 and 9 beta/10
    and do not count: 6/7, 4/7 and 2/7 ('>=' would give 7/7, 5/7, 3/7).
    f[11..18] (d <= 1, 2, 4, ..., 128) are 0, 0, 0, 0, 4/7 and then 1."""
    n = 40
    rc = [(30, 10), (31, 21), (32, 17), (33, 15), (34, 23), (35, 19), (36, 17)]
    rowptr = np.zeros(n + 1, np.int32)
    for r, _ in rc:
        rowptr[r + 1:] += 1
    L = synth.Lower(n, rowptr, np.array([c for _, c in rc], np.int32), np.ones(len(rc)))
    assert sorted(r - c for r, c in rc) == [10, 11, 15, 16, 18, 19, 20]
    f = oracle.features(L)
    assert f[3] == 20 / n and f[4] == np.log2(21)
    assert list(f[19:22]) == [6 / 7, 4 / 7, 2 / 7]
    assert list(f[11:19]) == [0.0, 0.0, 0.0, 0.0, 4 / 7, 1.0, 1.0, 1.0]
