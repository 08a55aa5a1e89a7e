"""Shifted skew-symmetric form of alpha*I + D + S (J = alpha*I + D diagonal,
positive definite; Section 1) and MRS through it, against the oracle.

Bars: S~ values within 2 ulp of the oracle's (the scaling of an entry that
crosses the diagonal multiplies its two factors in the other order), its
structure bit-exact; MRS iteration counts within 2 + 1% of the oracle's,
returned solutions' original-system residual (oracle FP64 product) <= tol and
within 1e-8 of the oracle's solutions."""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_17651_amd as p3
import synth
from gpu_util import rel_inf, to_dev

pytestmark = pytest.mark.gpu


def diag_for(n, seed, spread=4.0):
    return np.abs(synth.values(n, seed)) * spread


def true_relres(L, alpha, d, b, x):
    r = b - oracle.spmv(L, alpha, x, diag=d)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


@pytest.mark.parametrize("maker", [lambda: synth.rgg2d(20000, 12.0, 8), lambda: synth.grid3d(20, 3, "normal")])
def test_skew_form_values(maker):
    L = maker()
    d = diag_for(L.n, 3)
    M = p3.Matrix(L, diag=d).reorder()
    Bt = M.skew_form(0.25)
    perm = oracle.rcm(L)
    Lt, _ = oracle.skew_form(L, 0.25, d)
    want = oracle.permute(Lt, perm)
    rp, col, val, _ = Bt.permuted_lower()
    assert np.array_equal(rp, want.rowptr) and np.array_equal(col, want.col)
    assert np.all(np.abs(val - want.val) <= 2 * np.spacing(np.abs(want.val)))
    assert np.array_equal(Bt.perm(), perm)
    assert p3.pars3_get_kind(Bt.h) == (p3.SKEW, False)


@pytest.mark.parametrize("order", [p3.ORDER_RCM, p3.ORDER_ORIGINAL])
def test_mrs_matches_oracle(order):
    L = synth.workload(0)
    d = diag_for(L.n, 5)
    alpha = 0.2
    b0 = synth.values(L.n, 6)
    M = p3.Matrix(L, diag=d).reorder()
    perm = oracle.rcm(L)
    b = b0[perm] if order == p3.ORDER_RCM else b0
    x = torch.zeros(L.n, dtype=torch.float64, device="cuda")
    st, info, _ = M.mrs(alpha, to_dev(b), x, order=order, tol=1e-10, maxit=5000)
    assert st == p3.OK, info
    xo = x.cpu().numpy()
    if order == p3.ORDER_RCM:
        xr = np.empty_like(xo)
        xr[perm] = xo
        xo = xr
    res = true_relres(L, alpha, d, b0, xo)
    assert res <= 1e-10 and abs(res - info["relres"]) <= 1e-3 * res + 1e-15
    xw, iw, _ = oracle.mrs_shifted(L, alpha, d, b0, tol=1e-10, maxit=5000)
    assert abs(info["iters"] - iw["iters"]) <= 2 + iw["iters"] // 100, (info["iters"], iw["iters"])
    assert rel_inf(xo, xw) <= 1e-8


def test_initial_guess_and_wide_diagonal():
    L = synth.rgg2d(8000, 10.0, 2)
    d = np.geomspace(1e-2, 1e2, L.n)[np.random.default_rng(1).permutation(L.n)]
    M = p3.Matrix(L, diag=d).reorder()
    b = synth.values(L.n, 3)
    x0 = synth.values(L.n, 4)
    x = to_dev(x0)
    st, info, _ = M.mrs(0.0, to_dev(b), x, order=p3.ORDER_ORIGINAL, tol=1e-9, maxit=20000)
    assert st == p3.OK
    assert true_relres(L, 0.0, d, b, x.cpu().numpy()) <= 1e-9
    _, iw, _ = oracle.mrs_shifted(L, 0.0, d, b, x0, tol=1e-9, maxit=20000)
    assert abs(info["iters"] - iw["iters"]) <= 2 + iw["iters"] // 100


def test_zero_diagonal_matches_plain_solver():
    L = synth.grid2d(80, 4)
    b = to_dev(oracle.spmv(L, 0.6, np.ones(L.n)))
    M1 = p3.Matrix(L, diag=np.zeros(L.n)).reorder()
    M2 = p3.Matrix(L).reorder()
    x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
    _, i1, _ = M1.mrs(0.6, b, x1, order=p3.ORDER_ORIGINAL, tol=1e-11, maxit=3000)
    _, i2, _ = M2.mrs(0.6, b, x2, order=p3.ORDER_ORIGINAL, tol=1e-11, maxit=3000)
    assert abs(i1["iters"] - i2["iters"]) <= 1
    assert rel_inf(x1.cpu().numpy(), x2.cpu().numpy()) <= 1e-9


def test_mixed_precision_inner_solves():
    L = synth.grid3d(30, 7, "normal")
    d = diag_for(L.n, 8, 2.0)
    M = p3.Matrix(L, diag=d).reorder(value_dtype=p3.F32, keep_fp64=1)
    b = synth.values(L.n, 9)
    x = torch.zeros(L.n, dtype=torch.float64, device="cuda")
    st, info, _ = M.mrs(0.1, to_dev(b), x, order=p3.ORDER_ORIGINAL, tol=1e-10, maxit=5000, precision=p3.F32)
    assert st == p3.OK and info["refinements"] >= 1
    assert true_relres(L, 0.1, d, b, x.cpu().numpy()) <= 1e-10


def test_cache_follows_alpha_and_resplit():
    L = synth.rgg2d(6000, 8.0, 5)
    d = diag_for(L.n, 2)
    M = p3.Matrix(L, diag=d).reorder()
    b = synth.values(L.n, 3)
    for alpha, params in ((0.5, {}), (1.5, {}), (1.5, {"tile_rows": 64, "w_in": 2})):
        if params:
            M.reorder(**params)
        x = torch.zeros(L.n, dtype=torch.float64, device="cuda")
        st, _, _ = M.mrs(alpha, to_dev(b), x, order=p3.ORDER_ORIGINAL, tol=1e-10, maxit=5000)
        assert st == p3.OK and true_relres(L, alpha, d, b, x.cpu().numpy()) <= 1e-10


def test_errors():
    L = synth.grid2d(12, 1)
    d = np.zeros(L.n)
    d[5] = -2.0
    M = p3.Matrix(L, diag=d)
    with pytest.raises(p3.Pars3Error) as e:
        M.skew_form(1.0)
    assert e.value.status == p3.ESTATE
    M.reorder()
    b = to_dev(np.ones(L.n))
    for alpha in (1.0, 2.0 - 1e-12):
        with pytest.raises(p3.Pars3Error) as e:
            M.mrs(alpha, b, torch.zeros_like(b))
        assert e.value.status == p3.EINVAL
    with pytest.raises(p3.Pars3Error) as e:
        p3.Matrix(L).reorder().skew_form(0.0)  # alpha*I with alpha = 0
    assert e.value.status == p3.EINVAL
    S = p3.Matrix(L, diag=np.ones(L.n), symmetric=True).reorder()
    with pytest.raises(p3.Pars3Error) as e:
        S.mrs(1.0, b, torch.zeros_like(b))
    assert e.value.status == p3.ESTATE


def test_workload1_full_size():
    """The 3D 128^3 matrix with a diagonal D ~ |U[-1,1]|, alpha = 0.5, b = A 1,
    solved to 1e-10; the residual checked with the oracle's product."""
    L = synth.workload(1)
    d = np.abs(synth.values(L.n, 1204))
    print("[gpu] shifted mrs workload1", flush=True)
    M = p3.Matrix(L, diag=d).reorder()
    b = oracle.spmv(L, 0.5, np.ones(L.n), diag=d)
    x = torch.zeros(L.n, dtype=torch.float64, device="cuda")
    st, info, _ = M.mrs(0.5, to_dev(b), x, order=p3.ORDER_ORIGINAL, tol=1e-10, maxit=5000)
    print(f"[gpu] shifted mrs workload1 iters={info['iters']} ms={info['time_ms']:.1f}", flush=True)
    assert st == p3.OK
    assert true_relres(L, 0.5, d, b, x.cpu().numpy()) <= 1e-10
