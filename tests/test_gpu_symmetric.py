"""Symmetric variant and SSS diagonal array on the GPU, against the oracle.

The same one-triangle storage serves S = L + L^T (symmetric, the SSS format
of Section 1) and a diagonal array D beside the triangle; products compute
y = shift x + D x + S x.  Bars as for the skew product: FP64 <= 1e-12,
FP32/BF16 values with FP32 vectors <= 1e-5 relative infinity-norm error
against the oracle on the same rounded values, diagonal and vectors;
integer-valued inputs bit-exact; the permutation and the permuted diagonal
bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_17651_amd as p3
import synth
from gpu_util import gpu_spmv, rel_inf, to_dev

pytestmark = pytest.mark.gpu

TOL = {p3.F64: 1e-12, p3.F32: 1e-5, p3.BF16: 1e-5}
KINDS = {"skew+diag": (False, True), "sym": (True, False), "sym+diag": (True, True)}
KIND = {p3.F64: "f64", p3.F32: "f32", p3.BF16: "bf16"}


def make(L, sym, with_diag, seed=5):
    d = synth.values(L.n, seed, "normal") if with_diag else None
    return d, p3.Matrix(L, diag=d, symmetric=sym)


def oracle_product(L, d, sym, shift, X, value_dtype):
    """The oracle on the oracle's own reordering, with values, diagonal and
    vectors rounded to what the GPU path is given."""
    perm = oracle.rcm(L)
    B = oracle.permute(L, perm, symmetric=sym)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    Bv = type(B)(**{**B.__dict__, "val": oracle.rounded_values(B.val, KIND[value_dtype])})
    dp = None if d is None else d[perm]
    if dp is not None and vec == p3.F32:
        dp = oracle.rounded_values(dp, "f32")
    Xr = X if vec == p3.F64 else X.astype(np.float32).astype(np.float64)
    return oracle.spmv(Bv, shift, Xr, diag=dp, symmetric=sym)


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("maker", [lambda: synth.rgg2d(20000, 12.0, 8), lambda: synth.grid3d(20, 3, "normal"),
                                   lambda: synth.chung_lu(12000, 10.0, 2.5, 5)])
def test_permutation_and_diagonal_bit_exact(kind, maker):
    L = maker()
    sym, wd = KINDS[kind]
    d, M = make(L, sym, wd)
    M.reorder()
    perm = oracle.rcm(L)
    B = oracle.permute(L, perm, symmetric=sym)
    rp, col, val, _ = M.permuted_lower()
    assert np.array_equal(rp, B.rowptr) and np.array_equal(col, B.col) and np.array_equal(val, B.val)
    assert p3.pars3_get_kind(M.h) == (p3.SYMMETRIC if sym else p3.SKEW, wd)
    if wd:
        assert np.array_equal(M.diagonal(), d[perm])


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("value_dtype", [p3.F64, p3.F32, p3.BF16])
@pytest.mark.parametrize("k", [1, 4, 8])
def test_product_parity(kind, value_dtype, k):
    L = synth.rgg2d(30000, 16.0, 4)
    sym, wd = KINDS[kind]
    print(f"[gpu] symmetric spmv kind={kind} dtype={value_dtype} k={k}", flush=True)
    d, M = make(L, sym, wd)
    M.reorder(value_dtype=value_dtype)
    X = synth.vector(L.n, 21, k)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    want = oracle_product(L, d, sym, -0.3, X, value_dtype)
    assert rel_inf(gpu_spmv(M, -0.3, X, vec), want) <= TOL[value_dtype]


@pytest.mark.parametrize("params", [dict(tile_rows=64), dict(tile_rows=1024), dict(w_in=4), dict(w_in=16, t_out=40),
                                    dict(w_in=0, t_out=0), dict(w_in=64), dict(permute=0)])
def test_layout_variants(params):
    """Inner band (both directions), middle and outer parts all carry the
    symmetric sign; permute=0 keeps the given numbering."""
    L = synth.rgg2d(20000, 12.0, 9)
    d, M = make(L, True, True)
    M.reorder(**params)
    x = synth.vector(L.n, 3)
    if params.get("permute", 1):
        want = oracle_product(L, d, True, 0.75, x, p3.F64)
    else:
        want = oracle.spmv(L, 0.75, x, diag=d, symmetric=True)
    assert rel_inf(gpu_spmv(M, 0.75, x), want) <= 1e-12


@pytest.mark.parametrize("value_dtype", [p3.F64, p3.F32, p3.BF16])
@pytest.mark.parametrize("params", [dict(), dict(w_in=3), dict(tile_rows=64)])
def test_integer_inputs_bit_exact(value_dtype, params):
    L = synth.rgg2d(8000, 10.0, 12, "int4")
    d = np.floor(synth.values(L.n, 4) * 3.999)
    M = p3.Matrix(L, diag=d, symmetric=True).reorder(value_dtype=value_dtype, **params)
    perm = oracle.rcm(L)
    B = oracle.permute(L, perm, symmetric=True)
    x = np.floor(synth.vector(L.n, 3) * 4.999)
    want = oracle.spmv(B, 2.0, x, diag=d[perm], symmetric=True)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    assert np.array_equal(gpu_spmv(M, 2.0, x, vec), want)


@pytest.mark.parametrize("kind", list(KINDS))
def test_original_order(kind):
    L = synth.grid2d(150, 7)
    sym, wd = KINDS[kind]
    d, M = make(L, sym, wd)
    M.reorder()
    x = synth.vector(L.n, 8)
    want = oracle.spmv(L, 1.25, x, diag=d, symmetric=sym)
    assert rel_inf(gpu_spmv(M, 1.25, x, order=p3.ORDER_ORIGINAL), want) <= 1e-12


def test_symmetry_identity_on_the_gpu():
    """z^T (A x) = x^T (A z) for the symmetric product (A = A^T), to rounding."""
    L = synth.grid3d(24, 6, "normal")
    d, M = make(L, True, True)
    M.reorder()
    x, z = synth.vector(L.n, 1), synth.vector(L.n, 2)
    Ax, Az = gpu_spmv(M, 0.5, x), gpu_spmv(M, 0.5, z)
    assert abs(z @ Ax - x @ Az) <= 1e-12 * np.linalg.norm(z) * np.linalg.norm(Ax)


def test_empty_and_tiny():
    for L in (synth.from_edges(1, [], seed=1), synth.from_edges(2, [(1, 0)], seed=2),
              synth.from_edges(5, [], seed=3)):
        d = synth.values(L.n, 9)
        M = p3.Matrix(L, diag=d, symmetric=True).reorder()
        x = synth.vector(L.n, 4)
        perm = oracle.rcm(L)
        want = oracle.spmv(oracle.permute(L, perm, symmetric=True), 0.5, x, diag=d[perm], symmetric=True)
        assert rel_inf(gpu_spmv(M, 0.5, x), want) <= 1e-15
    M0 = p3.Matrix(synth.from_edges(0, [], seed=0), diag=np.zeros(0), symmetric=True).reorder()
    x0 = torch.zeros(0, dtype=torch.float64, device="cuda")
    M0.spmv(1.0, x0, torch.zeros_like(x0))


@pytest.mark.parametrize("order", [p3.ORDER_RCM, p3.ORDER_ORIGINAL])
@pytest.mark.parametrize("kind", list(KINDS))
def test_full_csr_path(order, kind):
    L = synth.rgg2d(10000, 10.0, 6)
    sym, wd = KINDS[kind]
    d, M = make(L, sym, wd)
    M.reorder()
    perm = oracle.rcm(L)
    if order == p3.ORDER_RCM:
        B, dd = oracle.permute(L, perm, symmetric=sym), (None if d is None else d[perm])
    else:
        B, dd = L, d
    C = p3.pars3_csr_create(M.h, order, p3.F64)
    try:
        rp, col, val = p3.pars3_csr_get(C)
        frow, fcol, fval = oracle.full_csr(B, 0.0, diag=dd, symmetric=sym)
        assert np.array_equal(rp, frow) and np.array_equal(col, fcol) and np.array_equal(val, fval)
        x = synth.vector(L.n, 5)
        xd = to_dev(x)
        for engine, shift in ((0, 0.5), (1, 0.0)):
            y = torch.full_like(xd, float("nan"))
            p3.pars3_csr_spmv(C, shift, xd, y, engine)
            torch.cuda.synchronize()
            want = oracle.spmv(B, shift, x, diag=dd, symmetric=sym)
            assert rel_inf(y.cpu().numpy(), want) <= 1e-12, engine
    finally:
        p3.pars3_csr_destroy(C)


@pytest.mark.parametrize("k,value_dtype", [(1, p3.F64), (8, p3.F32)])
def test_batch_mixes_kinds(k, value_dtype):
    """Skew, skew+diag, symmetric and symmetric+diag matrices in one batch."""
    specs = synth.batch_specs(8, 61, 2000, 20000)
    Ls = [synth.make(s, "uniform_f32") for s in specs]
    kinds = [(False, False), (False, True), (True, False), (True, True)] * 2
    ds, mats = [], []
    for i, L in enumerate(Ls):
        d, M = make(L, *kinds[i], seed=30 + i)
        ds.append(d)
        mats.append(M.reorder(value_dtype=value_dtype, tile_rows=(256, 512)[i % 2]))
    bat = p3.Batch(mats)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    tdt = torch.float64 if vec == p3.F64 else torch.float32
    Xs = [synth.vector(L.n, 100 + i, k) for i, L in enumerate(Ls)]
    xs = [to_dev(X, tdt) for X in Xs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    shifts = np.array([s["alpha"] for s in specs])
    bat.spmv(xs, ys, shifts, k=k, vec_dtype=vec)
    torch.cuda.synchronize()
    for i, L in enumerate(Ls):
        want = oracle_product(L, ds[i], kinds[i][0], shifts[i], Xs[i], value_dtype)
        assert rel_inf(ys[i].cpu().numpy().astype(np.float64), want) <= TOL[value_dtype], i


def test_solvers_reject_non_skew():
    """MRS needs S skew: a symmetric handle is refused by both solvers; a
    skew handle with a diagonal array is solved through its shifted skew
    form only when alpha*I + D is positive definite (EINVAL here: the N(0,1)
    diagonal has negative entries), and never batched."""
    L = synth.grid2d(20, 1)
    b = to_dev(np.ones(L.n))
    for sym, wd, single in ((True, False, p3.ESTATE), (False, True, p3.EINVAL)):
        d, M = make(L, sym, wd)
        M.reorder()
        x = torch.zeros_like(b)
        with pytest.raises(p3.Pars3Error) as e:
            M.mrs(1.0, b, x)
        assert e.value.status == single
        bat = p3.Batch([M])
        with pytest.raises(p3.Pars3Error) as e:
            bat.mrs([1.0], [b], [x])
        assert e.value.status == p3.ESTATE


def test_errors():
    L = synth.grid2d(10, 1)
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_create_sss(L.n, L.nnz, L.rowptr, L.col, L.val, None, 2)
    assert e.value.status == p3.EINVAL
    M = p3.Matrix(L, symmetric=True)
    with pytest.raises(p3.Pars3Error) as e:
        M.diagonal()
    assert e.value.status == p3.ESTATE  # before reorder
    M.reorder()
    with pytest.raises(p3.Pars3Error) as e:
        M.diagonal()
    assert e.value.status == p3.ESTATE  # no diagonal array


@pytest.mark.parametrize("value_dtype", [p3.F64, p3.F32])
def test_workload1_full_size_symmetric_with_diagonal(value_dtype):
    """The 3D 128^3 benchmark matrix taken as symmetric with a diagonal, in
    the benchmark's launch configuration, every output against the oracle."""
    L = synth.workload(1)
    print(f"[gpu] symmetric workload1 dtype={value_dtype}", flush=True)
    d, M = make(L, True, True, seed=77)
    M.reorder(value_dtype=value_dtype, tile_rows=128)
    x = synth.vector(L.n, 1102)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    want = oracle_product(L, d, True, 0.5, x, value_dtype)
    assert rel_inf(gpu_spmv(M, 0.5, x, vec), want) <= TOL[value_dtype]
