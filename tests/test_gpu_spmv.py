"""GPU skew-symmetric product against the oracle's full-CSR FP64 product.

Bars: FP64 <= 1e-12, FP32 <= 1e-5 and BF16 <= 1e-5 relative infinity-norm error
against the oracle run on the same rounded values and vectors; integer-valued
inputs bit-exact in every precision (every partial sum is an exact integer)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_17651_amd as p3
import synth
from gpu_util import gpu_spmv, oracle_reordered, rel_inf, to_dev

pytestmark = pytest.mark.gpu

TOL = {p3.F64: 1e-12, p3.F32: 1e-5, p3.BF16: 1e-5}


def check_product(L, shift=0.5, k=1, value_dtype=p3.F64, seed=11, **params):
    perm, B = oracle_reordered(L) if params.get("permute", 1) else (None, L)
    M = p3.Matrix(L).reorder(value_dtype=value_dtype, **params)
    x = synth.vector(L.n, seed, k)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    xr = x if vec == p3.F64 else x.astype(np.float32).astype(np.float64)
    Bv = type(B)(**{**B.__dict__, "val": oracle.rounded_values(B.val, {0: "f64", 1: "f32", 2: "bf16"}[value_dtype])})
    want = oracle.spmv(Bv, shift, xr)
    got = gpu_spmv(M, shift, x, vec)
    err = rel_inf(got, want)
    assert err <= TOL[value_dtype], err
    return M, err


@pytest.mark.parametrize("name,maker", [
    ("workload0", lambda: synth.workload(0)),
    ("grid3d_20", lambda: synth.grid3d(20, 3, "normal")),
    ("rgg_30000", lambda: synth.rgg2d(30000, 16.0, 4)),
    ("chung_lu_20000", lambda: synth.chung_lu(20000, 16.0, 2.5, 5)),
    ("pieces", lambda: synth.from_edges(40, [(i, i + 1) for i in range(0, 38, 3)], relabel=True, seed=3)),
    ("star_hub", lambda: synth.from_edges(3000, [(0, i) for i in range(1, 3000)] + [(i, i + 1) for i in range(1, 2999)],
                                         relabel=True, seed=4)),
])
@pytest.mark.parametrize("value_dtype", [p3.F64, p3.F32, p3.BF16])
def test_product_parity(name, maker, value_dtype):
    print(f"[gpu] spmv {name} dtype={value_dtype}", flush=True)
    check_product(maker(), value_dtype=value_dtype)


@pytest.mark.parametrize("params", [
    dict(tile_rows=64), dict(tile_rows=128), dict(tile_rows=512), dict(tile_rows=1024),
    dict(w_in=4), dict(w_in=16, t_out=40), dict(t_out=5), dict(w_in=0, t_out=0), dict(w_in=64), dict(permute=0),
])
def test_layout_variants(params):
    print(f"[gpu] spmv layout {params}", flush=True)
    check_product(synth.rgg2d(20000, 12.0, 8), shift=-0.25, **params)


@pytest.mark.parametrize("value_dtype", [p3.F64, p3.F32, p3.BF16])
@pytest.mark.parametrize("params", [dict(), dict(w_in=3), dict(t_out=2), dict(tile_rows=64), dict(tile_rows=512),
                                    dict(tile_rows=1024)])
def test_integer_inputs_bit_exact(value_dtype, params):
    """Values and x in {-4..4}: exact in every precision and summation order.
    Tiles of up to 256 rows store 16-bit entry words, taller ones 32-bit
    words; n = 8000 leaves a ragged last tile for every height."""
    L = synth.rgg2d(8000, 10.0, 12, "int4")
    print(f"[gpu] spmv integer dtype={value_dtype} {params}", flush=True)
    perm, B = oracle_reordered(L)
    M = p3.Matrix(L).reorder(value_dtype=value_dtype, **params)
    x = np.floor(synth.vector(L.n, 3) * 4.999)
    want = oracle.spmv(B, 2.0, x)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    got = gpu_spmv(M, 2.0, x, vec)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("k", [2, 4, 8])
@pytest.mark.parametrize("value_dtype", [p3.F64, p3.F32])
def test_block_right_hand_sides(k, value_dtype):
    L = synth.grid3d(16, 21, "normal")
    print(f"[gpu] spmv k={k} dtype={value_dtype}", flush=True)
    perm, B = oracle_reordered(L)
    M = p3.Matrix(L).reorder(value_dtype=value_dtype)
    X = synth.vector(L.n, 5, k)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    Xr = X if vec == p3.F64 else X.astype(np.float32).astype(np.float64)
    Bv = type(B)(**{**B.__dict__, "val": oracle.rounded_values(B.val, "f64" if vec == p3.F64 else "f32")})
    want = oracle.spmv(Bv, 0.75, Xr)
    got = gpu_spmv(M, 0.75, X, vec)
    assert rel_inf(got, want) <= TOL[value_dtype]
    # each column equals the single right-hand-side product
    for c in range(k):
        one = gpu_spmv(M, 0.75, np.ascontiguousarray(X[:, c]), vec)
        assert rel_inf(got[:, c], one) <= TOL[value_dtype]


@pytest.mark.parametrize("value_dtype", [p3.F64, p3.F32])
@pytest.mark.parametrize("tile_rows,k", [(1024, 8), (512, 8), (64, 8)])
def test_block_right_hand_sides_tile_sizes(tile_rows, k, value_dtype):
    """Largest LDS accumulator (1024 rows x 8 right-hand sides in FP64) and
    the smallest tiles, with 32-bit (1024, 512) and 16-bit (64) entry words;
    8 right-hand sides take the gathers of a group in parts."""
    L = synth.rgg2d(30000, 12.0, 17)
    print(f"[gpu] spmv tile_rows={tile_rows} k={k} dtype={value_dtype}", flush=True)
    perm, B = oracle_reordered(L)
    M = p3.Matrix(L).reorder(tile_rows=tile_rows, value_dtype=value_dtype)
    X = synth.vector(L.n, 6, k)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    Xr = X if vec == p3.F64 else X.astype(np.float32).astype(np.float64)
    Bv = type(B)(**{**B.__dict__, "val": oracle.rounded_values(B.val, "f64" if vec == p3.F64 else "f32")})
    got = gpu_spmv(M, -0.5, X, vec)
    assert rel_inf(got, oracle.spmv(Bv, -0.5, Xr)) <= TOL[value_dtype]


def test_misaligned_block_vectors_rejected():
    L = synth.grid2d(20, 1)
    M = p3.Matrix(L).reorder()
    buf = torch.zeros(2 * L.n + 1, dtype=torch.float64, device="cuda")
    y = torch.zeros(2 * L.n, dtype=torch.float64, device="cuda")
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_spmv(M.h, 0.0, buf[1:], y, 2, p3.F64, p3.ORDER_RCM)
    assert e.value.status == p3.EINVAL
    p3.pars3_spmv(M.h, 0.0, buf[1:1 + L.n], y[:L.n], 1, p3.F64, p3.ORDER_RCM)  # k = 1: any alignment


def test_original_order():
    L = synth.rgg2d(10000, 10.0, 14)
    M = p3.Matrix(L).reorder()
    x = synth.vector(L.n, 8)
    got = gpu_spmv(M, 1.5, x, p3.F64, p3.ORDER_ORIGINAL)
    assert rel_inf(got, oracle.spmv(L, 1.5, x)) <= 1e-12


def test_worked_example():
    """Section 3.1.2, eqs. (2)-(6): only A30 stored."""
    L = synth.Lower(4, np.array([0, 0, 0, 0, 1], np.int32), np.array([0], np.int32), np.array([2.5]))
    M = p3.Matrix(L).reorder(permute=0)
    got = gpu_spmv(M, 0.0, np.array([3.0, -1.0, 7.0, -2.0]))
    assert got.tolist() == [5.0, 0.0, 0.0, 7.5]


def test_degenerate_sizes():
    for L in (synth.from_edges(1, []), synth.from_edges(6, []), synth.Lower(0, np.zeros(1, np.int32),
                                                                              np.zeros(0, np.int32), np.zeros(0))):
        M = p3.Matrix(L).reorder()
        if L.n:
            x = synth.vector(L.n, 1)
            assert np.array_equal(gpu_spmv(M, 0.5, x), 0.5 * x)


def test_errors():
    L = synth.grid2d(8, 1)
    M = p3.Matrix(L)
    x = to_dev(np.ones(L.n))
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_spmv(M.h, 0.0, x, x.clone(), 1, p3.F64, p3.ORDER_RCM)
    assert e.value.status == p3.ESTATE
    M.reorder()
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_spmv(M.h, 0.0, x, x, 1, p3.F64, p3.ORDER_RCM)
    assert e.value.status == p3.EINVAL
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_spmv(M.h, 0.0, x, x.clone(), 3, p3.F64, p3.ORDER_RCM)
    assert e.value.status == p3.EINVAL
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_spmv(M.h, 0.0, x.float(), x.float().clone(), 1, p3.F32, p3.ORDER_RCM)
    assert e.value.status == p3.ESTATE
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_create(3, 1, np.array([0, 0, 0, 1], np.int32), np.array([2], np.int32), np.ones(1))
    assert e.value.status == p3.ENOTLOWER


def test_workload1_full_size_fp64():
    """The benchmark workload (3D 128^3, N(0,1) values) in the benchmark's
    launch configuration, every output compared with the oracle."""
    L = synth.workload(1)
    print("[gpu] spmv workload1 fp64", flush=True)
    M, err = check_product(L, shift=0.5, value_dtype=p3.F64, seed=1101)
    print(f"[gpu] workload1 fp64 rel err {err:.3e}", flush=True)


@pytest.mark.parametrize("value_dtype", [p3.F32, p3.BF16])
def test_workload1_full_size_low_precision(value_dtype):
    """The benchmark workload with FP32 and BF16 stored values (FP32 vectors),
    every output against the oracle run on the same rounded values and
    vectors."""
    L = synth.workload(1)
    print(f"[gpu] spmv workload1 dtype={value_dtype}", flush=True)
    M, err = check_product(L, shift=0.5, value_dtype=value_dtype, seed=1101)
    print(f"[gpu] workload1 dtype={value_dtype} rel err {err:.3e}", flush=True)


@pytest.mark.parametrize("k", [1, 8])
def test_original_order_in_a_graph(k):
    """A product in the caller's numbering (gather, product, scatter) captured
    in a graph: the call neither allocates nor waits, so capture succeeds on
    a handle's first such call, and every replay, with eager work and
    synchronisations between them, equals the eager result and the oracle."""
    L = synth.rgg2d(12000, 10.0, 31)
    M = p3.Matrix(L).reorder()
    X = synth.vector(L.n, 9, k) if k > 1 else synth.vector(L.n, 9)
    x = to_dev(X)
    y = torch.full_like(x, float("nan"))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            p3.pars3_spmv(M.h, 0.75, x, y, k, p3.F64, p3.ORDER_ORIGINAL)
    torch.cuda.synchronize()
    want = oracle.spmv(L, 0.75, X)
    eager = gpu_spmv(M, 0.75, X, p3.F64, p3.ORDER_ORIGINAL)
    assert rel_inf(eager, want) <= 1e-12
    for r in range(4):
        y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        # the LDS sums may add in another order from run to run
        assert rel_inf(got, eager) <= 1e-12 and rel_inf(got, want) <= 1e-12, r
        _ = gpu_spmv(M, -1.0, X, p3.F64, p3.ORDER_RCM)  # eager work between replays


@pytest.fixture(scope="module")
def workload2():
    L = synth.workload(2)
    return L, oracle.permute(L, oracle.rcm(L))


@pytest.mark.parametrize("value_dtype", [p3.F64, p3.F32])
def test_workload2_full_size(workload2, value_dtype):
    """Random geometric graph, n = 4M, mean degree 16, in full: every output
    against the oracle."""
    L, B = workload2
    print(f"[gpu] spmv workload2 n={L.n} nnz={L.nnz} dtype={value_dtype}", flush=True)
    M = p3.Matrix(L).reorder(value_dtype=value_dtype)
    x = synth.vector(L.n, 12)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    xr = x if vec == p3.F64 else x.astype(np.float32).astype(np.float64)
    Bv = type(B)(**{**B.__dict__, "val": oracle.rounded_values(B.val, "f64" if vec == p3.F64 else "f32")})
    want = oracle.spmv(Bv, 0.25, xr)
    assert rel_inf(gpu_spmv(M, 0.25, x, vec), want) <= TOL[value_dtype]


def test_profiling_counters():
    L = synth.grid3d(20, 2)
    M = p3.Matrix(L).reorder()
    x = to_dev(synth.vector(L.n, 1))
    y = torch.empty_like(x)
    p3.pars3_set_profiling(M.h, True)
    for _ in range(3):
        p3.pars3_spmv(M.h, 0.5, x, y, 1, p3.F64, p3.ORDER_RCM)
    pr = p3.pars3_get_profile(M.h)
    assert pr["calls"] == 3 and pr["ms_band"] > 0 and pr["ms_fixup"] == 0
    p3.pars3_spmv(M.h, 0.5, x, y, 1, p3.F64, p3.ORDER_ORIGINAL)
    pr = p3.pars3_get_profile(M.h)
    assert pr["calls"] == 1 and pr["ms_band"] > 0 and pr["ms_fixup"] > 0
    assert p3.pars3_get_profile(M.h)["calls"] == 0  # reset by the read
    p3.pars3_set_profiling(M.h, False)
    p3.pars3_spmv(M.h, 0.5, x, y, 1, p3.F64, p3.ORDER_RCM)
    assert p3.pars3_get_profile(M.h)["calls"] == 0
