"""Batched products (one graph-captured launch over many matrices, one
workgroup per matrix tile, block right-hand sides) and batched MRS, against
the oracle per matrix.

Bars: as for single products (FP64 <= 1e-12, FP32 <= 1e-5 relative
infinity-norm against the oracle on the same rounded values and vectors);
every MRS solution has an oracle FP64 relative residual <= 1e-10."""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_17651_amd as p3
import synth
from gpu_util import rel_inf, to_dev

pytestmark = pytest.mark.gpu


def mixed_set(count, seed, n_lo=2000, n_hi=30000):
    specs = synth.batch_specs(count, seed, n_lo, n_hi)
    return specs, [synth.make(s, "uniform_f32") for s in specs]


TILES = (64, 128, 256, 512, 1024)


def reordered(Ls, value_dtype, keep=0, tiles=None):
    mats = []
    for i, L in enumerate(Ls):
        T = TILES[i % len(TILES)] if tiles is None else tiles
        mats.append(p3.Matrix(L).reorder(value_dtype=value_dtype, keep_fp64=keep, tile_rows=T,
                                         w_in=(i % 3 == 0) * 2))
    return mats


def oracle_product(L, shift, X, vec):
    B = oracle.permute(L, oracle.rcm(L))
    Xr = X if vec == p3.F64 else X.astype(np.float32).astype(np.float64)
    Bv = type(B)(**{**B.__dict__, "val": oracle.rounded_values(B.val, "f64" if vec == p3.F64 else "f32")})
    return oracle.spmv(Bv, shift, Xr)


@pytest.mark.parametrize("k,value_dtype", [(8, p3.F32), (1, p3.F64), (4, p3.F64), (2, p3.BF16)])
def test_batch_products_match_oracle(k, value_dtype):
    specs, Ls = mixed_set(12, 77 + k)
    print(f"[gpu] batch spmv k={k} dtype={value_dtype} sizes={[L.n for L in Ls]}", flush=True)
    mats = reordered(Ls, value_dtype)
    bat = p3.Batch(mats)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    tdt = torch.float64 if vec == p3.F64 else torch.float32
    Xs = [synth.vector(L.n, 100 + i, k) if k > 1 else synth.vector(L.n, 100 + i) for i, L in enumerate(Ls)]
    xs = [to_dev(X, tdt) for X in Xs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    shifts = np.array([s["alpha"] for s in specs])
    bat.spmv(xs, ys, shifts, k=k, vec_dtype=vec)
    bat.spmv(xs, ys, shifts, k=k, vec_dtype=vec)  # graph replay
    torch.cuda.synchronize()
    tol = 1e-12 if vec == p3.F64 else 1e-5
    if value_dtype == p3.BF16:
        tol = 1e-5
    for i, L in enumerate(Ls):
        B = oracle.permute(L, oracle.rcm(L))
        Xr = Xs[i] if vec == p3.F64 else Xs[i].astype(np.float32).astype(np.float64)
        kind = {p3.F64: "f64", p3.F32: "f32", p3.BF16: "bf16"}[value_dtype]
        Bv = type(B)(**{**B.__dict__, "val": oracle.rounded_values(B.val, kind)})
        want = oracle.spmv(Bv, shifts[i], Xr)
        assert rel_inf(ys[i].cpu().numpy().astype(np.float64), want) <= tol, i


@pytest.mark.parametrize("tiles", [128, 512])
def test_batch_of_one_entry_width(tiles):
    """Every matrix at one tile height: all 16-bit entry words (128 rows) or
    all 32-bit ones (512 rows), each served by its own kernel (the mixed set
    above takes the per-item choice)."""
    specs, Ls = mixed_set(6, 41 + tiles)
    print(f"[gpu] batch spmv one tile height T={tiles} sizes={[L.n for L in Ls]}", flush=True)
    mats = reordered(Ls, p3.F32, tiles=tiles)
    bat = p3.Batch(mats)
    Xs = [synth.vector(L.n, 300 + i, 8) for i, L in enumerate(Ls)]
    xs = [to_dev(X, torch.float32) for X in Xs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    shifts = np.array([s["alpha"] for s in specs])
    bat.spmv(xs, ys, shifts, k=8, vec_dtype=p3.F32)
    torch.cuda.synchronize()
    for i, L in enumerate(Ls):
        want = oracle_product(L, shifts[i], Xs[i], p3.F32)
        assert rel_inf(ys[i].cpu().numpy().astype(np.float64), want) <= 1e-5, i


def test_batch_rejects_a_matrix_split_again():
    """The work list and LDS size of a batch come from the layouts at its
    creation; a matrix split again afterwards (here to taller tiles) is
    refused before any launch."""
    L = synth.grid2d(40, 3)
    M = p3.Matrix(L).reorder(tile_rows=128)
    bat = p3.Batch([M])
    x = to_dev(synth.vector(L.n, 1))
    y = torch.empty_like(x)
    bat.spmv([x], [y], np.array([0.5]))
    torch.cuda.synchronize()
    M.reorder(tile_rows=512)
    with pytest.raises(p3.Pars3Error) as e:
        bat.spmv([x], [y], np.array([0.5]))
    assert e.value.status == p3.ESTATE
    b = to_dev(np.ones(L.n))
    with pytest.raises(p3.Pars3Error) as e:
        bat.mrs([1.0], [b], [torch.zeros_like(b)])
    assert e.value.status == p3.ESTATE


def test_batch_recapture_on_new_pointers_and_shifts():
    specs, Ls = mixed_set(6, 5)
    mats = reordered(Ls, p3.F64)
    bat = p3.Batch(mats)
    xs = [to_dev(synth.vector(L.n, i)) for i, L in enumerate(Ls)]
    y1 = [torch.empty_like(x) for x in xs]
    y2 = [torch.empty_like(x) for x in xs]
    bat.spmv(xs, y1, np.ones(6))
    bat.spmv(xs, y2, np.full(6, -2.0))
    bat.spmv(xs, y1, np.ones(6))
    torch.cuda.synchronize()
    for i, L in enumerate(Ls):
        x = xs[i].cpu().numpy()
        B = oracle.permute(L, oracle.rcm(L))
        assert rel_inf(y1[i].cpu().numpy(), oracle.spmv(B, 1.0, x)) <= 1e-12
        assert rel_inf(y2[i].cpu().numpy(), oracle.spmv(B, -2.0, x)) <= 1e-12


def test_batch_queues_cover_every_item():
    specs, Ls = mixed_set(20, 9)
    mats = reordered(Ls, p3.F64)
    bat = p3.Batch(mats)
    info = bat.info()
    q = info["queues"]
    assert q[0] == 0 and q[8] == info["n_items"] and np.all(np.diff(q) >= 0)
    assert info["n_items"] == sum(m.info()["n_tiles"] for m in mats)
    assert info["grid"] == 8 * max(int(np.diff(q).max()), 1)


def test_batch_with_empty_and_tiny_matrices():
    Ls = [synth.grid2d(30, 1), synth.from_edges(1, [], seed=1), synth.from_edges(2, [(1, 0)], seed=2),
          synth.rgg2d(3000, 8.0, 3)]
    mats = [p3.Matrix(L).reorder() for L in Ls]
    bat = p3.Batch(mats)
    xs = [to_dev(synth.vector(L.n, 7 + i)) for i, L in enumerate(Ls)]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    bat.spmv(xs, ys, np.full(4, 0.25))
    torch.cuda.synchronize()
    for i, L in enumerate(Ls):
        B = oracle.permute(L, oracle.rcm(L))
        assert rel_inf(ys[i].cpu().numpy(), oracle.spmv(B, 0.25, xs[i].cpu().numpy())) <= 1e-12


@pytest.mark.parametrize("order", [p3.ORDER_ORIGINAL, p3.ORDER_RCM])
def test_batch_mrs_converges_per_system(order):
    specs, Ls = mixed_set(10, 31, 2000, 20000)
    alphas = np.array([s["alpha"] for s in specs])
    print(f"[gpu] batch mrs order={order} alphas={alphas.round(2).tolist()}", flush=True)
    mats = reordered(Ls, p3.F32, keep=1)
    bat = p3.Batch(mats)
    bs, xs, bh = [], [], []
    for i, L in enumerate(Ls):
        b = oracle.spmv(L, alphas[i], np.ones(L.n))
        if order == p3.ORDER_RCM:
            b = b[oracle.rcm(L)]
        bh.append(b)
        bs.append(to_dev(b))
        xs.append(torch.zeros(L.n, dtype=torch.float64, device="cuda"))
    st, infos = bat.mrs(alphas, bs, xs, order=order, tol=1e-10, maxit=5000)
    torch.cuda.synchronize()
    assert st == p3.OK, infos
    for i, L in enumerate(Ls):
        x = xs[i].cpu().numpy()
        if order == p3.ORDER_RCM:
            perm = oracle.rcm(L)
            xo = np.empty_like(x)
            xo[perm] = x
            b = np.empty_like(bh[i])
            b[perm] = bh[i]
        else:
            xo, b = x, bh[i]
        res = oracle.residual(L, alphas[i], b, xo)
        assert res <= 1e-10, (i, res, infos[i])
        assert abs(res - infos[i]["relres"]) <= 1e-3 * res + 1e-15
        _, io, _ = oracle.mrs(L, alphas[i], b, tol=1e-10, maxit=5000)
        assert abs(infos[i]["iters"] - io["iters"]) <= 2 + io["iters"] // 100, (i, infos[i]["iters"], io["iters"])


def test_batch_mrs_matches_single_solves():
    specs, Ls = mixed_set(5, 41, 3000, 8000)
    alphas = np.array([s["alpha"] for s in specs])
    mats = reordered(Ls, p3.F64, tiles=256)
    bat = p3.Batch(mats)
    bs = [to_dev(oracle.spmv(L, alphas[i], synth.vector(L.n, i))) for i, L in enumerate(Ls)]
    xs = [torch.zeros(L.n, dtype=torch.float64, device="cuda") for L in Ls]
    st, infos = bat.mrs(alphas, bs, xs, order=p3.ORDER_ORIGINAL, tol=1e-11, maxit=3000)
    assert st == p3.OK
    for i, M in enumerate(mats):
        x1 = torch.zeros_like(xs[i])
        st1, info1, _ = M.mrs(alphas[i], bs[i], x1, order=p3.ORDER_ORIGINAL, tol=1e-11, maxit=3000)
        assert abs(info1["iters"] - infos[i]["iters"]) <= 1
        assert rel_inf(xs[i].cpu().numpy(), x1.cpu().numpy()) <= 1e-9


def test_batch_errors():
    L = synth.grid2d(10, 1)
    with pytest.raises(p3.Pars3Error) as e:
        p3.Batch([p3.Matrix(L)])
    assert e.value.status == p3.ESTATE
    bat = p3.Batch([p3.Matrix(L).reorder()])
    b = to_dev(np.ones(L.n))
    x = to_dev(np.zeros(L.n))
    with pytest.raises(p3.Pars3Error) as e:
        bat.mrs([1.0], [b], [x], precision=p3.F32)
    assert e.value.status == p3.EINVAL
    with pytest.raises(p3.Pars3Error) as e:
        bat.spmv([x], [b], k=3)
    assert e.value.status == p3.EINVAL
    with pytest.raises(p3.Pars3Error) as e:
        bat.spmv([x], [b], vec_dtype=p3.F32)  # FP64 values only
    assert e.value.status == p3.ESTATE


@pytest.fixture(scope="module")
def full_batch():
    """The 256-matrix workload (n log-uniform in [2k, 200k], 2D/3D stencils
    and random geometric graphs, FP32-representable values), the oracle's
    reordering of each matrix, and k = 8 FP32 right-hand sides."""
    specs = synth.batch_specs(256)
    Ls = [synth.make(s, "uniform_f32") for s in specs]
    Bs = [oracle.permute(L, oracle.rcm(L)) for L in Ls]
    Xs = [synth.vector(L.n, 500 + i, 8).astype(np.float32) for i, L in enumerate(Ls)]
    return specs, Ls, Bs, Xs


@pytest.mark.parametrize("tiles", [256, 512])
def test_batched_workload_full_size(full_batch, tiles):
    """The whole 256-matrix workload in one launch with k = 8 FP32
    right-hand sides, at 256-row tiles (16-bit entry words) and at 512-row
    tiles (32-bit words, the benchmark's configuration): every output of
    every matrix against the oracle on the same rounded values and vectors."""
    specs, Ls, Bs, Xs = full_batch
    print(f"[gpu] batch full size T={tiles} sum_n={sum(L.n for L in Ls)} sum_nnz={sum(L.nnz for L in Ls)}",
          flush=True)
    mats = [p3.Matrix(L).reorder(value_dtype=p3.F32, keep_fp64=1, tile_rows=tiles) for L in Ls]
    bat = p3.Batch(mats)
    xs = [to_dev(X, torch.float32) for X in Xs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    shifts = np.array([s["alpha"] for s in specs])
    bat.spmv(xs, ys, shifts, k=8, vec_dtype=p3.F32)
    bat.spmv(xs, ys, shifts, k=8, vec_dtype=p3.F32)  # graph replay
    torch.cuda.synchronize()
    worst = 0.0
    for i, L in enumerate(Ls):
        Bv = type(Bs[i])(**{**Bs[i].__dict__, "val": oracle.rounded_values(Bs[i].val, "f32")})
        want = oracle.spmv(Bv, shifts[i], Xs[i].astype(np.float64))
        err = rel_inf(ys[i].cpu().numpy().astype(np.float64), want)
        worst = max(worst, err)
        assert err <= 1e-5, (i, L.n, err)
    print(f"[gpu] batch full size T={tiles} worst rel err {worst:.3e}", flush=True)


def test_batched_mrs_full_size_every_system(full_batch):
    """The benchmark's 256 batched FP64 MRS solves (alpha_i in [0.1, 2],
    b_i = A_i 1, x0 = 0, tolerance 1e-10): the oracle recomputes every
    system's FP64 relative residual from the returned x."""
    specs, Ls, Bs, Xs = full_batch
    alphas = np.array([s["alpha"] for s in specs])
    print(f"[gpu] batch mrs full size alpha in [{alphas.min():.3f}, {alphas.max():.3f}]", flush=True)
    mats = [p3.Matrix(L).reorder(value_dtype=p3.F32, keep_fp64=1, tile_rows=256) for L in Ls]
    bat = p3.Batch(mats)
    bh = [oracle.spmv(L, alphas[i], np.ones(L.n)) for i, L in enumerate(Ls)]
    bs = [to_dev(b) for b in bh]
    xs = [torch.zeros(L.n, dtype=torch.float64, device="cuda") for L in Ls]
    st, infos = bat.mrs(alphas, bs, xs, order=p3.ORDER_ORIGINAL, tol=1e-10, maxit=20000)
    assert st == p3.OK
    worst = 0.0
    for i, L in enumerate(Ls):
        res = oracle.residual(L, alphas[i], bh[i], xs[i].cpu().numpy())
        worst = max(worst, res)
        assert res <= 1e-10, (i, L.n, alphas[i], res, infos[i])
        assert infos[i]["status"] == 0
    print(f"[gpu] batch mrs full size worst oracle residual {worst:.3e}, "
          f"iterations max {max(i['iters'] for i in infos)}", flush=True)


def test_batched_mrs_nan_system_reports_enan():
    """One system with a NaN in b among converging ones: that system ends
    with status 3 and the batch returns ENAN; the others still converge."""
    specs, Ls = mixed_set(4, 91, 3000, 8000)
    alphas = np.array([s["alpha"] for s in specs])
    mats = reordered(Ls, p3.F64, tiles=256)
    bat = p3.Batch(mats)
    bh = [oracle.spmv(L, alphas[i], np.ones(L.n)) for i, L in enumerate(Ls)]
    bh[2][5] = np.nan
    bs = [to_dev(b) for b in bh]
    xs = [torch.zeros(L.n, dtype=torch.float64, device="cuda") for L in Ls]
    st, infos = bat.mrs(alphas, bs, xs, check=False, order=p3.ORDER_ORIGINAL, tol=1e-10, maxit=3000)
    assert st == p3.ENAN
    assert infos[2]["status"] == 3
    for i in (0, 1, 3):
        assert infos[i]["status"] == 0
        assert oracle.residual(Ls[i], alphas[i], bh[i], xs[i].cpu().numpy()) <= 1e-10


@pytest.mark.parametrize("k,value_dtype", [(8, p3.F32), (1, p3.F64)])
def test_batch_autotune_leaves_the_fastest_height(k, value_dtype):
    """pars3_batch_autotune times whole batch launches per tile height, leaves
    every handle split with the fastest, and a batch made then multiplies as
    the oracle does."""
    specs, Ls = mixed_set(10, 91 + k)
    print(f"[gpu] batch autotune k={k} dtype={value_dtype}", flush=True)
    mats = reordered(Ls, value_dtype, tiles=256)
    heights = (128, 256, 512)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    us, best = p3.pars3_batch_autotune(mats, heights, k=k, vec_dtype=vec, reps=5)
    assert us.shape == (3,) and np.all(us > 0) and best == int(np.argmin(us))
    for M in mats:
        assert M.info()["tile_rows"] == heights[best]
        assert M.info()["value_dtype"] == value_dtype
    bat = p3.Batch(mats)
    tdt = torch.float64 if vec == p3.F64 else torch.float32
    Xs = [synth.vector(L.n, 300 + i, k) if k > 1 else synth.vector(L.n, 300 + i) for i, L in enumerate(Ls)]
    xs = [to_dev(X, tdt) for X in Xs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    shifts = np.array([s["alpha"] for s in specs])
    bat.spmv(xs, ys, shifts, k=k, vec_dtype=vec)
    torch.cuda.synchronize()
    tol = 1e-12 if vec == p3.F64 else 1e-5
    for i, L in enumerate(Ls):
        got = ys[i].double().cpu().numpy()
        assert rel_inf(got, oracle_product(L, shifts[i], Xs[i], vec)) <= tol


def test_batch_autotune_errors():
    Ls = [synth.grid2d(30, 1), synth.grid2d(20, 2)]
    mats = [p3.Matrix(L).reorder() for L in Ls]
    for kw in (dict(tile_rows=(100,)), dict(k=3), dict(vec_dtype=p3.BF16), dict(reps=0), dict(tile_rows=())):
        with pytest.raises(p3.Pars3Error) as e:
            p3.pars3_batch_autotune(mats, **kw)
        assert e.value.status == p3.EINVAL, kw
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_batch_autotune(mats + [p3.Matrix(synth.grid2d(10, 3))])
    assert e.value.status == p3.ESTATE
    # a batch made before the call sees the re-split (another tile height)
    bat = p3.Batch(mats)
    p3.pars3_batch_autotune(mats, (128,), reps=1)
    x = [torch.zeros(L.n, dtype=torch.float64, device="cuda") for L in Ls]
    with pytest.raises(p3.Pars3Error) as e:
        bat.spmv(x, [torch.empty_like(v) for v in x])
    assert e.value.status == p3.ESTATE
