"""Autotuner: every configuration of the grid is applied and timed, the
fastest is reported and left applied, and the product stays exact against the
oracle under every configuration the tuner tried."""
import numpy as np
import pytest

import oracle
import paper_2407_17651_amd as p3
import synth
from gpu_util import gpu_spmv, oracle_reordered, rel_inf

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("value_dtype", [p3.F64, p3.F32, p3.BF16])
def test_default_grid(value_dtype):
    """40 tile configurations, then the full-CSR engine (FP64 and FP32 values
    only)."""
    g = p3.pars3_tune_grid_default(value_dtype)
    tiles = [c for c in g if c.engine == p3.ENGINE_TILES]
    assert len(tiles) == 40
    assert {(c.tile_rows, c.w_in, c.t_out) for c in tiles} == {
        (T, w, t) for T in (64, 128, 256, 512, 1024) for w in (0, 1, 2, 4) for t in (-1, -2)}
    if value_dtype == p3.BF16:
        assert len(g) == 40
    else:
        assert len(g) == 41 and g[40].engine == p3.ENGINE_CSR and g[40].value_dtype == value_dtype


@pytest.mark.parametrize("value_dtype", [p3.F64, p3.F32, p3.BF16])
def test_autotune_picks_fastest_and_leaves_it_applied(value_dtype):
    L = synth.rgg2d(40000, 12.0, 3)
    print(f"[gpu] autotune rgg dtype={value_dtype}", flush=True)
    M = p3.Matrix(L)
    res, best = p3.pars3_autotune(M.h, k=1, reps=5, value_dtype=value_dtype)
    us = np.array([r["us"] for r in res])
    assert np.all(us > 0) and best == int(np.argmin(us))
    info = M.info()
    beta = info["beta"]
    for r in res:
        assert r["t_out"] in (max(beta - 3, 0, r["w_in"]), max(beta // 2, r["w_in"]))
    b = res[best]
    assert (info["tile_rows"], info["w_in"], info["t_out"], info["value_dtype"]) == (
        b["tile_rows"], b["w_in"], b["t_out"], value_dtype)
    # the product under the applied configuration
    _, B = oracle_reordered(L)
    x = synth.vector(L.n, 2)
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    xr = x if vec == p3.F64 else x.astype(np.float32).astype(np.float64)
    kind = {p3.F64: "f64", p3.F32: "f32", p3.BF16: "bf16"}[value_dtype]
    Bv = type(B)(**{**B.__dict__, "val": oracle.rounded_values(B.val, kind)})
    assert rel_inf(gpu_spmv(M, 0.5, x, vec), oracle.spmv(Bv, 0.5, xr)) <= (1e-12 if vec == p3.F64 else 1e-5)


def test_autotune_every_config_is_exact():
    L = synth.grid3d(14, 4, "normal")
    _, B = oracle_reordered(L)
    x = synth.vector(L.n, 3)
    want = oracle.spmv(B, 0.5, x)
    M = p3.Matrix(L)
    res, _ = p3.pars3_autotune(M.h, k=2, reps=2)
    for r in res:
        M.reorder(tile_rows=r["tile_rows"], w_in=r["w_in"], t_out=r["t_out"])
        assert rel_inf(gpu_spmv(M, 0.5, x), want) <= 1e-12, r


def test_autotune_tiny_bandwidth_raises_t_out():
    L = synth.from_edges(50, [(i + 1, i) for i in range(49)], seed=1)  # beta = 1 after RCM
    M = p3.Matrix(L)
    res, best = p3.pars3_autotune(M.h, reps=2)
    assert all(r["t_out"] >= r["w_in"] for r in res)
    assert all(r["us"] > 0 for r in res)


def test_autotune_errors():
    M = p3.Matrix(synth.grid2d(8, 1))
    g = p3.pars3_tune_grid_default()
    with pytest.raises(p3.Pars3Error):
        p3.pars3_autotune(M.h, grid=g, k=3)
    with pytest.raises(p3.Pars3Error):
        p3.pars3_autotune(M.h, grid=g, reps=0)
