"""Entry order inside the layout's tile-pair blocks.  pars3_reorder regroups
the entries of a block into aligned runs of 16 (a quarter of a wavefront's
LDS add) whose row offsets and column offsets fall into distinct LDS bank
classes (offset mod 32) where that pays,
so the product's LDS adds take fewer passes.  The split info reports the
passes of the sorted (diagonal) order, which must equal the oracle's count
exactly, and of the stored order, which is never worse; the products over a
regrouped layout match the oracle to the usual bars."""
import numpy as np
import pytest

import oracle
import paper_2407_17651_amd as p3
import synth
from gpu_util import gpu_spmv, oracle_reordered, rel_inf

pytestmark = pytest.mark.gpu

CASES = {
    "rgg2d_60000": lambda: synth.rgg2d(60000, 16.0, 31),
    "grid3d_30": lambda: synth.grid3d(30, 32, "normal"),
    "grid2d_200": lambda: synth.grid2d(200, 33),
    "chung_lu_20000": lambda: synth.chung_lu(20000, 16.0, 2.5, 34),
}


@pytest.mark.parametrize("tile_rows", [64, 256, 1024])
@pytest.mark.parametrize("name", sorted(CASES))
def test_sorted_order_passes_match_the_oracle(name, tile_rows):
    L = CASES[name]()
    print(f"[gpu] bank order {name} T={tile_rows}", flush=True)
    info = p3.Matrix(L).reorder(tile_rows=tile_rows, value_dtype=p3.F32).info()
    _, B = oracle_reordered(L)
    runs, passes = oracle.lds_passes_sorted(B, tile_rows)
    assert info["lds_runs"] == runs
    assert info["lds_passes_sorted"] == passes
    assert 2 * runs <= info["lds_passes"] <= passes


def test_irregular_blocks_take_fewer_passes():
    """Random geometric graphs leave sparse, scattered diagonals in a block:
    the regrouped order needs at least a fifth fewer passes."""
    info = p3.Matrix(CASES["rgg2d_60000"]()).reorder().info()
    print(f"[gpu] bank order rgg: {info['lds_passes']} of {info['lds_passes_sorted']} passes", flush=True)
    assert info["lds_passes"] <= 0.8 * info["lds_passes_sorted"]


def test_conflict_free_order_is_kept():
    """A path graph in its own numbering: every run is 16 consecutive rows of
    one diagonal, already at the floor of 2 passes, so nothing moves."""
    n = 256 * 5
    L = synth.from_edges(n, [(i, i + 1) for i in range(n - 1)], relabel=False, seed=5)
    info = p3.Matrix(L).reorder(permute=0).info()
    assert info["lds_passes"] == info["lds_passes_sorted"] == 2 * info["lds_runs"]


@pytest.mark.parametrize("tile_rows", [64, 256, 1024])
@pytest.mark.parametrize("k,value_dtype", [(1, p3.F64), (1, p3.BF16), (8, p3.F32), (8, p3.F64)])
def test_products_over_regrouped_blocks(k, value_dtype, tile_rows):
    """Element-wise against the oracle's full-CSR product, on a matrix whose
    blocks were regrouped (FP64 1e-12, FP32 and BF16 1e-5 relative)."""
    L = synth.rgg2d(40000, 16.0, 35)
    print(f"[gpu] bank order product k={k} dtype={value_dtype} T={tile_rows}", flush=True)
    _, B = oracle_reordered(L)
    M = p3.Matrix(L).reorder(value_dtype=value_dtype, tile_rows=tile_rows)
    info = M.info()
    assert info["lds_passes"] < info["lds_passes_sorted"]
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    X = synth.vector(L.n, 36, k) if k > 1 else synth.vector(L.n, 36)
    Xr = X if vec == p3.F64 else X.astype(np.float32).astype(np.float64)
    Bv = type(B)(**{**B.__dict__, "val": oracle.rounded_values(B.val, {0: "f64", 1: "f32", 2: "bf16"}[value_dtype])})
    got = gpu_spmv(M, 0.25, X, vec)
    assert rel_inf(got, oracle.spmv(Bv, 0.25, Xr)) <= (1e-12 if value_dtype == p3.F64 else 1e-5)
