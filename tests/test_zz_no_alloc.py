"""The allocation-free product in the caller's numbering (pars3_spmv_noalloc)
against pars3_spmv with PARS3_ORDER_ORIGINAL on the same handle and vectors,
and against the oracle: two calls in a row, the second on a smaller input, in
FP64, FP32 and with 8 right-hand sides; the size limit; a captured graph."""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_17651_amd as p3
import synth
from gpu_util import rel_inf, to_dev

pytestmark = pytest.mark.gpu

LIMIT_PER_VECTOR = (64 << 20) // 2


def both(M, shift, X, k, vec):
    """Results of pars3_spmv_noalloc and of pars3_spmv (caller order)."""
    tdt = torch.float64 if vec == p3.F64 else torch.float32
    x = to_dev(X, tdt)
    y0 = torch.full_like(x, float("nan"))
    y1 = torch.full_like(x, float("nan"))
    p3.pars3_spmv_noalloc(M.h, shift, x, y1, k, vec)
    p3.pars3_spmv(M.h, shift, x, y0, k, vec, p3.ORDER_ORIGINAL)
    torch.cuda.synchronize()
    return y1.cpu().numpy().astype(np.float64), y0.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("value_dtype,k", [(p3.F64, 1), (p3.F32, 1), (p3.F64, 8), (p3.BF16, 8)])
def test_two_calls_second_smaller(value_dtype, k):
    vec = p3.F64 if value_dtype == p3.F64 else p3.F32
    tol = 1e-12 if vec == p3.F64 else 1e-5
    name = {p3.F64: "f64", p3.F32: "f32", p3.BF16: "bf16"}[value_dtype]
    for step, L in enumerate([synth.grid3d(30, 41, "normal"), synth.rgg2d(9000, 12.0, 42)]):
        print(f"[gpu] spmv_noalloc call {step} n={L.n} dtype={name} k={k}", flush=True)
        M = p3.Matrix(L).reorder(value_dtype=value_dtype)
        X = synth.vector(L.n, 43 + step, k) if k > 1 else synth.vector(L.n, 43 + step)
        Xr = X if vec == p3.F64 else X.astype(np.float32).astype(np.float64)
        got, ref = both(M, -0.625, X, k, vec)
        assert np.all(np.isfinite(got))
        assert rel_inf(got, ref) <= tol, step
        # the oracle works in the caller's numbering on the rounded values
        vals = oracle.rounded_values(L.val, name)
        Lv = type(L)(**{**L.__dict__, "val": vals})
        want = oracle.spmv(Lv, -0.625, Xr)
        assert rel_inf(got, want) <= tol, step
        M.close()


def test_integer_inputs_bit_exact():
    """Integer values and vectors: every partial sum is exact, so both entry
    points and the oracle agree bit for bit (second call on a smaller input)."""
    for step, L in enumerate([synth.grid3d(22, 7), synth.grid2d(31, 3)]):
        L = type(L)(**{**L.__dict__, "val": np.round(L.val * 8.0)})
        X = np.round(synth.vector(L.n, 8 + step) * 16.0)
        M = p3.Matrix(L).reorder()
        got, ref = both(M, 2.0, X, 1, p3.F64)
        want = oracle.spmv(L, 2.0, X)
        assert np.array_equal(got, ref) and np.array_equal(got, want), step
        M.close()


def test_size_limit():
    """n x k x 8 bytes above half of the 64 MiB array is refused (EINVAL) and
    changes nothing; the same handle still works within the limit."""
    side = 725  # 525,625 rows: 8 FP64 right-hand sides need 33.6 MB per vector
    L = synth.grid2d(side, 5)
    assert L.n * 8 * 8 > LIMIT_PER_VECTOR >= L.n * 1 * 8
    M = p3.Matrix(L).reorder()
    x = torch.zeros((L.n, 8), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_spmv_noalloc(M.h, 1.0, x, y, 8, p3.F64)
    assert e.value.status == p3.EINVAL and "limit" in str(e.value)
    X = synth.vector(L.n, 6)
    got, ref = both(M, 1.0, X, 1, p3.F64)
    assert rel_inf(got, ref) <= 1e-12
    assert rel_inf(got, oracle.spmv(L, 1.0, X)) <= 1e-12


def test_errors():
    L = synth.grid2d(20, 1)
    M = p3.Matrix(L)
    x = torch.zeros(L.n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_spmv_noalloc(M.h, 1.0, x, y, 1, p3.F64)
    assert e.value.status == p3.ESTATE
    M.reorder()
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_spmv_noalloc(M.h, 1.0, x, x, 1, p3.F64)
    assert e.value.status == p3.EINVAL
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_spmv_noalloc(M.h, 1.0, x, y, 3, p3.F64)
    assert e.value.status == p3.EINVAL


def test_in_a_graph():
    """Captured in a graph (no allocation, no wait); every replay, with eager
    work and synchronisations between them, matches the eager result and the
    oracle."""
    L = synth.rgg2d(15000, 10.0, 51)
    M = p3.Matrix(L).reorder()
    X = synth.vector(L.n, 52)
    x = to_dev(X)
    y = torch.full_like(x, float("nan"))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            p3.pars3_spmv_noalloc(M.h, 0.5, x, y, 1, p3.F64)
    torch.cuda.synchronize()
    want = oracle.spmv(L, 0.5, X)
    for r in range(4):
        y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        assert rel_inf(got, want) <= 1e-12, r
        other = synth.grid2d(40, r)  # eager work on the same array between replays
        Mo = p3.Matrix(other).reorder()
        Xo = synth.vector(other.n, 60 + r)
        go, _ = both(Mo, 1.0, Xo, 1, p3.F64)
        assert rel_inf(go, oracle.spmv(other, 1.0, Xo)) <= 1e-12
        Mo.close()
