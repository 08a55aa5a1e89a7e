"""Full-CSR comparison path: the GPU-built full CSR equals the oracle's full
CSR of S exactly, and both engines (own kernel, rocSPARSE) match the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_17651_amd as p3
import synth
from gpu_util import oracle_reordered, rel_inf, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("order", [p3.ORDER_RCM, p3.ORDER_ORIGINAL])
def test_full_csr_structure_exact(order):
    L = synth.rgg2d(5000, 10.0, 3)
    M = p3.Matrix(L).reorder()
    B = oracle_reordered(L)[1] if order == p3.ORDER_RCM else L
    C = p3.pars3_csr_create(M.h, order, p3.F64)
    rp, col, val = p3.pars3_csr_get(C, L.n, 2 * L.nnz)
    frow, fcol, fval = oracle.full_csr(B, 0.0)
    assert np.array_equal(rp, frow) and np.array_equal(col, fcol)
    assert np.array_equal(val, fval)
    p3.pars3_csr_destroy(C)


@pytest.mark.parametrize("engine", [0, 1])
@pytest.mark.parametrize("dtype", [p3.F64, p3.F32])
@pytest.mark.parametrize("name,maker", [("grid3d_24", lambda: synth.grid3d(24, 1, "normal")),
                                        ("chung_lu", lambda: synth.chung_lu(20000, 16.0, 2.5, 2))])
def test_full_csr_product(engine, dtype, name, maker):
    L = maker()
    print(f"[gpu] csr engine={engine} dtype={dtype} {name}", flush=True)
    M = p3.Matrix(L).reorder()
    perm, B = oracle_reordered(L)
    C = p3.pars3_csr_create(M.h, p3.ORDER_RCM, dtype)
    x = synth.vector(L.n, 4)
    tdt = torch.float64 if dtype == p3.F64 else torch.float32
    xd = to_dev(x, tdt)
    yd = torch.full_like(xd, float("nan"))
    shift = 0.0 if engine == 1 else 0.5
    p3.pars3_csr_spmv(C, shift, xd, yd, engine)
    torch.cuda.synchronize()
    Bv = type(B)(**{**B.__dict__, "val": oracle.rounded_values(B.val, "f64" if dtype == p3.F64 else "f32")})
    xr = x if dtype == p3.F64 else x.astype(np.float32).astype(np.float64)
    want = oracle.spmv(Bv, shift, xr)
    assert rel_inf(yd.cpu().numpy(), want) <= (1e-12 if dtype == p3.F64 else 1e-5)
    p3.pars3_csr_destroy(C)
