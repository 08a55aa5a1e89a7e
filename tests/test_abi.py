"""The C-ABI library loads on the host and exports every declared symbol;
host-only validation agrees with the oracle's validation codes.  No device
work is started here."""
import glob
import os
import re

import numpy as np
import pytest

import oracle
import paper_2407_17651_amd as p3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(pars3_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(p3.LIB_PATH):
        import paper_2407_17651_amd.build as b
        b.build()
    return p3.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert "pars3_spmv" in names and "pars3_create" in names
    for name in names:
        assert hasattr(L, name), name
        assert name in p3.SIGNATURES, f"binding lacks {name}"


CASES = [
    (3, 3, [0, 0, 1, 3], [0, 0, 1]),
    (3, 3, [0, 0, 1, 3], [0, 1, 0]),
    (3, 3, [0, 0, 1, 3], [0, 1, 1]),
    (3, 3, [0, 0, 1, 3], [1, 0, 1]),
    (3, 3, [0, 0, 1, 3], [0, 0, 2]),
    (3, 3, [0, 0, 1, 3], [-1, 0, 1]),
    (3, 2, [0, 0, 1, 3], [0, 0, 1]),
    (3, 3, [0, 2, 1, 3], [0, 0, 1]),
    (0, 0, [0], []),
    (1, 0, [0, 0], []),
    (2, 0, [1, 0, 0], []),
]


@pytest.mark.parametrize("n,nnz,rowptr,col", CASES)
def test_validation_matches_oracle(L, n, nnz, rowptr, col):
    rp = np.array(rowptr, np.int32)
    c = np.array(col, np.int32) if col else None
    assert p3.pars3_validate(n, nnz, rp, c) == oracle.validate(n, nnz, rp, c)


def test_validation_negative_sizes(L):
    assert p3.pars3_validate(-1, 0, np.zeros(1, np.int32), None) == p3.EINVAL
    assert p3.pars3_validate(1, -1, np.zeros(2, np.int32), None) == p3.EINVAL
    assert p3.pars3_validate(1, 0, None, None) == p3.EINVAL
    assert "rowptr" in p3.pars3_last_error()


def test_validation_on_generated_inputs(L):
    import synth
    m = synth.rgg2d(3000, 8.0, 1)
    assert p3.pars3_validate(m.n, m.nnz, m.rowptr, m.col) == p3.OK
    bad = m.col.copy()
    r = int(np.flatnonzero(np.diff(m.rowptr) >= 2)[0])
    e = m.rowptr[r]
    bad[e], bad[e + 1] = bad[e + 1], bad[e]
    assert p3.pars3_validate(m.n, m.nnz, m.rowptr, bad) == p3.EUNSORTED


def test_split_params_default(L):
    p = p3.pars3_split_params_default()
    assert (p.w_in, p.t_out, p.tile_rows, p.permute, p.value_dtype, p.keep_fp64, p.engine) == \
        (-1, -1, 256, 1, p3.F64, 0, p3.ENGINE_TILES)


def test_binding_refuses_non_row_major_arrays():
    """A column selection of a row-major array is Fortran-ordered; the library
    reads row-major data, so the binding refuses it rather than pass a
    pointer to differently laid-out memory."""
    a = np.zeros((4, 3), np.float32)
    with pytest.raises(ValueError):
        p3._ptr(np.zeros((4, 41))[:, np.arange(41)])
    with pytest.raises(ValueError):
        p3._ptr(np.asfortranarray(a))
    assert p3._ptr(a) == a.ctypes.data and p3._ptr(np.zeros(0)) is None
