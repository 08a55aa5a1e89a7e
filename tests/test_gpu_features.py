"""GPU sparsity features against the oracle's, bit-exact: every feature is a
ratio of integer counts formed by the same FP64 operations."""
import numpy as np
import pytest

import oracle
import paper_2407_17651_amd as p3
import synth

pytestmark = pytest.mark.gpu

GRAPHS = {
    "workload0": lambda: synth.workload(0),
    "grid3d_20": lambda: synth.grid3d(20, 3, "normal"),
    "rgg_50000": lambda: synth.rgg2d(50000, 16.0, 4),
    "chung_lu_30000": lambda: synth.chung_lu(30000, 12.0, 2.5, 5),
    "pieces": lambda: synth.from_edges(40, [(i, i + 1) for i in range(0, 38, 3)], relabel=True, seed=3),
    "no_edges": lambda: synth.from_edges(300, [], seed=1),
    "single": lambda: synth.from_edges(1, [], seed=1),
    "star": lambda: synth.from_edges(700, [(0, i) for i in range(1, 700)], relabel=True, seed=2),
    "path_1000": lambda: synth.from_edges(1000, [(i + 1, i) for i in range(999)], relabel=True, seed=5),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_features_bit_exact(name):
    L = GRAPHS[name]()
    print(f"[gpu] features {name} n={L.n}", flush=True)
    M = p3.Matrix(L).reorder()
    B = oracle.permute(L, oracle.rcm(L))
    got = M.features()
    want = oracle.features(B)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), np.flatnonzero(got != want)


def test_features_keep_order_and_workload1():
    L = synth.grid2d(50, 2)
    M = p3.Matrix(L).reorder(permute=0)
    assert np.array_equal(M.features(), oracle.features(L))
    L = synth.workload(1)
    M = p3.Matrix(L).reorder()
    assert np.array_equal(M.features(), oracle.features(oracle.permute(L, oracle.rcm(L))))


def test_features_before_reorder_is_an_error():
    M = p3.Matrix(synth.grid2d(5, 1))
    with pytest.raises(p3.Pars3Error) as e:
        M.features()
    assert e.value.status == p3.ESTATE


def _rows_lower(n, rc):
    rowptr = np.zeros(n + 1, np.int32)
    for r, _ in rc:
        rowptr[r + 1:] += 1
    order = sorted(rc)
    return synth.Lower(n, rowptr, np.array([c for _, c in order], np.int32), np.ones(len(rc)))


@pytest.mark.parametrize("name,L", [
    # the 160 KiB window: exactly full, 16 bytes over, exactly full only with the last tile clipped
    ("window_boundaries", _rows_lower(20600, [(10300, 256), (15400, 15616 - 10241), (20590, 20600 - 10240)])),
    # distances exactly at beta/2, 3 beta/4 and 9 beta/10 (beta = 20)
    ("distance_thresholds", _rows_lower(40, [(30, 10), (31, 21), (32, 17), (33, 15), (34, 23), (35, 19), (36, 17)])),
])
def test_features_at_their_boundaries_bit_exact(name, L):
    """The hand-built boundary cases of the oracle's pins, in the given
    order (no reordering), bit for bit."""
    M = p3.Matrix(L).reorder(permute=0)
    got, want = M.features(), oracle.features(L)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), np.flatnonzero(got != want)


def test_features_on_a_stream():
    """pars3_features on a side stream, after work queued there."""
    import torch
    L = synth.grid3d(20, 3, "normal")
    M = p3.Matrix(L).reorder()
    s = torch.cuda.Stream()
    got = p3.pars3_features(M.h, s)
    assert np.array_equal(got, oracle.features(oracle.permute(L, oracle.rcm(L))))
