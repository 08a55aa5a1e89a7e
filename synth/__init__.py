"""Seeded synthetic inputs: sparsity patterns, random relabelling, i.i.d. values.

The generators return the strictly lower triangle L of a skew-symmetric
S = L - L^T in CSR form (int32 row pointers and columns, float64 values,
columns ascending in every row).  This module holds no part of the method's
arithmetic; it serves the product tests, the oracle tests and the benchmark
alike.  See ``synth.c`` for the generator definitions.

Workloads (all seeded):
  * ``grid2d(k)``   : k x k five-point stencil graph, 2k(k-1) stored entries.
  * ``grid3d(k)``   : k^3 seven-point stencil graph, 3k^2(k-1) stored entries.
  * ``rgg2d(n, d)`` : random geometric graph in the unit square, mean degree d.
  * ``chung_lu(n, d, gamma)`` : power-law expected-degree graph.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")

VALUES = {"uniform": 0, "normal": 1, "uniform_f32": 2, "int4": 3, "ones": 4}


def build(force: bool = False) -> str:
    """Compile ``libsynth.so`` with gcc (host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _SynMatrix(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("rowptr", ctypes.POINTER(ctypes.c_int32)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("val", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_SynMatrix)
        u64, i64, i32, d, i = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int
        lib.syn_grid2d.argtypes = [i32, u64, i, i, P]
        lib.syn_grid3d.argtypes = [i32, u64, i, i, P]
        lib.syn_rgg2d.argtypes = [i64, d, u64, i, i, P]
        lib.syn_chung_lu.argtypes = [i64, d, d, u64, i, i, P]
        lib.syn_from_edges.argtypes = [i64, i64, ctypes.c_void_p, ctypes.c_void_p, u64, i, i, P]
        lib.syn_free.argtypes = [P]
        lib.syn_values.argtypes = [i64, u64, i, ctypes.c_void_p]
        lib.syn_rgg2d_radius.argtypes = [i64, d]
        lib.syn_rgg2d_radius.restype = d
        lib.syn_rgg3d.argtypes = [i64, d, u64, i, i, P]
        lib.syn_rgg3d_radius.argtypes = [i64, d]
        lib.syn_rgg3d_radius.restype = d
        for f in ("syn_grid2d", "syn_grid3d", "syn_rgg2d", "syn_rgg3d", "syn_chung_lu", "syn_from_edges"):
            getattr(lib, f).restype = i
        _lib = lib
    return _lib


@dataclass
class Lower:
    """Strictly lower triangle L (CSR) of S = L - L^T."""

    n: int
    rowptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def _take(sm: _SynMatrix, name: str) -> Lower:
    n, m = int(sm.n), int(sm.nnz)
    rowptr = np.ctypeslib.as_array(sm.rowptr, shape=(n + 1,)).copy()
    col = np.ctypeslib.as_array(sm.col, shape=(max(m, 1),))[:m].copy() if m else np.zeros(0, np.int32)
    val = np.ctypeslib.as_array(sm.val, shape=(max(m, 1),))[:m].copy() if m else np.zeros(0, np.float64)
    _L().syn_free(ctypes.byref(sm))
    return Lower(n, rowptr, col, val, name)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"synth: {what} failed with code {rc}")


def grid2d(k: int, seed: int, values: str = "uniform", relabel: bool = True) -> Lower:
    sm = _SynMatrix()
    _check(_L().syn_grid2d(k, seed, VALUES[values], int(relabel), ctypes.byref(sm)), "grid2d")
    return _take(sm, f"grid2d_{k}")


def grid3d(k: int, seed: int, values: str = "normal", relabel: bool = True) -> Lower:
    sm = _SynMatrix()
    _check(_L().syn_grid3d(k, seed, VALUES[values], int(relabel), ctypes.byref(sm)), "grid3d")
    return _take(sm, f"grid3d_{k}")


def rgg2d(n: int, deg: float, seed: int, values: str = "uniform", relabel: bool = True) -> Lower:
    sm = _SynMatrix()
    _check(_L().syn_rgg2d(n, deg, seed, VALUES[values], int(relabel), ctypes.byref(sm)), "rgg2d")
    return _take(sm, f"rgg2d_{n}")


def rgg2d_radius(n: int, deg: float) -> float:
    return float(_L().syn_rgg2d_radius(n, deg))


def rgg3d(n: int, deg: float, seed: int, values: str = "uniform", relabel: bool = True) -> Lower:
    """Random geometric graph in the unit cube with expected mean degree deg."""
    sm = _SynMatrix()
    _check(_L().syn_rgg3d(n, deg, seed, VALUES[values], int(relabel), ctypes.byref(sm)), "rgg3d")
    return _take(sm, f"rgg3d_{n}")


def rgg3d_radius(n: int, deg: float) -> float:
    return float(_L().syn_rgg3d_radius(n, deg))


def chung_lu(n: int, deg: float, gamma: float, seed: int, values: str = "uniform", relabel: bool = True) -> Lower:
    sm = _SynMatrix()
    _check(_L().syn_chung_lu(n, deg, gamma, seed, VALUES[values], int(relabel), ctypes.byref(sm)), "chung_lu")
    return _take(sm, f"chung_lu_{n}")


def from_edges(n: int, edges, seed: int = 0, values: str = "uniform", relabel: bool = False) -> Lower:
    """Matrix with the given undirected edges (pairs of distinct node ids)."""
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    a = np.ascontiguousarray(e[:, 0])
    b = np.ascontiguousarray(e[:, 1])
    sm = _SynMatrix()
    _check(_L().syn_from_edges(n, e.shape[0], a.ctypes.data, b.ctypes.data, seed, VALUES[values], int(relabel),
                               ctypes.byref(sm)), "from_edges")
    return _take(sm, f"edges_{n}")


def values(m: int, seed: int, kind: str = "uniform") -> np.ndarray:
    out = np.empty(m, dtype=np.float64)
    if m:
        _L().syn_values(m, seed, VALUES[kind], out.ctypes.data)
    return out


# ---------------------------------------------------------------------------
# The five benchmark workloads (default seed 1000 + index).

def workload(idx: int, seed: int | None = None) -> Lower:
    """Single-matrix workloads 0-2.

    0: 2D 100x100 grid, values U[-1,1], random relabelling.
    1: 3D 128^3 grid, values N(0,1), random relabelling.
    2: random geometric graph in the unit square, n = 4,000,000, mean degree 16,
       values U[-1,1], random relabelling.
    """
    s = 1000 + idx if seed is None else seed
    if idx == 0:
        return grid2d(100, s, "uniform")
    if idx == 1:
        return grid3d(128, s, "normal")
    if idx == 2:
        return rgg2d(4_000_000, 16.0, s, "uniform")
    raise ValueError(idx)


def vector(n: int, seed: int, k: int = 1, kind: str = "uniform") -> np.ndarray:
    """n x k row-major vector block with i.i.d. entries (U[-1,1] by default)."""
    return values(n * k, seed, kind).reshape(n, k) if k > 1 else values(n, seed, kind)


def batch_specs(count: int = 256, seed: int = 1003, n_lo: int = 2_000, n_hi: int = 200_000):
    """Family and size of each matrix of the batched workload: n log-uniform in
    [n_lo, n_hi], family uniform over {2D grid, 3D grid, RGG(deg 16)}, shift
    alpha ~ U[0.1, 2]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n_t = int(round(float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))))
        fam = int(rng.integers(0, 3))
        alpha = float(rng.uniform(0.1, 2.0))
        out.append({"family": ("grid2d", "grid3d", "rgg2d")[fam], "n_target": n_t, "alpha": alpha,
                    "seed": seed * 10_000 + i})
    return out


def selector_specs(count: int = 2000, seed: int = 1004, n_lo: int = 10_000, n_hi: int = 1_000_000):
    """Workload of the learned selector: family uniform over {2D grid, 3D grid,
    RGG(deg 16), Chung-Lu(gamma 2.5, mean degree 16)}, n log-uniform."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n_t = int(round(float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))))
        fam = int(rng.integers(0, 4))
        out.append({"family": ("grid2d", "grid3d", "rgg2d", "chung_lu")[fam], "n_target": n_t,
                    "seed": seed * 10_000 + i})
    return out


def make(spec: dict, values_kind: str = "uniform_f32") -> Lower:
    """Build the matrix a batch/selector spec describes."""
    fam, n_t, s = spec["family"], spec["n_target"], spec["seed"]
    if fam == "grid2d":
        return grid2d(max(2, int(round(n_t ** 0.5))), s, values_kind)
    if fam == "grid3d":
        return grid3d(max(2, int(round(n_t ** (1.0 / 3.0)))), s, values_kind)
    if fam == "rgg2d":
        return rgg2d(n_t, 16.0, s, values_kind)
    if fam == "chung_lu":
        return chung_lu(n_t, 16.0, 2.5, s, values_kind)
    raise ValueError(fam)
