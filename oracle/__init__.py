"""Oracle for the skew-symmetric SpMV path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct host implementations of every step of the
path (validation, reverse Cuthill-McKee with fixed tie-breaking, the
sign-fixing symmetric permutation, the three-way band split, full-CSR and
serial SSS products, precision rounding, MRS, sparsity features; the MLP lives
in ``oracle.mlp``).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may use it.  It shares no code with the
library under ``paper_2407_17651_amd`` and never imports it.

Matrices are passed as any object with ``n``, ``rowptr`` (int32[n+1]),
``col`` (int32[nnz]) and ``val`` (float64[nnz]) holding the strictly lower
triangle L of S = L - L^T (or, where ``symmetric=True`` is passed, of the
symmetric S = L + L^T; a diagonal array D may join the scalar shift).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from types import SimpleNamespace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_vp = ctypes.c_void_p


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i32, i64, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "or_validate": ([i64, i64, _vp, _vp], ctypes.c_int),
            "or_rcm": ([i32, _vp, _vp, _vp], ctypes.c_int),
            "or_permute": ([i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
            "or_permute_sign": ([i32, _vp, _vp, _vp, _vp, d, _vp, _vp, _vp], ctypes.c_int),
            "or_split": ([i32, _vp, _vp, i32, i32, _vp, _vp, _vp], ctypes.c_int),
            "or_full_csr": ([i32, _vp, _vp, _vp, d, _vp, _vp, _vp], i64),
            "or_full_csr_ex": ([i32, _vp, _vp, _vp, d, _vp, d, _vp, _vp, _vp], i64),
            "or_csr_spmv": ([i32, _vp, _vp, _vp, _vp, _vp], None),
            "or_csr_spmv_par": ([i32, _vp, _vp, _vp, _vp, _vp], None),
            "or_num_threads": ([], ctypes.c_int),
            "or_sss_spmv": ([i32, _vp, _vp, _vp, d, _vp, _vp], None),
            "or_sss_spmv_ex": ([i32, _vp, _vp, _vp, d, _vp, d, _vp, _vp], None),
            "or_round_f32": ([i64, _vp, _vp], None),
            "or_round_bf16": ([i64, _vp, _vp], None),
            "or_bf16_to_f64": ([i64, _vp, _vp], None),
            "or_mrs": ([i32, _vp, _vp, _vp, d, _vp, _vp, d, i32, _vp, _vp], ctypes.c_int),
            "or_features": ([i32, _vp, _vp, _vp], ctypes.c_int),
            "or_conflict_map": ([i32, _vp, _vp, _vp, i32, _vp, _vp], ctypes.c_int),
            "or_conflict_features": ([i32, _vp, _vp, i32, _vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data if a is not None and a.size else None


def _arrs(L):
    return (int(L.n), np.ascontiguousarray(L.rowptr, np.int32), np.ascontiguousarray(L.col, np.int32),
            np.ascontiguousarray(L.val, np.float64))


def validate(n, nnz, rowptr, col) -> int:
    """0 ok, 1 malformed sizes/row pointers, 2 entry not strictly lower,
    3 unsorted or duplicate columns."""
    rp = None if rowptr is None else np.ascontiguousarray(rowptr, np.int32)
    c = None if col is None else np.ascontiguousarray(col, np.int32)
    if rp is not None and rp.shape[0] < max(n, 0) + 1:
        return 1
    if c is not None and nnz > 0 and c.shape[0] < nnz:
        return 1
    return int(_L().or_validate(n, nnz, _p(rp), _p(c)))


def rcm(L) -> np.ndarray:
    """Reverse Cuthill-McKee permutation: new position k holds old node perm[k]."""
    n, rp, c, _ = _arrs(L)
    perm = np.zeros(max(n, 0), np.int32)
    if n > 0 and _L().or_rcm(n, _p(rp), _p(c), _p(perm)) != 0:
        raise MemoryError("or_rcm")
    return perm


def permute(L, perm, symmetric: bool = False) -> SimpleNamespace:
    """Strictly lower triangle of P S P^T, rows sorted.  An entry that crosses
    the diagonal is stored transposed with its sign flipped for a
    skew-symmetric S (eq. (2)), unchanged for a symmetric S."""
    n, rp, c, v = _arrs(L)
    perm = np.ascontiguousarray(perm, np.int32)
    nnz = c.shape[0]
    orow = np.zeros(n + 1, np.int32)
    ocol = np.zeros(nnz, np.int32)
    oval = np.zeros(nnz, np.float64)
    if n > 0 and _L().or_permute_sign(n, _p(rp), _p(c), _p(v), _p(perm), 1.0 if symmetric else -1.0, _p(orow),
                                      _p(ocol), _p(oval)) != 0:
        raise MemoryError("or_permute")
    return SimpleNamespace(n=n, rowptr=orow, col=ocol, val=oval, nnz=int(nnz))


def split(L, w_in: int = -1, t_out: int = -1):
    """Three-way split: (part int8[nnz], counts int64[3], (w_in, t_out, beta))."""
    n, rp, c, _ = _arrs(L)
    part = np.zeros(c.shape[0], np.int8)
    cnt = np.zeros(3, np.int64)
    params = np.zeros(3, np.int32)
    if _L().or_split(n, _p(rp), _p(c), w_in, t_out, _p(part), cnt.ctypes.data, params.ctypes.data) != 0:
        raise ValueError("w_in > t_out")
    return part, cnt, tuple(int(t) for t in params)


def full_csr(L, alpha: float = 0.0, diag=None, symmetric: bool = False):
    """Full CSR (frow, fcol, fval) of alpha*I + D + S, columns ascending;
    S = L - L^T (skew, default) or L + L^T (symmetric); diag: D or None."""
    n, rp, c, v = _arrs(L)
    cap = 2 * c.shape[0] + n
    frow = np.zeros(n + 1, np.int32)
    fcol = np.zeros(max(cap, 1), np.int32)
    fval = np.zeros(max(cap, 1), np.float64)
    d = None if diag is None else np.ascontiguousarray(diag, np.float64)
    m = _L().or_full_csr_ex(n, _p(rp), _p(c), _p(v), float(alpha), _p(d) if d is not None else None,
                            1.0 if symmetric else -1.0, _p(frow), _p(fcol), _p(fval))
    if m < 0:
        raise MemoryError("or_full_csr")
    return frow, fcol[:m].copy(), fval[:m].copy()


def csr_spmv(frow, fcol, fval, x) -> np.ndarray:
    n = frow.shape[0] - 1
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros(n, np.float64)
    if n > 0:
        _L().or_csr_spmv(n, _p(frow), _p(fcol), _p(fval), _p(x), _p(y))
    return y


def csr_spmv_par(frow, fcol, fval, x) -> np.ndarray:
    """csr_spmv with the rows shared among the host's threads (the same sums,
    bit for bit): the all-core CPU baseline."""
    n = frow.shape[0] - 1
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros(n, np.float64)
    if n > 0:
        _L().or_csr_spmv_par(n, _p(frow), _p(fcol), _p(fval), _p(x), _p(y))
    return y


def num_threads() -> int:
    """Threads csr_spmv_par uses."""
    return int(_L().or_num_threads())


def spmv(L, alpha: float, x, diag=None, symmetric: bool = False) -> np.ndarray:
    """y = (alpha*I + D + S) x by the full-CSR definition; x may be n or n x k."""
    x = np.asarray(x, np.float64)
    frow, fcol, fval = full_csr(L, alpha, diag, symmetric)
    if x.ndim == 1:
        return csr_spmv(frow, fcol, fval, x)
    return np.stack([csr_spmv(frow, fcol, fval, np.ascontiguousarray(x[:, j])) for j in range(x.shape[1])], 1)


def sss_spmv(L, alpha: float, x, diag=None, symmetric: bool = False) -> np.ndarray:
    """Serial SSS product (the paper's baseline kernel semantics): skew by
    default, symmetric on request, with an optional diagonal array."""
    n, rp, c, v = _arrs(L)
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros(n, np.float64)
    if n > 0:
        if diag is None and not symmetric:
            _L().or_sss_spmv(n, _p(rp), _p(c), _p(v), float(alpha), _p(x), _p(y))
        else:
            d = None if diag is None else np.ascontiguousarray(diag, np.float64)
            _L().or_sss_spmv_ex(n, _p(rp), _p(c), _p(v), float(alpha), _p(d) if d is not None else None,
                                1.0 if symmetric else -1.0, _p(x), _p(y))
    return y


def round_f32(a) -> np.ndarray:
    a = np.ascontiguousarray(a, np.float64)
    out = np.zeros(a.shape, np.float32)
    if a.size:
        _L().or_round_f32(a.size, _p(a), _p(out))
    return out


def round_bf16(a) -> np.ndarray:
    """FP32 -> BF16 bits (uint16), round to nearest even."""
    a = np.ascontiguousarray(a, np.float32)
    out = np.zeros(a.shape, np.uint16)
    if a.size:
        _L().or_round_bf16(a.size, _p(a), _p(out))
    return out


def bf16_to_f64(b) -> np.ndarray:
    b = np.ascontiguousarray(b, np.uint16)
    out = np.zeros(b.shape, np.float64)
    if b.size:
        _L().or_bf16_to_f64(b.size, _p(b), _p(out))
    return out


def rounded_values(val, dtype: str) -> np.ndarray:
    """Stored values after the precision conversion, as float64."""
    if dtype == "f64":
        return np.asarray(val, np.float64).copy()
    f = round_f32(val)
    if dtype == "f32":
        return f.astype(np.float64)
    if dtype == "bf16":
        return bf16_to_f64(round_bf16(f))
    raise ValueError(dtype)


def mrs(L, alpha: float, b, x0=None, tol: float = 1e-10, maxit: int = 1000):
    """MRS for (alpha*I + S) x = b.  Returns (x, info, hist) with info keys
    iters, status (0 converged / 1 maxit / 2 breakdown), eta, relres."""
    n, rp, c, v = _arrs(L)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros(n, np.float64) if x0 is None else np.array(x0, np.float64, copy=True)
    hist = np.zeros(max(maxit, 1), np.float64)
    info = np.zeros(4, np.float64)
    if _L().or_mrs(n, _p(rp), _p(c), _p(v), float(alpha), _p(b), _p(x), float(tol), int(maxit), _p(hist),
                   info.ctypes.data) != 0:
        raise MemoryError("or_mrs")
    it = int(info[0])
    return x, {"iters": it, "status": int(info[1]), "eta": float(info[2]), "relres": float(info[3])}, hist[:it].copy()


def residual(L, alpha: float, b, x) -> float:
    """||b - (alpha*I + S) x||_2 / ||b||_2 by the full-CSR definition."""
    r = np.asarray(b, np.float64) - spmv(L, alpha, x)
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(r)) / (nb if nb > 0 else 1.0)


def skew_form(L, alpha: float, diag):
    """Shifted skew-symmetric form of A = J + S, J = alpha*I + D positive
    definite and diagonal (Section 1 names A = J - S with J symmetric positive
    semi-definite as reducible to the alpha*I + S form).  With J = diag(j_i)
    the two-sided scaling J^(-1/2) A J^(-1/2) = I + S~ is exact, S~_ik =
    s_ik / sqrt(j_i j_k) still skew.  Returns (L~, ds) with ds_i =
    1 / sqrt(j_i); the solution of A x = b is x = ds * x~ where
    (I + S~) x~ = ds * b."""
    n, rp, c, v = _arrs(L)
    j = float(alpha) + np.asarray(diag, np.float64)
    if j.shape != (n,):
        raise ValueError("diag must hold n values")
    if n and not np.all(j > 0):
        raise ValueError("alpha*I + D is not positive definite")
    ds = 1.0 / np.sqrt(j)
    rows = np.repeat(np.arange(n), np.diff(rp))
    return SimpleNamespace(n=n, rowptr=rp, col=c, val=v * ds[rows] * ds[c], nnz=int(c.shape[0])), ds


def mrs_shifted(L, alpha: float, diag, b, x0=None, tol: float = 1e-10, maxit: int = 1000):
    """MRS for (alpha*I + D + S) x = b through the shifted skew-symmetric
    form: MRS on (I + S~) x~ = ds * b from x~0 = x0 / ds, to the tolerance
    tol / sqrt(max j / min j), which bounds the relative residual of the
    returned x = ds * x~ in the original system by tol.  Returns (x, info,
    hist); info["relres"] is that original-system residual."""
    Lt, ds = skew_form(L, alpha, diag)
    j = float(alpha) + np.asarray(diag, np.float64)
    cond = float(j.max() / j.min()) if len(j) else 1.0
    b = np.asarray(b, np.float64)
    xt0 = None if x0 is None else np.asarray(x0, np.float64) / ds
    xt, info, hist = mrs(Lt, 1.0, ds * b, xt0, tol / np.sqrt(cond), maxit)
    x = ds * xt
    r = b - spmv(L, alpha, x, diag=diag)
    nb = float(np.linalg.norm(b))
    info = dict(info, relres=float(np.linalg.norm(r)) / (nb if nb > 0 else 1.0), inner_tol=tol / np.sqrt(cond))
    return x, info, hist


def features(L) -> np.ndarray:
    n, rp, c, _ = _arrs(L)
    f = np.zeros(32, np.float64)
    if _L().or_features(n, _p(rp), _p(c), f.ctypes.data) != 0:
        raise MemoryError("or_features")
    return f


def bandwidth(L) -> int:
    """max(i - j) over stored entries (0 when empty)."""
    n, rp, c, _ = _arrs(L)
    if c.size == 0:
        return 0
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    return int((rows - c).max())


CONFLICT_FIELDS = ("first_row", "rows", "safe_inner", "safe_middle", "safe_outer", "conflict_inner",
                   "conflict_middle", "conflict_outer", "reach", "partners", "halo")


def conflict_map(L, part, nblocks: int, bounds=None) -> np.ndarray:
    """Per-block conflict counts of a block-row distribution (Section 3,
    Fig. 2): int64[nblocks, 11] with the columns of CONFLICT_FIELDS.  part:
    the split class of every entry of L; bounds: nblocks + 1 row boundaries
    or None (balanced)."""
    n, rp, c, _ = _arrs(L)
    pt = np.ascontiguousarray(part, np.int8)
    b = None if bounds is None else np.ascontiguousarray(bounds, np.int64)
    out = np.zeros((max(int(nblocks), 1), 11), np.int64)
    r = _L().or_conflict_map(n, _p(rp), _p(c), _p(pt), int(nblocks), _p(b) if b is not None else None,
                             out.ctypes.data)
    if r == 1:
        raise ValueError("bad block count or bounds")
    if r != 0:
        raise MemoryError("or_conflict_map")
    return out[:nblocks]


def conflict_features(L, nblocks: int = 8) -> np.ndarray:
    """The 3 conflict features of L over nblocks balanced row blocks (R2
    share of the entries, largest halo per block row, largest reach per
    block row; Section 3, Fig. 2), in the numbering L is given in."""
    n, rp, c, _ = _arrs(L)
    f = np.zeros(3, np.float64)
    r = _L().or_conflict_features(n, _p(rp), _p(c), int(nblocks), f.ctypes.data)
    if r == 1:
        raise ValueError("bad block count")
    if r != 0:
        raise MemoryError("or_conflict_features")
    return f


def lds_passes_sorted(L, tile_rows: int = 256, w_in: int = -1, t_out: int = -1, run: int = 16):
    """LDS bank passes of the product's block entries in sorted order -- a
    property of the GPU layout's bank model, not of the paper's method (pinned
    by closed forms in the tests).  The middle and outer entries of L (in the
    numbering L is given in; split as ``split``) form tile-pair blocks (row
    tile, part, column tile), each sorted by block diagonal (column offset -
    row offset mod tile_rows) and then row offset.  Each block is cut into
    aligned runs of ``run`` entries; a run takes as many passes as its most
    frequent row offset mod 32 plus its most frequent column offset mod 32.
    Returns (runs, passes)."""
    n, rp, c, _ = _arrs(L)
    part, _, _ = split(L, w_in, t_out)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    cols = c.astype(np.int64)
    keep = part != 0
    if not keep.any():
        return 0, 0
    T = int(tile_rows)
    r, cc, p = rows[keep], cols[keep], part[keep].astype(np.int64)
    t, u, ri, cj = r // T, cc // T, r % T, cc % T
    g = (cj - ri) % T
    order = np.lexsort((ri, g, u, p, t))
    t, p, u, ri, cj = t[order], p[order], u[order], ri[order], cj[order]
    new_block = np.r_[True, (t[1:] != t[:-1]) | (p[1:] != p[:-1]) | (u[1:] != u[:-1])]
    block = np.cumsum(new_block) - 1
    first = np.flatnonzero(new_block)
    pos = np.arange(len(ri)) - first[block]
    rid = np.unique(np.stack([block, pos // run]), axis=1, return_inverse=True)[1].ravel()
    runs = int(rid.max()) + 1
    passes = 0
    for cls in (ri % 32, cj % 32):
        key = rid * 32 + cls
        cnt = np.bincount(key, minlength=runs * 32).reshape(runs, 32)
        passes += int(cnt.max(axis=1).sum())
    return runs, passes
