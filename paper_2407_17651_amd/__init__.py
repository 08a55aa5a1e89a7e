"""Skew-symmetric SpMV with reverse Cuthill-McKee reordering on MI355X (gfx950).

Python binding of the C ABI declared in ``include/pars3.h``: the functions
below carry the same names and only marshal arguments; every step runs in the
HIP kernels of ``libpars3.so``.  PyTorch provides device memory and streams
(tensors' ``data_ptr()`` and ``torch.cuda.current_stream().cuda_stream``).

The library is built in-tree by ``python -m paper_2407_17651_amd.build``.  If it
is missing, importing this package still works but every call raises
``Pars3Unavailable``: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpars3.so")

# pars3_status
OK, EINVAL, ENOTLOWER, EUNSORTED, ENOMEM, EHIP, ESTATE, ENOCONV, EBREAKDOWN, ENAN, EIO = range(11)
STATUS_NAMES = ["OK", "EINVAL", "ENOTLOWER", "EUNSORTED", "ENOMEM", "EHIP", "ESTATE", "ENOCONV", "EBREAKDOWN",
                "ENAN", "EIO"]
# pars3_dtype
F64, F32, BF16 = 0, 1, 2
ORDER_RCM, ORDER_ORIGINAL = 0, 1
SKEW, SYMMETRIC = 0, 1
ENGINE_TILES, ENGINE_CSR = 0, 1


class Pars3Unavailable(RuntimeError):
    """The HIP library is not built or cannot be loaded."""


class Pars3Error(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{where}: {name}: {message}")


class SplitParams(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("w_in", "t_out", "tile_rows", "value_dtype", "keep_fp64", "permute",
                                              "engine")]


class SplitInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("beta", ctypes.c_int32), ("w_in", ctypes.c_int32), ("t_out", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32), ("value_dtype", ctypes.c_int32), ("permute", ctypes.c_int32),
        ("nnz_inner", ctypes.c_int64), ("nnz_middle", ctypes.c_int64), ("nnz_outer", ctypes.c_int64),
        ("n_tiles", ctypes.c_int32), ("n_blocks", ctypes.c_int32), ("max_blocks", ctypes.c_int32),
        ("n_components", ctypes.c_int32), ("bfs_levels", ctypes.c_int32), ("engine", ctypes.c_int32),
        ("lds_runs", ctypes.c_int64), ("lds_passes_sorted", ctypes.c_int64), ("lds_passes", ctypes.c_int64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Profile(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64), ("ms_band", ctypes.c_double), ("ms_fixup", ctypes.c_double),
                ("ms_other", ctypes.c_double)]


class BlockConflicts(ctypes.Structure):
    _fields_ = [("first_row", ctypes.c_int64), ("rows", ctypes.c_int64), ("safe", ctypes.c_int64 * 3),
                ("conflict", ctypes.c_int64 * 3), ("reach", ctypes.c_int64), ("partners", ctypes.c_int64),
                ("halo", ctypes.c_int64)]


class TuneResult(ctypes.Structure):
    _fields_ = [("params", SplitParams), ("us", ctypes.c_double)]


class MrsOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int32),
                ("order", ctypes.c_int32), ("hist_len", ctypes.c_int32), ("hist", ctypes.c_void_p)]


class MrsInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("refinements", ctypes.c_int32), ("status", ctypes.c_int32),
                ("relres", ctypes.c_double), ("eta", ctypes.c_double), ("time_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp = ctypes.c_void_p
_i32, _i64, _d = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_st = ctypes.c_int

# name -> (argtypes, restype); the exported C ABI
SIGNATURES = {
    "pars3_split_params_default": ([ctypes.POINTER(SplitParams)], None),
    "pars3_validate": ([_i64, _i64, _vp, _vp], _st),
    "pars3_create": ([_i64, _i64, _vp, _vp, _vp, ctypes.POINTER(_vp)], _st),
    "pars3_create_sss": ([_i64, _i64, _vp, _vp, _vp, _vp, _i32, ctypes.POINTER(_vp)], _st),
    "pars3_get_kind": ([_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)], _st),
    "pars3_get_diagonal": ([_vp, _vp], _st),
    "pars3_skew_form": ([_vp, _d, ctypes.POINTER(_vp), _vp], _st),
    "pars3_destroy": ([_vp], None),
    "pars3_reorder": ([_vp, ctypes.POINTER(SplitParams), _vp], _st),
    "pars3_spmv": ([_vp, _d, _vp, _vp, _i32, _i32, _i32, _vp], _st),
    "pars3_spmv_noalloc": ([_vp, _d, _vp, _vp, _i32, _i32, _vp], _st),
    "pars3_get_perm": ([_vp, _vp], _st),
    "pars3_get_permuted_lower": ([_vp, _vp, _vp, _vp, _vp], _st),
    "pars3_get_split_info": ([_vp, ctypes.POINTER(SplitInfo)], _st),
    "pars3_get_values": ([_vp, _i32, _vp], _st),
    "pars3_set_profiling": ([_vp, _i32], _st),
    "pars3_get_profile": ([_vp, ctypes.POINTER(Profile)], _st),
    "pars3_csr_create": ([_vp, _i32, _i32, ctypes.POINTER(_vp)], _st),
    "pars3_csr_spmv": ([_vp, _d, _vp, _vp, _i32, _vp], _st),
    "pars3_csr_get": ([_vp, _vp, _vp, _vp], _st),
    "pars3_csr_size": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)], _st),
    "pars3_conflict_map": ([_vp, _i32, _vp, ctypes.POINTER(BlockConflicts), _vp], _st),
    "pars3_conflict_features": ([_vp, _i32, _vp, _vp], _st),
    "pars3_csr_destroy": ([_vp], None),
    "pars3_features": ([_vp, _vp, _vp], _st),
    "pars3_tune_grid_default": ([_i32, _vp, _i32, ctypes.POINTER(_i32)], _st),
    "pars3_autotune": ([_vp, _vp, _i32, _i32, _i32, _vp, ctypes.POINTER(_i32), _vp], _st),
    "pars3_batch_create": ([_i32, _vp, ctypes.POINTER(_vp)], _st),
    "pars3_batch_destroy": ([_vp], None),
    "pars3_batch_info": ([_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), _vp], _st),
    "pars3_batch_spmv": ([_vp, _vp, _vp, _vp, _i32, _i32, _i32, _vp], _st),
    "pars3_batch_mrs_solve": ([_vp, _vp, _vp, _vp, ctypes.POINTER(MrsOpts), _vp, _vp], _st),
    "pars3_batch_autotune": ([_vp, _i32, _vp, _i32, _i32, _i32, _i32, _vp, ctypes.POINTER(_i32), _vp], _st),
    "pars3_mlp_create": ([_i32, _i32, _i32, _i32, ctypes.c_uint64, ctypes.POINTER(_vp)], _st),
    "pars3_mlp_destroy": ([_vp], None),
    "pars3_mlp_sizes": ([_vp, _vp, ctypes.POINTER(_i64)], _st),
    "pars3_mlp_set_params": ([_vp, _vp], _st),
    "pars3_mlp_get_params": ([_vp, _vp], _st),
    "pars3_mlp_get_grads": ([_vp, _vp], _st),
    "pars3_mlp_set_scaler": ([_vp, _vp, _vp], _st),
    "pars3_mlp_get_scaler": ([_vp, _vp, _vp], _st),
    "pars3_mlp_fit_scaler": ([_vp, _vp, _i32, _vp], _st),
    "pars3_mlp_forward": ([_vp, _vp, _i32, _i32, _vp, _vp], _st),
    "pars3_mlp_loss_grad": ([_vp, _vp, _vp, _vp, _i32, _i32, ctypes.POINTER(_d), _vp], _st),
    "pars3_mlp_adam": ([_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp], _st),
    "pars3_mlp_train": ([_vp, _vp, _vp, _vp, _i32, _i32, _i32, ctypes.c_float, ctypes.c_uint64, _vp, _vp], _st),
    "pars3_mlp_select_rows": ([_vp, _vp, _i32, _vp, _vp, _vp], _st),
    "pars3_select": ([_vp, _vp, _vp, _i32, ctypes.POINTER(_i32), _vp], _st),
    "pars3_mlp_set_grid": ([_vp, _vp, _i32], _st),
    "pars3_mlp_get_grid": ([_vp, _vp, _i32, ctypes.POINTER(_i32)], _st),
    "pars3_model_save": ([_vp, ctypes.c_char_p], _st),
    "pars3_model_load": ([ctypes.c_char_p, ctypes.POINTER(_vp)], _st),
    "pars3_model_use": ([_vp], _st),
    "pars3_mrs_opts_default": ([ctypes.POINTER(MrsOpts)], None),
    "pars3_mrs_solve": ([_vp, _d, _vp, _vp, ctypes.POINTER(MrsOpts), ctypes.POINTER(MrsInfo), _vp], _st),
    "pars3_last_error": ([], ctypes.c_char_p),
}

_lib = None


def lib():
    """The loaded ``libpars3.so`` (raises ``Pars3Unavailable`` if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise Pars3Unavailable(f"{LIB_PATH} is not built; run python -m paper_2407_17651_amd.build")
        # PyTorch ships its own HIP runtime.  Loading it first makes the
        # library bind to that same runtime (it is already loaded under the
        # soname the library needs), so torch's streams and allocations are
        # valid in the library's calls and only one runtime owns the device.
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover - the library also works without torch
            pass
        try:
            L = ctypes.CDLL(LIB_PATH)
        except OSError as e:  # pragma: no cover - depends on the machine
            raise Pars3Unavailable(str(e)) from e
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != OK:
        raise Pars3Error(status, where, pars3_last_error())


def _ptr(a):
    """Host numpy array or device torch tensor -> address (None for empty).
    The library reads row-major contiguous data: anything else is refused."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if a.size and not a.flags.c_contiguous:
            raise ValueError("array must be C-contiguous (row-major)")
        return a.ctypes.data if a.size else None
    if hasattr(a, "data_ptr"):
        if a.numel() and not a.is_contiguous():
            raise ValueError("tensor must be contiguous (row-major)")
        return a.data_ptr() if a.numel() else None
    return int(a)


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


# ------------------------------------------------------------------ the C ABI
def pars3_last_error() -> str:
    return (lib().pars3_last_error() or b"").decode()


def pars3_split_params_default() -> SplitParams:
    p = SplitParams()
    lib().pars3_split_params_default(ctypes.byref(p))
    return p


def pars3_validate(n, nnz, rowptr, col) -> int:
    """Returns the pars3_status of the host-side validation (no device use)."""
    rp = None if rowptr is None else np.ascontiguousarray(rowptr, np.int32)
    c = None if col is None else np.ascontiguousarray(col, np.int32)
    return int(lib().pars3_validate(n, nnz, _ptr(rp), _ptr(c)))


def pars3_create(n, nnz, rowptr, col, val):
    rp = np.ascontiguousarray(rowptr, np.int32)
    c = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    h = _vp()
    _check(lib().pars3_create(n, nnz, _ptr(rp), _ptr(c), _ptr(v), ctypes.byref(h)), "pars3_create")
    return h


def pars3_create_sss(n, nnz, rowptr, col, val, diag=None, kind=SKEW):
    rp = np.ascontiguousarray(rowptr, np.int32)
    c = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    d = None if diag is None else np.ascontiguousarray(diag, np.float64)
    if d is not None and d.shape != (n,):
        raise ValueError("diag must hold n values")
    h = _vp()
    dp = None if d is None else d.ctypes.data  # numpy gives empty arrays an address too
    _check(lib().pars3_create_sss(n, nnz, _ptr(rp), _ptr(c), _ptr(v), dp, int(kind), ctypes.byref(h)),
           "pars3_create_sss")
    return h


def pars3_skew_form(h, alpha, stream=None):
    out = _vp()
    _check(lib().pars3_skew_form(h, float(alpha), ctypes.byref(out), _stream(stream)), "pars3_skew_form")
    return out


def pars3_get_kind(h):
    k, d = _i32(), _i32()
    _check(lib().pars3_get_kind(h, ctypes.byref(k), ctypes.byref(d)), "pars3_get_kind")
    return int(k.value), bool(d.value)


def pars3_get_diagonal(h, n):
    out = np.zeros(max(n, 1), np.float64)
    _check(lib().pars3_get_diagonal(h, _ptr(out)), "pars3_get_diagonal")
    return out[:n]


def pars3_destroy(h):
    if h:
        lib().pars3_destroy(h)


def pars3_reorder(h, params: SplitParams | None = None, stream=None):
    _check(lib().pars3_reorder(h, ctypes.byref(params) if params is not None else None, _stream(stream)),
           "pars3_reorder")


def pars3_spmv(h, shift, x, y, k=1, vec_dtype=F64, order=ORDER_RCM, stream=None):
    _check(lib().pars3_spmv(h, float(shift), _ptr(x), _ptr(y), int(k), int(vec_dtype), int(order), _stream(stream)),
           "pars3_spmv")


def pars3_spmv_noalloc(h, shift, x, y, k=1, vec_dtype=F64, stream=None):
    _check(lib().pars3_spmv_noalloc(h, float(shift), _ptr(x), _ptr(y), int(k), int(vec_dtype), _stream(stream)),
           "pars3_spmv_noalloc")


def pars3_get_perm(h, n) -> np.ndarray:
    out = np.zeros(n, np.int32)
    _check(lib().pars3_get_perm(h, _ptr(out) or _ptr(np.zeros(1, np.int32))), "pars3_get_perm")
    return out


def pars3_get_split_info(h) -> SplitInfo:
    info = SplitInfo()
    _check(lib().pars3_get_split_info(h, ctypes.byref(info)), "pars3_get_split_info")
    return info


def pars3_get_permuted_lower(h, n, nnz):
    rp = np.zeros(n + 1, np.int32)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz, np.float64)
    part = np.zeros(nnz, np.int8)
    _check(lib().pars3_get_permuted_lower(h, _ptr(rp), _ptr(col), _ptr(val), _ptr(part)), "pars3_get_permuted_lower")
    return rp, col, val, part


def pars3_get_values(h, dtype, nnz) -> np.ndarray:
    out = np.zeros(nnz, {F64: np.float64, F32: np.float32, BF16: np.uint16}[dtype])
    if nnz:
        _check(lib().pars3_get_values(h, int(dtype), _ptr(out)), "pars3_get_values")
    return out


def pars3_set_profiling(h, enable: bool):
    _check(lib().pars3_set_profiling(h, int(bool(enable))), "pars3_set_profiling")


def pars3_get_profile(h) -> dict:
    p = Profile()
    _check(lib().pars3_get_profile(h, ctypes.byref(p)), "pars3_get_profile")
    return {"calls": p.calls, "ms_band": p.ms_band, "ms_fixup": p.ms_fixup, "ms_other": p.ms_other}


def pars3_csr_create(h, order=ORDER_RCM, value_dtype=F64):
    c = _vp()
    _check(lib().pars3_csr_create(h, int(order), int(value_dtype), ctypes.byref(c)), "pars3_csr_create")
    return c


def pars3_csr_spmv(c, shift, x, y, engine=0, stream=None):
    _check(lib().pars3_csr_spmv(c, float(shift), _ptr(x), _ptr(y), int(engine), _stream(stream)), "pars3_csr_spmv")


CONFLICT_FIELDS = ("first_row", "rows", "safe_inner", "safe_middle", "safe_outer", "conflict_inner",
                   "conflict_middle", "conflict_outer", "reach", "partners", "halo")


def pars3_conflict_map(h, nblocks, bounds=None, stream=None) -> np.ndarray:
    """Per-block conflict counts, int64[nblocks, 11] with the columns of
    CONFLICT_FIELDS."""
    nb = int(nblocks)
    out = (BlockConflicts * max(nb, 1))()
    b = None if bounds is None else np.ascontiguousarray(bounds, np.int64)
    _check(lib().pars3_conflict_map(h, nb, _ptr(b), out, _stream(stream)), "pars3_conflict_map")
    return np.frombuffer(out, np.int64).reshape(-1, 11)[:nb].copy()  # 11 packed int64 per block


SELECT_BLOCKS = 8  # PARS3_SELECT_BLOCKS


def pars3_conflict_features(h, nblocks=SELECT_BLOCKS, stream=None) -> np.ndarray:
    """The 3 conflict features over nblocks balanced row blocks (float64[3])."""
    out = np.zeros(3, np.float64)
    _check(lib().pars3_conflict_features(h, int(nblocks), _ptr(out), _stream(stream)), "pars3_conflict_features")
    return out


def pars3_csr_size(c):
    n, m = _i64(), _i64()
    _check(lib().pars3_csr_size(c, ctypes.byref(n), ctypes.byref(m)), "pars3_csr_size")
    return int(n.value), int(m.value)


def pars3_csr_get(c, n=None, nnz_full=None):
    if n is None or nnz_full is None:
        n, nnz_full = pars3_csr_size(c)
    rp = np.zeros(n + 1, np.int32)
    col = np.zeros(nnz_full, np.int32)
    val = np.zeros(nnz_full, np.float64)
    _check(lib().pars3_csr_get(c, _ptr(rp), _ptr(col), _ptr(val)), "pars3_csr_get")
    return rp, col, val


def pars3_csr_destroy(c):
    if c:
        lib().pars3_csr_destroy(c)


def pars3_tune_grid_default(value_dtype=F64):
    cnt = _i32()
    _check(lib().pars3_tune_grid_default(int(value_dtype), None, 0, ctypes.byref(cnt)), "pars3_tune_grid_default")
    grid = (SplitParams * cnt.value)()
    _check(lib().pars3_tune_grid_default(int(value_dtype), grid, cnt.value, ctypes.byref(cnt)),
           "pars3_tune_grid_default")
    return grid


def pars3_autotune(h, grid=None, k=1, reps=20, stream=None, value_dtype=F64):
    """Returns (results, best): results is a list of dicts {w_in, t_out,
    tile_rows, value_dtype, engine, us}."""
    if grid is None:
        grid = pars3_tune_grid_default(value_dtype)
    out = (TuneResult * len(grid))()
    best = _i32()
    _check(lib().pars3_autotune(h, grid, len(grid), int(k), int(reps), out, ctypes.byref(best), _stream(stream)),
           "pars3_autotune")
    res = [{"w_in": r.params.w_in, "t_out": r.params.t_out, "tile_rows": r.params.tile_rows,
            "value_dtype": r.params.value_dtype, "engine": r.params.engine, "us": r.us} for r in out]
    return res, best.value


def pars3_features(h, stream=None) -> np.ndarray:
    f = np.zeros(32, np.float64)
    _check(lib().pars3_features(h, _ptr(f), _stream(stream)), "pars3_features")
    return f


def pars3_mrs_opts_default() -> MrsOpts:
    o = MrsOpts()
    lib().pars3_mrs_opts_default(ctypes.byref(o))
    return o


def pars3_mrs_solve(h, alpha, b, x, opts: MrsOpts | None = None, stream=None, check=True):
    """Solves (alpha*I + S) x = b in place of x (device FP64 tensors).  Returns
    (status, info dict); raises Pars3Error on a non-OK status when check."""
    info = MrsInfo()
    st = int(lib().pars3_mrs_solve(h, float(alpha), _ptr(b), _ptr(x), ctypes.byref(opts) if opts is not None else None,
                                   ctypes.byref(info), _stream(stream)))
    if check:
        _check(st, "pars3_mrs_solve")
    return st, info.as_dict()


class MLP:
    """Owning wrapper of a ``pars3_mlp`` (the learned configuration selector).
    Device inputs are float32 torch tensors; parameters move as numpy
    float32 arrays packed W1, b1, W2, b2, W3, b3 (input-major weights)."""

    NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")

    def __init__(self, n_in=32, h1=64, h2=64, n_out=40, seed=1):
        h = _vp()
        _check(lib().pars3_mlp_create(int(n_in), int(h1), int(h2), int(n_out), int(seed), ctypes.byref(h)),
               "pars3_mlp_create")
        self.h = h
        self.sizes = (int(n_in), int(h1), int(h2), int(n_out))
        npar = _i64()
        _check(lib().pars3_mlp_sizes(h, None, ctypes.byref(npar)), "pars3_mlp_sizes")
        self.n_params = npar.value

    def close(self):
        if self.h:
            lib().pars3_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shapes(self):
        n_in, h1, h2, n_out = self.sizes
        return {"W1": (n_in, h1), "b1": (h1,), "W2": (h1, h2), "b2": (h2,), "W3": (h2, n_out), "b3": (n_out,)}

    def unpack(self, flat):
        out, o = {}, 0
        for k, shp in self.shapes().items():
            m = int(np.prod(shp))
            out[k] = np.asarray(flat[o:o + m]).reshape(shp)
            o += m
        return out

    def pack(self, params):
        return np.concatenate([np.asarray(params[k], np.float32).ravel() for k in self.NAMES])

    def get_params(self):
        f = np.zeros(self.n_params, np.float32)
        _check(lib().pars3_mlp_get_params(self.h, _ptr(f)), "pars3_mlp_get_params")
        return self.unpack(f)

    def set_params(self, params):
        f = np.ascontiguousarray(self.pack(params), np.float32)
        _check(lib().pars3_mlp_set_params(self.h, _ptr(f)), "pars3_mlp_set_params")

    def get_grads(self):
        f = np.zeros(self.n_params, np.float32)
        _check(lib().pars3_mlp_get_grads(self.h, _ptr(f)), "pars3_mlp_get_grads")
        return self.unpack(f)

    def set_scaler(self, mean, std):
        m = np.ascontiguousarray(mean, np.float32)
        s = np.ascontiguousarray(std, np.float32)
        _check(lib().pars3_mlp_set_scaler(self.h, _ptr(m), _ptr(s)), "pars3_mlp_set_scaler")

    def get_scaler(self):
        m = np.zeros(self.sizes[0], np.float32)
        s = np.zeros(self.sizes[0], np.float32)
        _check(lib().pars3_mlp_get_scaler(self.h, _ptr(m), _ptr(s)), "pars3_mlp_get_scaler")
        return m, s

    def fit_scaler(self, X, stream=None):
        _check(lib().pars3_mlp_fit_scaler(self.h, _ptr(X), int(X.shape[0]), _stream(stream)), "pars3_mlp_fit_scaler")

    def forward(self, X, standardize=False, stream=None):
        import torch
        out = torch.empty((X.shape[0], self.sizes[3]), dtype=torch.float32, device=X.device)
        _check(lib().pars3_mlp_forward(self.h, _ptr(X), int(X.shape[0]), int(bool(standardize)), _ptr(out),
                                       _stream(stream)), "pars3_mlp_forward")
        return out

    def loss_grad(self, X, T, M, standardize=False, stream=None):
        loss = _d()
        _check(lib().pars3_mlp_loss_grad(self.h, _ptr(X), _ptr(T), _ptr(M), int(X.shape[0]),
                                         int(bool(standardize)), ctypes.byref(loss), _stream(stream)),
               "pars3_mlp_loss_grad")
        return loss.value

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib().pars3_mlp_adam(self.h, float(lr), float(beta1), float(beta2), float(eps), _stream(stream)),
               "pars3_mlp_adam")

    def train(self, X, T, M, batch=128, epochs=100, lr=1e-3, seed=1, stream=None):
        hist = np.zeros(max(int(epochs), 1), np.float64)
        _check(lib().pars3_mlp_train(self.h, _ptr(X), _ptr(T), _ptr(M), int(X.shape[0]), int(batch), int(epochs),
                                     float(lr), int(seed), _ptr(hist), _stream(stream)), "pars3_mlp_train")
        return hist[:epochs]

    def set_grid(self, grid):
        """The configurations the outputs stand for (a ctypes array of
        SplitParams, as pars3_tune_grid_default returns)."""
        _check(lib().pars3_mlp_set_grid(self.h, grid, len(grid)), "pars3_mlp_set_grid")

    def get_grid(self):
        cnt = _i32()
        _check(lib().pars3_mlp_get_grid(self.h, None, 0, ctypes.byref(cnt)), "pars3_mlp_get_grid")
        grid = (SplitParams * max(cnt.value, 1))()
        _check(lib().pars3_mlp_get_grid(self.h, grid, cnt.value, ctypes.byref(cnt)), "pars3_mlp_get_grid")
        return grid[:cnt.value]

    def save(self, path):
        _check(lib().pars3_model_save(self.h, os.fsencode(path)), "pars3_model_save")

    @classmethod
    def load(cls, path):
        """A network read by pars3_model_load (weights, scaler and grid)."""
        h = _vp()
        _check(lib().pars3_model_load(os.fsencode(path), ctypes.byref(h)), "pars3_model_load")
        m = cls.__new__(cls)
        m.h = h
        sz = (_i32 * 4)()
        npar = _i64()
        _check(lib().pars3_mlp_sizes(h, sz, ctypes.byref(npar)), "pars3_mlp_sizes")
        m.sizes = tuple(int(v) for v in sz)
        m.n_params = npar.value
        return m

    def use(self):
        """Makes this network the one pars3_reorder(A, NULL) consults."""
        _check(lib().pars3_model_use(self.h), "pars3_model_use")

    def select_rows(self, X, valid=None, stream=None):
        import torch
        choice = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
        _check(lib().pars3_mlp_select_rows(self.h, _ptr(X), int(X.shape[0]), _ptr(valid), _ptr(choice),
                                           _stream(stream)), "pars3_mlp_select_rows")
        return choice


def pars3_batch_autotune(mats, tile_rows=(256, 512, 1024), k=1, vec_dtype=F64, reps=10, stream=None):
    """Tile height of a batch by timing whole batch launches over reordered
    ``Matrix`` objects (left split with the fastest).  Returns (us, best):
    microseconds per launch for each height and the index of the fastest."""
    arr = (_vp * len(mats))(*[m.h for m in mats])
    tr = np.ascontiguousarray(tile_rows, np.int32)
    us = np.zeros(len(tr), np.float64)
    best = _i32()
    _check(lib().pars3_batch_autotune(arr, len(mats), _ptr(tr), len(tr), int(k), int(vec_dtype), int(reps), _ptr(us),
                                      ctypes.byref(best), _stream(stream)), "pars3_batch_autotune")
    return us, best.value


class Batch:
    """Owning wrapper of a ``pars3_batch`` over reordered ``Matrix`` objects
    (kept alive by the batch)."""

    def __init__(self, mats):
        self.mats = list(mats)
        arr = (_vp * len(self.mats))(*[m.h for m in self.mats])
        h = _vp()
        _check(lib().pars3_batch_create(len(self.mats), arr, ctypes.byref(h)), "pars3_batch_create")
        self.h = h

    def close(self):
        if self.h:
            lib().pars3_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        ni, g = _i32(), _i32()
        qb = np.zeros(9, np.int32)
        _check(lib().pars3_batch_info(self.h, ctypes.byref(ni), ctypes.byref(g), _ptr(qb)), "pars3_batch_info")
        return {"n_items": ni.value, "grid": g.value, "queues": qb}

    def spmv(self, xs, ys, shifts=None, k=1, vec_dtype=F64, value_dtype=-1, stream=None):
        m = len(self.mats)
        xa = (_vp * m)(*[_ptr(x) for x in xs])
        ya = (_vp * m)(*[_ptr(y) for y in ys])
        sh = None if shifts is None else np.ascontiguousarray(shifts, np.float64)
        _check(lib().pars3_batch_spmv(self.h, _ptr(sh), xa, ya, int(k), int(vec_dtype), int(value_dtype),
                                      _stream(stream)), "pars3_batch_spmv")

    def mrs(self, alphas, bs, xs, check=True, stream=None, **kw):
        m = len(self.mats)
        o = pars3_mrs_opts_default()
        for k, v in kw.items():
            setattr(o, k, type(getattr(o, k))(v))
        al = np.ascontiguousarray(alphas, np.float64)
        ba = (_vp * m)(*[_ptr(b) for b in bs])
        xa = (_vp * m)(*[_ptr(x) for x in xs])
        infos = (MrsInfo * m)()
        st = int(lib().pars3_batch_mrs_solve(self.h, _ptr(al), ba, xa, ctypes.byref(o), infos, _stream(stream)))
        if check:
            _check(st, "pars3_batch_mrs_solve")
        return st, [i.as_dict() for i in infos]


def pars3_select(h, mlp: MLP, grid=None, stream=None) -> int:
    """Selects and applies a configuration; grid None: the network's own."""
    c = _i32()
    _check(lib().pars3_select(h, mlp.h, grid, len(grid) if grid is not None else 0, ctypes.byref(c),
                              _stream(stream)), "pars3_select")
    return c.value


def pars3_model_use(mlp: MLP | None):
    """Sets (or with None clears) the network pars3_reorder(A, NULL) consults."""
    _check(lib().pars3_model_use(mlp.h if mlp is not None else None), "pars3_model_use")


# ------------------------------------------------------------------ convenience wrapper
class Matrix:
    """Owning wrapper of a ``pars3_matrix`` handle built from a strictly lower
    CSR (any object with n, rowptr, col, val)."""

    def __init__(self, L, diag=None, symmetric=False):
        self.n = int(L.n)
        self.nnz = int(len(L.col))
        self.kind = SYMMETRIC if symmetric else SKEW
        if diag is None and not symmetric:
            self.h = pars3_create(self.n, self.nnz, L.rowptr, L.col, L.val)
        else:
            self.h = pars3_create_sss(self.n, self.nnz, L.rowptr, L.col, L.val, diag, self.kind)

    @classmethod
    def _adopt(cls, h, n, nnz, kind=SKEW):
        """Wraps a handle the library created (the wrapper owns it)."""
        m = cls.__new__(cls)
        m.n, m.nnz, m.kind, m.h = int(n), int(nnz), kind, h
        return m

    def skew_form(self, alpha):
        """The shifted skew-symmetric form I + S~ of alpha*I + D + S (a new
        reordered handle holding S~)."""
        return Matrix._adopt(pars3_skew_form(self.h, alpha), self.n, self.nnz)

    def close(self):
        if self.h:
            pars3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reorder(self, stream=None, **kw):
        p = pars3_split_params_default()
        for k, v in kw.items():
            setattr(p, k, int(v))
        pars3_reorder(self.h, p, stream)
        return self

    def spmv(self, shift, x, y, order=ORDER_RCM, stream=None):
        import torch
        k = 1 if x.dim() == 1 else int(x.shape[1])
        vd = F64 if x.dtype == torch.float64 else F32
        pars3_spmv(self.h, shift, x, y, k, vd, order, stream)
        return y

    def mrs(self, alpha, b, x, hist_len=0, check=True, stream=None, **kw):
        """MRS solve; keyword options as in pars3_mrs_opts.  Returns
        (status, info, hist) with hist a numpy array of hist_len values."""
        o = pars3_mrs_opts_default()
        for k, v in kw.items():
            setattr(o, k, type(getattr(o, k))(v))
        hist = np.zeros(max(hist_len, 1), np.float64)
        o.hist_len = int(hist_len)
        o.hist = hist.ctypes.data if hist_len else None
        st, info = pars3_mrs_solve(self.h, alpha, b, x, o, stream, check)
        return st, info, hist[:min(hist_len, info["iters"])].copy()

    def features(self):
        return pars3_features(self.h)

    def conflict_map(self, nblocks, bounds=None):
        return pars3_conflict_map(self.h, nblocks, bounds)

    def conflict_features(self, nblocks=SELECT_BLOCKS):
        return pars3_conflict_features(self.h, nblocks)

    def diagonal(self):
        """The diagonal array in the reordered numbering."""
        return pars3_get_diagonal(self.h, self.n)

    def perm(self):
        return pars3_get_perm(self.h, self.n)

    def info(self):
        return pars3_get_split_info(self.h).as_dict()

    def permuted_lower(self):
        return pars3_get_permuted_lower(self.h, self.n, self.nnz)

    def values(self, dtype):
        return pars3_get_values(self.h, dtype, self.nnz)
