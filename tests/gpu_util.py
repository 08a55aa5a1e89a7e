"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np
import torch

import oracle
import paper_2407_17651_amd as p3


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def rel_inf(got, want):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    scale = np.abs(want).max() if want.size else 0.0
    if scale == 0.0:
        return 0.0 if np.all(got == 0) else np.inf
    return float(np.abs(got - want).max() / scale)


def oracle_reordered(L):
    """Oracle reordering of L: (perm, permuted lower)."""
    perm = oracle.rcm(L)
    return perm, oracle.permute(L, perm)


def gpu_spmv(M, shift, x_np, vec=p3.F64, order=p3.ORDER_RCM):
    """Runs pars3_spmv on a host vector block and returns the host result."""
    tdt = torch.float64 if vec == p3.F64 else torch.float32
    x = to_dev(x_np, tdt)
    y = torch.full_like(x, float("nan"))
    k = 1 if x.dim() == 1 else int(x.shape[1])
    p3.pars3_spmv(M.h, shift, x, y, k, vec, order)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)
