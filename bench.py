#!/usr/bin/env python3
"""Benchmark of the skew-symmetric SpMV hot path on one MI355X.

A step is one product y = shift*x + S*x (S = L - L^T, reordered by reverse
Cuthill-McKee, three-way split) over the 3D 7-point stencil workload
(128^3 grid, N(0,1) values, random relabelling), with x and the matrix already
resident in HBM.  Throughput is the algorithmic byte count of one product
(the stored triangle once, row pointers, x and y) divided by the step time.
To measure HBM rather than the 256 MB Infinity Cache, consecutive steps rotate
over independent copies of (matrix, x, y) whose total exceeds 768 MB.

Prints one JSON line (see the keys below).  Options: --steps, --warmup,
--gpus (only 1 is supported: the library runs on one GPU), --dtype.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, 8 TB/s
METRIC = "skew-SpMV GB/s (% HBM peak) vs full-CSR GPU SpMV; MRS time to 1e-10 resid"
SIZES = {"f64": (8, 8), "f32": (4, 4), "bf16": (2, 4)}  # (value bytes, vector bytes)


def kernel_name(dtype, tile_rows=256):
    """Name of the product kernel the bench times: value and vector types, one
    right-hand side, no solver epilogue, skew kind, and the entry word type
    (16-bit for tiles of at most 256 rows)."""
    v, x = {"f64": ("double", "double"), "f32": ("float", "float"), "bf16": ("unsigned short", "float")}[dtype]
    e = "unsigned short" if tile_rows <= 256 else "unsigned int"
    return f"p3::k_tile_product<{v}, {x}, 1, false, false, {e}>"


def source_hash():
    """Hash of the sources that decide the product kernel's memory traffic."""
    import hashlib
    h = hashlib.sha256()
    for f in ("spmv.hip", "layout.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_2407_17651_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(dtype, tile_rows=256, w_in=0):
    """HBM bytes per launch of the product kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's readings),
    or None when there is none for this precision, the layout differs from
    the one it was taken on (256-row tiles, no inner band), or the kernel
    sources changed since it was taken."""
    if tile_rows != 256 or w_in != 0:
        return None
    path = os.path.join(ROOT, "profiles", f"k_tile_product_3d128_{dtype}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


SETTLE_MS = 30.0  # untimed busy time before the warm-up steps of every leg


def timed_steps(fn, copies, warmup, steps, torch):
    """Average milliseconds per call of fn(s) over `steps` timed calls.  Every
    rotation copy is used once first (its first use may run one-time work
    such as a library's analysis); then untimed calls for SETTLE_MS of wall
    time, since the GPU reaches its steady clock only after some
    milliseconds of continuous work (200 products right after a few warm-up
    calls measured 29.8 us per step, then 28.3 and 28.0 in the next two runs
    of 200); then `warmup` untimed calls, then the timed ones between two
    HIP events on the current stream."""
    for c in range(copies):
        fn(c)
    torch.cuda.synchronize()
    t0, s = time.perf_counter(), 0
    while (time.perf_counter() - t0) * 1e3 < SETTLE_MS:
        for _ in range(copies):
            fn(s)
            s += 1
        torch.cuda.synchronize()
    for s in range(warmup):
        fn(s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for s in range(steps):
        fn(s)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def skew_bytes(n, nnz, dtype, k=1):
    sv, sx = SIZES[dtype]
    return nnz * (sv + 4) + (n + 1) * 4 + n * k * (sx + sx)


def batched(args, p3, synth, torch, np):
    """256 skew matrices (2D/3D stencils and random geometric graphs, n
    log-uniform in [2k, 200k]) with k = 8 FP32 right-hand sides in one
    graph-captured launch (one workgroup per matrix tile); then 256 MRS
    solves (alpha_i in [0.1, 2], b_i = A_i 1) to 1e-10 together.  The tile
    height of the batch is tuned per operation by timing whole batch launches
    (each matrix keeps its reordering; only the split is rebuilt)."""
    specs = synth.batch_specs(256)
    print("[bench] batched: generating 256 matrices", file=sys.stderr, flush=True)
    Ls = [synth.make(s, "uniform_f32") for s in specs]
    t0 = time.perf_counter()
    mats = [p3.Matrix(L).reorder(value_dtype=p3.F32, keep_fp64=1) for L in Ls]
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    xs = [torch.from_numpy(synth.vector(L.n, 500 + i, 8)).to(dev, torch.float32) for i, L in enumerate(Ls)]
    ys = [torch.empty_like(x) for x in xs]
    shifts = np.array([s["alpha"] for s in specs])
    ones = [torch.ones(L.n, dtype=torch.float64, device=dev) for L in Ls]
    bs = [torch.empty_like(o) for o in ones]

    def time_launch(bat, xs_, ys_, k, vec, reps):
        # the settling of the single-matrix legs (untimed launches for
        # SETTLE_MS of wall time; the first one captures the launch graph),
        # then 3 warm-up launches
        t0 = time.perf_counter()
        while (time.perf_counter() - t0) * 1e3 < SETTLE_MS:
            for _ in range(4):
                bat.spmv(xs_, ys_, shifts, k=k, vec_dtype=vec)
            torch.cuda.synchronize()
        for _ in range(3):
            bat.spmv(xs_, ys_, shifts, k=k, vec_dtype=vec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            bat.spmv(xs_, ys_, shifts, k=k, vec_dtype=vec)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def split_all(T):
        for M in mats:
            M.reorder(value_dtype=p3.F32, keep_fp64=1, tile_rows=T)
        return p3.Batch(mats)

    # the batch's tile height, per operation, by the library's batch-level
    # autotuner (whole batch launches timed per height; the handles are left
    # split with the fastest)
    tiles = (256, 512, 1024)
    us1, b1 = p3.pars3_batch_autotune(mats, tiles, k=1, vec_dtype=p3.F64, reps=5)
    us8, b8 = p3.pars3_batch_autotune(mats, tiles, k=8, vec_dtype=p3.F32, reps=5)
    tune = {T: (us8[j] * 1e-3, us1[j] * 1e-3) for j, T in enumerate(tiles)}
    t8, t1 = tiles[b8], tiles[b1]
    bat = p3.Batch(mats)
    reps = max(10, args.steps // 4)
    ms = time_launch(bat, xs, ys, 8, p3.F32, reps)
    nsum = sum(L.n for L in Ls)
    nnzsum = sum(L.nnz for L in Ls)
    Bb = sum(skew_bytes(L.n, L.nnz, "f32", 8) for L in Ls)
    out = {"workload": "256 skew matrices (2D/3D stencils, RGG deg 16), n log-uniform in [2k, 200k], "
                       "k = 8 FP32 right-hand sides, one graph-captured launch",
           "sum_n": nsum, "sum_nnz_lower": nnzsum, "tile_rows": t8,
           "tuning_ms": {str(T): [round(a, 4), round(b, 4)] for T, (a, b) in tune.items()},
           "ms_per_launch": round(ms, 4), "gbs": round(Bb / (ms * 1e-3) / 1e9, 1),
           "gflops": round(4.0 * 8 * nnzsum / (ms * 1e-3) / 1e9, 1), "prep_s": round(prep_s, 2)}
    # batched MRS on the tile height tuned for the FP64 product
    del bat
    bat = split_all(t1)
    bat.spmv(ones, bs, shifts, k=1, vec_dtype=p3.F64)
    xs0 = [torch.zeros_like(o) for o in ones]
    print("[bench] batched MRS", file=sys.stderr, flush=True)
    st, infos = bat.mrs(shifts, bs, xs0, check=False, order=p3.ORDER_RCM, tol=1e-10, maxit=20000)
    for x in xs0:
        x.zero_()
    st, infos = bat.mrs(shifts, bs, xs0, check=False, order=p3.ORDER_RCM, tol=1e-10, maxit=20000)
    it = np.array([i["iters"] for i in infos])
    out["mrs"] = {"status": p3.STATUS_NAMES[st], "tile_rows": t1, "ms": round(infos[0]["time_ms"], 2),
                  "max_relres": float(max(i["relres"] for i in infos)), "iters_max": int(it.max()),
                  "iters_mean": round(float(it.mean()), 1), "systems": len(infos)}
    return out


# Stand-ins for the paper's six test matrices (its Table 1: rows, nonzeros of
# the full matrix, RCM bandwidth): 3D random geometric graphs in the unit cube
# with the same number of rows and mean degree nonzeros / rows - 1.  They
# have the kind of structure of those meshes, not their bandwidths.
TABLE1 = [(914_898, 40_878_708, 13_727), (923_136, 40_373_538, 14_672), (952_203, 42_493_817, 8_707),
          (503_625, 17_550_675, 1_274), (1_391_349, 64_131_971, 87_872), (943_695, 77_651_847, 35_102)]


def table1(args, p3, synth, torch):
    """FP64 skew product (RCM + the paper's split, the library's default
    tiles) against rocSPARSE on the full CSR of the same reordered matrix, on
    each stand-in, rotating over enough copies to exceed the 256 MB
    Infinity Cache."""
    dev = torch.device("cuda:0")
    rows = []
    for q, (nr, nz, bw) in enumerate(TABLE1):
        deg = nz / nr - 1.0
        print(f"[bench] table 1 stand-in {q + 1}: n={nr} mean degree {deg:.1f}", file=sys.stderr, flush=True)
        L = synth.rgg3d(nr, deg, 1300 + q, "uniform")
        n, nnz = L.n, L.nnz
        B = skew_bytes(n, nnz, "f64")
        copies = max(2, math.ceil(768e6 / B))
        mats = [p3.Matrix(L).reorder(value_dtype=p3.F64) for _ in range(copies)]
        info = mats[0].info()
        x0 = torch.from_numpy(synth.vector(n, 1401 + q)).to(dev, torch.float64)
        xs = [x0.clone() for _ in range(copies)]
        ys = [torch.empty_like(x0) for _ in range(copies)]
        cs = [p3.pars3_csr_create(m.h, p3.ORDER_RCM, p3.F64) for m in mats]

        def timed(fn):
            return timed_steps(fn, copies, args.warmup, args.steps, torch)

        ms = timed(lambda s: p3.pars3_spmv(mats[s % copies].h, 0.0, xs[s % copies], ys[s % copies], 1, p3.F64,
                                           p3.ORDER_RCM))
        cms = timed(lambda s: p3.pars3_csr_spmv(cs[s % copies], 0.0, xs[s % copies], ys[s % copies], 1))
        rows.append({"n": n, "nnz_lower": nnz, "mean_degree": round(2 * nnz / n, 2), "beta": info["beta"],
                     "paper_rcm_bandwidth": bw, "tile_rows": info["tile_rows"], "skew_ms": round(ms, 5),
                     "skew_gbs": round(B / (ms * 1e-3) / 1e9, 1), "rocsparse_full_csr_ms": round(cms, 5),
                     "skew_speedup": round(cms / ms, 3)})
        for c in cs:
            p3.pars3_csr_destroy(c)
        del mats, cs, xs, ys
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return {"workload": "3D random geometric graphs in the unit cube with the rows and mean degree of the "
                        "paper's Table 1 matrices, U[-1,1] values, random relabelling", "matrices": rows}


def workload2(args, p3, synth, torch):
    """The 4M-row random geometric graph (mean degree 16): skew product
    against rocSPARSE on the full CSR of the same reordered matrix, FP64 and
    FP32, rotating over enough copies to exceed the Infinity Cache."""
    dev = torch.device("cuda:0")
    print("[bench] workload 2: RGG n = 4M, mean degree 16", file=sys.stderr, flush=True)
    L = synth.workload(2)
    n, nnz = L.n, L.nnz
    res = {"workload": "random geometric graph in the unit square, n = 4,000,000, mean degree 16, U[-1,1] values, "
                       "random relabelling, RCM + paper split", "n": n, "nnz_lower": nnz}
    for dt, vdt, vec, tdt in (("f64", p3.F64, p3.F64, torch.float64), ("f32", p3.F32, p3.F32, torch.float32)):
        B = skew_bytes(n, nnz, dt)
        copies = max(2, math.ceil(768e6 / B))
        mats = [p3.Matrix(L).reorder(value_dtype=vdt) for _ in range(copies)]
        info = mats[0].info()
        x0 = torch.from_numpy(synth.vector(n, 1501)).to(dev, tdt)
        xs = [x0.clone() for _ in range(copies)]
        ys = [torch.empty_like(x0) for _ in range(copies)]
        cs = [p3.pars3_csr_create(m.h, p3.ORDER_RCM, vdt) for m in mats]

        def timed(fn):
            return timed_steps(fn, copies, args.warmup, args.steps, torch)

        ms = timed(lambda s: p3.pars3_spmv(mats[s % copies].h, 0.0, xs[s % copies], ys[s % copies], 1, vec,
                                           p3.ORDER_RCM))
        cms = timed(lambda s: p3.pars3_csr_spmv(cs[s % copies], 0.0, xs[s % copies], ys[s % copies], 1))
        res[dt] = {"beta": info["beta"], "tile_rows": info["tile_rows"], "skew_ms": round(ms, 5),
                   "skew_gbs": round(B / (ms * 1e-3) / 1e9, 1), "rocsparse_full_csr_ms": round(cms, 5),
                   "skew_speedup": round(cms / ms, 3)}
        for c in cs:
            p3.pars3_csr_destroy(c)
        del mats, cs, xs, ys
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return res


def host_cores():
    """Cores this process may run on (the container's share of the host)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover - not Linux
        return os.cpu_count() or 1


def cpu_baseline(args, oracle, synth, np, L, shift, mrs_out):
    """The oracle timed on the host's cores, on bounded samples of the same
    workload: its full-CSR FP64 product on one core (the reported value) and
    on every core (rows shared among threads, the same sums), the paper's
    serial SSS skew product on one core, and its FP64 MRS on one core to the
    FP64 residual 1e-10 on the small 2D workload and on this one."""
    n, nnz = L.n, L.nnz
    Bm = oracle.permute(L, oracle.rcm(L))  # the oracle's own reordering
    frow, fcol, fval = oracle.full_csr(Bm, shift)
    xh = synth.vector(n, 1101)
    budget = args.cpu_seconds

    def sample(fn, seconds):
        reps, t = 0, 0.0
        while t < seconds and reps < 10000:
            t1 = time.perf_counter()
            fn()
            t += time.perf_counter() - t1
            reps += 1
        return t / reps * 1e3, reps

    cpu_ms, reps = sample(lambda: oracle.csr_spmv(frow, fcol, fval, xh), budget / 2)
    par_ms, preps = sample(lambda: oracle.csr_spmv_par(frow, fcol, fval, xh), max(1.0, budget / 8))
    sss_ms, sreps = sample(lambda: oracle.sss_spmv(Bm, shift, xh), max(1.0, budget / 8))
    Bf = skew_bytes(n, nnz, "f64")
    res = {
        "value": round(Bf / (cpu_ms * 1e-3) / 1e9, 3),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "ms_per_product": round(cpu_ms, 3),
        "sample": f"{reps} oracle full-CSR FP64 products (plain C, one thread) of the same reordered "
                  f"3D 128^3 matrix; throughput counted with the FP64 skew byte count",
        "host_cores": host_cores(),
        "all_cores": {"cores": oracle.num_threads(), "ms_per_product": round(par_ms, 3),
                      "gbs": round(Bf / (par_ms * 1e-3) / 1e9, 3),
                      "sample": f"{preps} oracle full-CSR FP64 products with the rows shared among "
                                f"{oracle.num_threads()} OpenMP threads"},
        "sss_ms_per_product": round(sss_ms, 3),
        "sss_sample": f"{sreps} oracle serial SSS skew products (one thread)",
    }
    if mrs_out is not None:
        # oracle FP64 MRS to the FP64 relative residual 1e-10, one thread,
        # in full: the small 2D workload (alpha = 1) and this one (alpha = 0.5)
        mrs = {}
        for name, Lm, alpha in (("workload0_2d_100x100", synth.workload(0), 1.0),
                                ("workload1_3d_128", L, 0.5)):
            bh = oracle.spmv(Lm, alpha, np.ones(Lm.n))
            t1 = time.perf_counter()
            _, info, _ = oracle.mrs(Lm, alpha, bh, tol=1e-10, maxit=20000)
            ms = (time.perf_counter() - t1) * 1e3
            mrs[name] = {"ms": round(ms, 1), "iters": info["iters"], "relres": info["relres"],
                         "ms_per_iter": round(ms / max(info["iters"], 1), 3)}
        res["mrs_fp64_one_core"] = mrs
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", choices=sorted(SIZES), default="f64")
    ap.add_argument("--copies", type=int, default=0, help="rotation copies (0 = enough for 768 MB)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="budget of the oracle product samples")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-csr", action="store_true", help="skip the full-CSR comparison")
    ap.add_argument("--no-mrs", action="store_true", help="skip the MRS time-to-solution runs")
    ap.add_argument("--no-sym", action="store_true", help="skip the symmetric-with-diagonal product")
    ap.add_argument("--no-conflicts", action="store_true", help="skip the conflict-map timing")
    ap.add_argument("--tile-rows", type=int, default=0, help="tile height of the product (0 = the library default)")
    ap.add_argument("--w-in", type=int, default=-1, help="inner band half-width (-1 = the paper split, 0)")
    ap.add_argument("--mrs-reps", type=int, default=3, help="timed solves per MRS precision")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 256-matrix workload")
    ap.add_argument("--workload2", action="store_true",
                    help="also time the 4M-row random geometric graph (FP64 and FP32, against rocSPARSE)")
    ap.add_argument("--table1", action="store_true",
                    help="also time the stand-ins for the paper's six test matrices (about a minute)")
    ap.add_argument("--warm-cache", action="store_true",
                    help="also time the product without rotation (Infinity-Cache resident)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run 5 plain 1 GiB device copies first (reference for hardware byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this library runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2407_17651_amd as p3
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L = synth.workload(1)
    n, nnz = L.n, L.nnz
    vdt = {"f64": p3.F64, "f32": p3.F32, "bf16": p3.BF16}[args.dtype]
    vec = p3.F64 if args.dtype == "f64" else p3.F32
    tdt = torch.float64 if vec == p3.F64 else torch.float32
    B = skew_bytes(n, nnz, args.dtype)
    copies = args.copies or max(1, math.ceil(768e6 / B))
    print(f"[bench] workload 3D 128^3 n={n} nnz_L={nnz} dtype={args.dtype} copies={copies}", file=sys.stderr,
          flush=True)

    if args.calibrate_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # preprocessing (reported separately, not part of a step)
    mats = []
    t0 = time.perf_counter()
    split = dict(value_dtype=vdt, tile_rows=args.tile_rows, w_in=args.w_in)
    mats.append(p3.Matrix(L).reorder(**split))
    torch.cuda.synchronize()
    reorder_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(copies - 1):
        mats.append(p3.Matrix(L).reorder(**split))
    info = mats[0].info()
    KERNEL = kernel_name(args.dtype, info["tile_rows"])
    x0 = torch.from_numpy(synth.vector(n, 1101)).to(dev, tdt)
    xs = [x0.clone() for _ in range(copies)]
    ys = [torch.empty_like(x0) for _ in range(copies)]
    shift = 0.5

    def step(s):
        c = s % copies
        p3.pars3_spmv(mats[c].h, shift, xs[c], ys[c], 1, vec, p3.ORDER_RCM)

    ms = timed_steps(step, copies, args.warmup, args.steps, torch)
    value = B / (ms * 1e-3) / 1e9

    # same products without rotation (Infinity-Cache resident), for context
    warm_ms = None
    if args.warm_cache:
        w0, w1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0.record()
        for s in range(args.steps):
            step(0)
        w1.record()
        torch.cuda.synchronize()
        warm_ms = w0.elapsed_time(w1) / args.steps

    # every step is one launch of the product kernel on the timed stream, so
    # the timed region's average is that kernel's average launch duration
    t_band = ms
    achieved = B / (t_band * 1e-3) / 1e9
    traffic = measured_traffic(args.dtype, info["tile_rows"], info["w_in"])

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": "3D 7-point stencil 128^3, N(0,1) skew values, random relabelling, RCM + paper split",
            "n": n, "nnz_lower": nnz, "beta": info["beta"], "w_in": info["w_in"], "t_out": info["t_out"],
            "tile_rows": info["tile_rows"], "n_blocks": info["n_blocks"], "nnz_outer": info["nnz_outer"],
            "shift": shift, "rotation_copies": copies, "algorithmic_bytes_per_step": B,
        },
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "gflops": round(4.0 * nnz / (ms * 1e-3) / 1e9, 2),
        "warm_cache_gbs": round(B / (warm_ms * 1e-3) / 1e9, 2) if warm_ms else None,
        "reorder_ms": round(reorder_ms, 1),
        "kernel_ms": {KERNEL: round(t_band, 5)},
        "roofline": {
            "bound": "hbm",
            "kernel": KERNEL,
            "achieved": round(achieved, 2) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": traffic,
        },
        # HBM bytes the counters saw per launch over the launch time (the
        # layout stores 16-bit entry words, so this is below the algorithmic
        # count, which charges 4 bytes per index)
        "measured_hbm_gbs": round(traffic / (t_band * 1e-3) / 1e9, 2) if traffic else None,
    }

    # the same products with x and y in the caller's (input) numbering: a
    # gather of x into RCM order, the product, a scatter of y back; the
    # solvers permute once per solve instead, so this cost is reported apart
    def ostep(s):
        c = s % copies
        p3.pars3_spmv(mats[c].h, shift, xs[c], ys[c], 1, vec, p3.ORDER_ORIGINAL)

    oms = timed_steps(ostep, copies, args.warmup, args.steps, torch)
    out["original_order"] = {"ms": round(oms, 5), "permute_ms": round(oms - ms, 5),
                             "time_vs_rcm_order": round(oms / ms, 3)}

    # full-CSR GPU products of the same matrix (both triangles stored), same
    # rotation; own CSR-vector kernel and rocSPARSE, RCM and input numbering
    if args.dtype in ("f64", "f32") and not args.no_csr:
        Bc = skew_bytes(n, 2 * nnz, args.dtype)  # full CSR: every nonzero stored
        csr = {}
        for oname, order in (("rcm", p3.ORDER_RCM), ("input", p3.ORDER_ORIGINAL)):
            cs = [p3.pars3_csr_create(m.h, order, vdt) for m in mats]
            for ename, eng in (("own", 0), ("rocsparse", 1)):
                def cstep(s, cs=cs, eng=eng):
                    c = s % copies
                    p3.pars3_csr_spmv(cs[c], 0.0, xs[c], ys[c], eng)
                cms = timed_steps(cstep, copies, args.warmup, args.steps, torch)
                csr[f"{ename}_{oname}"] = {"ms": round(cms, 5), "gbs_csr_bytes": round(Bc / (cms * 1e-3) / 1e9, 1)}
            for c in cs:
                p3.pars3_csr_destroy(c)
        best = min(v["ms"] for v in csr.values())
        out["full_csr"] = {"algorithmic_bytes": Bc, **csr, "best_ms": best, "skew_speedup_vs_best": round(best / ms, 3)}

    # the symmetric variant with an SSS diagonal array on the same matrix and
    # rotation: y = shift x + D x + (L + L^T) x; the diagonal adds n reads of
    # the vector precision to the algorithmic bytes
    if not args.no_sym:
        dg = synth.values(n, 1203, "normal")
        smats = [p3.Matrix(L, diag=dg, symmetric=True).reorder(**split) for _ in range(copies)]

        def sstep(s):
            c = s % copies
            p3.pars3_spmv(smats[c].h, shift, xs[c], ys[c], 1, vec, p3.ORDER_RCM)

        sms = timed_steps(sstep, copies, args.warmup, args.steps, torch)
        Bs = B + n * SIZES[args.dtype][1]
        out["symmetric_diag"] = {"ms": round(sms, 5), "gbs": round(Bs / (sms * 1e-3) / 1e9, 2),
                                 "algorithmic_bytes": Bs, "time_vs_skew": round(sms / ms, 3)}
        del smats
        torch.cuda.synchronize()

    # conflict map (Section 3, Fig. 2) of the reordered matrix for 8 equal row
    # blocks (one per GPU of a node) and for the kernel's tiles: wall time of
    # the synchronous call, share of conflicting entries, largest halo
    if not args.no_conflicts:
        T = info["tile_rows"]
        nt = -(-n // T)
        cm = {}
        for cname, nb, bnd in (("blocks8", 8, None),
                               ("tiles", nt, np.minimum(np.arange(nt + 1, dtype=np.int64) * T, n))):
            p3.pars3_conflict_map(mats[0].h, nb, bnd)  # warm-up
            t0 = time.perf_counter()
            m = p3.pars3_conflict_map(mats[0].h, nb, bnd)
            cms = (time.perf_counter() - t0) * 1e3
            cm[cname] = {"blocks": nb, "ms": round(cms, 3),
                         "conflicting_fraction": round(float(m[:, 5:8].sum()) / nnz, 5),
                         "max_halo": int(m[:, 10].max()), "max_partners": int(m[:, 9].max()),
                         "max_reach_rows": int((m[:, 0] - m[:, 8]).max())}
        out["conflict_map"] = cm

    # MRS time to an FP64 relative residual of 1e-10 on (0.5 I + S) x = A 1:
    # FP64-only against mixed precision (FP32 or BF16 inner solves, FP64
    # refinement); wall time of pars3_mrs_solve, reorder excluded
    mrs_out = None
    if not args.no_mrs:
        alpha = 0.5
        mrs_out = {"workload": "3D 7-point stencil 128^3, alpha = 0.5, b = A 1, x0 = 0", "tol": 1e-10}
        ones = torch.ones(n, dtype=torch.float64, device=dev)
        for name, prec in (("f64", p3.F64), ("f32_refined", p3.F32), ("bf16_refined", p3.BF16)):
            print(f"[bench] mrs {name}", file=sys.stderr, flush=True)
            M = p3.Matrix(L).reorder(value_dtype=prec, keep_fp64=int(prec != p3.F64))
            b = torch.empty_like(ones)
            p3.pars3_spmv(M.h, alpha, ones, b, 1, p3.F64, p3.ORDER_ORIGINAL)
            runs = []
            for r in range(args.mrs_reps + 1):  # the first solve is a warm-up
                x = torch.zeros_like(ones)
                torch.cuda.synchronize()
                st, info, _ = M.mrs(alpha, b, x, order=p3.ORDER_ORIGINAL, tol=1e-10, maxit=20000, precision=prec)
                if r:
                    runs.append(info)
            runs.sort(key=lambda i: i["time_ms"])
            med = runs[len(runs) // 2]
            mrs_out[name] = {"ms": round(med["time_ms"], 3), "iters": med["iters"],
                             "refinements": med["refinements"], "relres": med["relres"],
                             "us_per_iter": round(1e3 * med["time_ms"] / max(med["iters"], 1), 2),
                             "min_ms": round(runs[0]["time_ms"], 3)}
            del M
        best_mixed = min(mrs_out["f32_refined"]["ms"], mrs_out["bf16_refined"]["ms"])
        mrs_out["mixed_speedup_vs_f64"] = round(mrs_out["f64"]["ms"] / best_mixed, 3)
        # (0.5 I + D + S) x = A 1 with D = |U[-1,1]| through the shifted skew
        # form (the scaled copy is built by the warm-up solve)
        print("[bench] mrs shifted form", file=sys.stderr, flush=True)
        dgs = np.abs(synth.values(n, 1204))
        M = p3.Matrix(L, diag=dgs).reorder()
        b = torch.empty_like(ones)
        p3.pars3_spmv(M.h, alpha, ones, b, 1, p3.F64, p3.ORDER_ORIGINAL)
        runs = []
        for r in range(args.mrs_reps + 1):
            x = torch.zeros_like(ones)
            torch.cuda.synchronize()
            st, info, _ = M.mrs(alpha, b, x, order=p3.ORDER_ORIGINAL, tol=1e-10, maxit=20000)
            if r:
                runs.append(info)
        runs.sort(key=lambda i: i["time_ms"])
        med = runs[len(runs) // 2]
        mrs_out["shifted_diag_f64"] = {"workload": "alpha = 0.5, D = |U[-1,1]|, b = (alpha I + D + S) 1",
                                       "ms": round(med["time_ms"], 3), "iters": med["iters"],
                                       "relres": med["relres"]}
        del M
        out["mrs"] = mrs_out

    if not args.no_batch:
        out["batched"] = batched(args, p3, synth, torch, np)

    if args.workload2:
        out["workload2"] = workload2(args, p3, synth, torch)

    if args.table1:
        out["table1_standins"] = table1(args, p3, synth, torch)

    if not args.no_cpu_baseline:
        import oracle  # CPU baseline leg only
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args, oracle, synth, np, L, shift, mrs_out)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
