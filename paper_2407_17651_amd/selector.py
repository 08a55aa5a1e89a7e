"""Learned configuration selector: sweep records, training and regret.

Section 3.1.2 leaves the outer bandwidth of the split to the user and suggests
choosing it from the bandwidth and density of the reordered matrix.  Here the
choice covers the whole layout configuration (inner band width w_in, outer
boundary t_out, tile height) and is learned:

* ``sweep``: for generated matrices (2D/3D stencils, random geometric graphs,
  Chung-Lu power-law graphs; n log-uniform), the exhaustive autotuner
  (``pars3_autotune``) times every configuration of the default grid on the
  GPU (40 tile configurations and the full-CSR engine), ``pars3_features``
  measures 32 features after reordering and ``pars3_conflict_features`` 3
  more: the conflicting (R2) share, halo and reach over 8 row blocks (Section
  3, Fig. 2).  These records are the training data.
* ``extend``: adds the conflict features and the full-CSR timing to a sweep
  file made before they existed (the 40 tile timings are kept).
* ``targets``: T[m, g] = log(t[m, g] / min_g t[m, g]), masked where a
  configuration failed.
* ``train``: the network (``pars3_mlp``: 35 -> 64 -> 64 -> |G|, ReLU) is
  fitted with the library's own forward, backward and Adam kernels.
* ``evaluate``: regret t(selected) / t(best) - 1 on held-out matrices, for
  the network, the paper's configuration (w_in = 0, t_out = beta - 3, 256-row
  tiles) and the single configuration best on average over the training set.

Command line (GPU):
  python -m paper_2407_17651_amd.selector sweep --start 0 --count 500 --out sweep_0.npz
  python -m paper_2407_17651_amd.selector extend --start 0 --count 500 --out ext_0.npz
  python -m paper_2407_17651_amd.selector merge OUT IN [IN ...]
  python -m paper_2407_17651_amd.selector evaluate [--data FILE]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(HERE, "data", "selector_sweep_f32.npz")
WEIGHTS = os.path.join(HERE, "data", "selector_mlp.npz")
N_MATRICES = 2000
N_HELD_OUT = 200
FAMILIES = ("grid2d", "grid3d", "rgg2d", "chung_lu")


def grid_table(grid):
    """(tile_rows, w_in, t_out code, engine) per configuration of a default
    grid."""
    return np.array([(g.tile_rows, g.w_in, g.t_out, g.engine) for g in grid], np.int32)


def paper_config_index(grid) -> int:
    """The paper's split (w_in = 0, outer bandwidth 3) with 256-row tiles."""
    for i, g in enumerate(grid):
        if g.tile_rows == 256 and g.w_in == 0 and g.t_out == -1 and g.engine == 0:
            return i
    raise ValueError("grid lacks the paper configuration")


def paper_index(table) -> int:
    """paper_config_index on a grid_table array."""
    t = np.asarray(table)
    eng = t[:, 3] if t.shape[1] > 3 else np.zeros(len(t), np.int32)
    return int(np.flatnonzero((t[:, 0] == 256) & (t[:, 1] == 0) & (t[:, 2] == -1) & (eng == 0))[0])


def features_of(M):
    """The selector's 35 inputs of a reordered handle: 32 features and 3
    conflict features over the 8 row blocks."""
    return np.concatenate([M.features(), M.conflict_features()])


def sweep(start: int, count: int, reps: int = 10, value_dtype: int | None = None, log=sys.stdout) -> dict:
    import synth
    import paper_2407_17651_amd as p3

    vd = p3.F32 if value_dtype is None else value_dtype
    grid = p3.pars3_tune_grid_default(vd)
    specs = synth.selector_specs(N_MATRICES)[start:start + count]
    F, Tm, meta = [], [], []
    t0 = time.time()
    for q, spec in enumerate(specs):
        L = synth.make(spec, "uniform_f32")
        M = p3.Matrix(L)
        res, best = p3.pars3_autotune(M.h, grid=grid, k=1, reps=reps)
        F.append(features_of(M))
        Tm.append([r["us"] for r in res])
        info = M.info()
        meta.append((start + q, FAMILIES.index(spec["family"]), L.n, L.nnz, info["beta"]))
        M.close()
        print(f"[sweep] {start + q} {spec['family']} n={L.n} nnz={L.nnz} best={best} "
              f"us={res[best]['us']:.1f} elapsed={time.time() - t0:.0f}s", file=log, flush=True)
    return {"features": np.array(F, np.float64), "times_us": np.array(Tm, np.float64),
            "meta": np.array(meta, np.int64), "grid": grid_table(grid)}


def extend(start: int, count: int, reps: int = 10, value_dtype: int | None = None, base: str = DATA,
           log=sys.stdout) -> dict:
    """The 3 conflict features and the full-CSR timing of the matrices
    [start, start + count) of a sweep file without them; the rows of the
    result replace the file's (its 40 tile timings kept)."""
    import synth
    import paper_2407_17651_amd as p3

    vd = p3.F32 if value_dtype is None else value_dtype
    grid = p3.pars3_tune_grid_default(vd)
    csr = [g for g in grid if g.engine == p3.ENGINE_CSR]
    old = load(base)
    specs = synth.selector_specs(N_MATRICES)
    F, Tm, meta = [], [], []
    t0 = time.time()
    for q in range(start, min(start + count, len(old["meta"]))):
        idx = int(old["meta"][q, 0])
        L = synth.make(specs[idx], "uniform_f32")
        M = p3.Matrix(L).reorder(value_dtype=vd)
        cf = M.conflict_features()
        res, _ = p3.pars3_autotune(M.h, grid=(p3.SplitParams * 1)(*csr), k=1, reps=reps)
        F.append(np.concatenate([old["features"][q, :32], cf]))
        Tm.append(np.concatenate([old["times_us"][q, :40], [res[0]["us"]]]))
        meta.append(old["meta"][q])
        tb = old["times_us"][q, :40]
        print(f"[extend] {idx} {specs[idx]['family']} n={L.n} csr_us={res[0]['us']:.1f} "
              f"best_tile_us={tb[tb > 0].min():.1f} elapsed={time.time() - t0:.0f}s", file=log, flush=True)
        M.close()
    return {"features": np.array(F, np.float64), "times_us": np.array(Tm, np.float64),
            "meta": np.array(meta, np.int64), "grid": grid_table(grid)}


def merge(paths, out):
    parts = [np.load(p) for p in paths]
    d = {k: np.concatenate([p[k] for p in parts]) for k in ("features", "times_us", "meta")}
    order = np.argsort(d["meta"][:, 0], kind="stable")
    d = {k: v[order] for k, v in d.items()}
    d["grid"] = parts[0]["grid"]
    if len(np.unique(d["meta"][:, 0])) != len(d["meta"]):
        raise ValueError("duplicate matrices in the sweep files")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    np.savez_compressed(out, **d)
    return out


def load(path: str = DATA) -> dict:
    with np.load(path) as z:
        return {k: z[k] for k in z.files}


def targets(times_us):
    """Log time ratio to the best configuration of each matrix, and the mask
    of configurations that were timed."""
    t = np.asarray(times_us, np.float64)
    valid = t > 0
    best = np.where(valid, t, np.inf).min(1, keepdims=True)
    T = np.where(valid, np.log(np.where(valid, t, 1.0) / best), 0.0)
    return T.astype(np.float32), valid.astype(np.float32)


def split(d, held_out: int = N_HELD_OUT):
    idx = d["meta"][:, 0]
    test = idx >= idx.max() + 1 - held_out if len(idx) else idx < 0
    return ~test, test


def train(features, times_us, epochs: int = 400, batch: int = 128, lr: float = 2e-3, seed: int = 7,
          hidden=(64, 64)):
    """Fits a selector network on the GPU; returns (mlp, loss history)."""
    import torch
    import paper_2407_17651_amd as p3

    T, Mk = targets(times_us)
    dev = torch.device("cuda:0")
    # row-major copies: column selections (fancy indexing) give Fortran order
    X = torch.from_numpy(np.ascontiguousarray(features, np.float32)).to(dev)
    Td = torch.from_numpy(np.ascontiguousarray(T)).to(dev)
    Md = torch.from_numpy(np.ascontiguousarray(Mk)).to(dev)
    mlp = p3.MLP(features.shape[1], hidden[0], hidden[1], T.shape[1], seed)
    mlp.fit_scaler(X)
    hist = mlp.train(X, Td, Md, batch=batch, epochs=epochs, lr=lr, seed=seed)
    return mlp, hist


def regrets(times_us, choice):
    t = np.asarray(times_us, np.float64)
    best = np.where(t > 0, t, np.inf).min(1)
    sel = t[np.arange(len(t)), choice]
    sel = np.where(sel > 0, sel, np.inf)
    return sel / best - 1.0


def summary(r):
    r = np.asarray(r, np.float64)
    return {"mean": float(r.mean()), "p90": float(np.quantile(r, 0.9)), "max": float(r.max()),
            "within_2pct": float((r <= 0.02).mean())}


def select(mlp, features, valid):
    """The network's choice per row of features (device inference)."""
    import torch

    X = torch.from_numpy(np.ascontiguousarray(features, np.float32)).to("cuda:0")
    V = torch.from_numpy(np.ascontiguousarray(valid, np.float32)).to("cuda:0")
    return mlp.select_rows(X, V).cpu().numpy()


def evaluate(d=None, epochs: int = 400, seed: int = 7, ablations: bool = True):
    """Trains on the first matrices, scores regret on the held-out ones
    against the best of every configuration (the 40 tile configurations and
    the full-CSR engine).  Ablations: the same network without the 3
    conflict features (32 inputs), without the full-CSR choice (40 outputs),
    and without both (the selector as it was before either)."""
    d = load() if d is None else d
    tr, te = split(d)
    F, T = d["features"], d["times_us"]
    te_t = T[te]
    grid = d["grid"]
    tiles = np.flatnonzero(grid[:, 3] == 0) if grid.shape[1] > 3 else np.arange(grid.shape[0])
    mlp, hist = train(F[tr], T[tr], epochs=epochs, seed=seed)
    choice = select(mlp, F[te], te_t > 0)
    paper = paper_index(grid)
    single = int(np.argmin(regrets_all(T[tr]).mean(0)))
    out = {
        "held_out": int(te.sum()), "trained_on": int(tr.sum()), "epochs": epochs,
        "inputs": int(F.shape[1]), "outputs": int(T.shape[1]),
        "final_loss": float(hist[-1]) if len(hist) else None,
        "mlp": summary(regrets(te_t, choice)),
        "paper_default": summary(regrets(te_t, np.full(len(te_t), paper))),
        "best_single": summary(regrets(te_t, np.full(len(te_t), single))),
        "best_single_config": grid[single].tolist(), "paper_config": grid[paper].tolist(),
        "held_out_csr_chosen": int(np.isin(choice, np.flatnonzero(grid[:, 3] == 1)).sum()) if grid.shape[1] > 3 else 0,
        "held_out_csr_best": int((np.argmin(np.where(te_t > 0, te_t, np.inf), 1)[:, None]
                                  == np.flatnonzero(grid[:, 3] == 1)[None, :]).any(1).sum())
        if grid.shape[1] > 3 else 0,
    }
    if ablations and len(tiles) < T.shape[1]:
        variants = {"no_conflict_features": (slice(0, 32), np.arange(T.shape[1])),
                    "no_csr_choice": (slice(None), tiles),
                    "neither": (slice(0, 32), tiles)}
        for name, (fc, gc) in variants.items():
            m2, _ = train(F[tr][:, fc], T[tr][:, gc], epochs=epochs, seed=seed)
            c2 = gc[select(m2, F[te][:, fc], te_t[:, gc] > 0)]
            r_all = regrets(te_t, c2)
            r_tiles = regrets(te_t[:, tiles], np.searchsorted(tiles, c2)) if np.all(np.isin(c2, tiles)) else None
            out[name] = {"vs_all": summary(r_all), "vs_tiles": summary(r_tiles) if r_tiles is not None else None}
    return out, mlp


def retimed(count: int = 16, reps: int = 10, log=None) -> dict:
    """Regret re-timed in one session, as regret is defined: for the first
    `count` held-out matrices, the trained network selects a configuration
    from features the library computes now (pars3_select), then
    pars3_autotune times every configuration of the grid in the same
    session; regret = t(selected) / t(best) - 1 over those timings (within 2%
    counts as a tie in ``within_2pct``).  The paper's configuration is scored
    on the same timings."""
    import synth
    import paper_2407_17651_amd as p3

    net, grid = load_trained(p3)
    table = grid_table(grid)
    paper = paper_index(table)
    specs = synth.selector_specs(N_MATRICES)
    first = N_MATRICES - N_HELD_OUT
    rs, rp, rows = [], [], []
    for q in range(first, first + count):
        L = synth.make(specs[q], "uniform_f32")
        M = p3.Matrix(L)
        c = p3.pars3_select(M.h, net, grid)
        res, best = p3.pars3_autotune(M.h, grid=grid, k=1, reps=reps)
        t = np.array([r["us"] for r in res], np.float64)
        rs.append(t[c] / t[best] - 1.0)
        rp.append(t[paper] / t[best] - 1.0)
        rows.append((q, specs[q]["family"], L.n, int(c), int(best)))
        M.close()
        if log is not None:
            print(f"[retimed] {q} {specs[q]['family']} n={L.n} selected={c} best={best} "
                  f"regret={rs[-1]:.4f} paper={rp[-1]:.4f}", file=log, flush=True)
    return {"matrices": count, "mlp": summary(rs), "paper_default": summary(rp), "rows": rows}


def regrets_all(times_us):
    t = np.asarray(times_us, np.float64)
    best = np.where(t > 0, t, np.inf).min(1, keepdims=True)
    return np.where(t > 0, t, np.inf) / best - 1.0


def save_trained(mlp, path: str = WEIGHTS):
    """Weights and scaler of a trained network (written by ``train-save``)."""
    P = mlp.get_params()
    mu, sd = mlp.get_scaler()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, sizes=np.array(mlp.sizes, np.int32), mean=mu, std=sd, **P)
    return path


def load_trained(p3, path: str = WEIGHTS, value_dtype=None):
    """(network, default grid) restored from ``save_trained``'s file."""
    with np.load(path) as z:
        sizes = [int(v) for v in z["sizes"]]
        P = {k: z[k] for k in p3.MLP.NAMES}
        mu, sd = z["mean"], z["std"]
    net = p3.MLP(*sizes, seed=0)
    net.set_params(P)
    net.set_scaler(mu, sd)
    grid = p3.pars3_tune_grid_default(p3.F32 if value_dtype is None else value_dtype)
    if len(grid) != sizes[3]:
        raise ValueError("the saved network does not match the default grid")
    net.set_grid(grid)
    return net, grid


class TuneDB:
    """Tuning records keyed by a hash of the matrix structure (JSON file)."""

    def __init__(self, path: str):
        self.path = path
        self.rec = {}
        if os.path.exists(path):
            with open(path) as f:
                self.rec = json.load(f)

    @staticmethod
    def key(L) -> str:
        h = hashlib.sha256()
        h.update(np.int64(L.n).tobytes())
        h.update(np.ascontiguousarray(L.rowptr, np.int32).tobytes())
        h.update(np.ascontiguousarray(L.col, np.int32).tobytes())
        return h.hexdigest()[:32]

    def get(self, L):
        return self.rec.get(self.key(L))

    def put(self, L, best: dict, results: list):
        self.rec[self.key(L)] = {"best": best, "results": results}

    def save(self):
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.rec, f)
        os.replace(tmp, self.path)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--start", type=int, default=0)
    s.add_argument("--count", type=int, default=N_MATRICES)
    s.add_argument("--reps", type=int, default=10)
    s.add_argument("--out", required=True)
    x = sub.add_parser("extend")
    x.add_argument("--start", type=int, default=0)
    x.add_argument("--count", type=int, default=N_MATRICES)
    x.add_argument("--reps", type=int, default=10)
    x.add_argument("--base", default=DATA)
    x.add_argument("--out", required=True)
    m = sub.add_parser("merge")
    m.add_argument("out")
    m.add_argument("inputs", nargs="+")
    t = sub.add_parser("train-save")
    t.add_argument("--data", default=DATA)
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--out", default=WEIGHTS)
    e = sub.add_parser("evaluate")
    e.add_argument("--data", default=DATA)
    e.add_argument("--epochs", type=int, default=400)
    r = sub.add_parser("retimed")
    r.add_argument("--count", type=int, default=N_HELD_OUT)
    r.add_argument("--reps", type=int, default=10)
    a = ap.parse_args(argv)
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    if a.cmd == "sweep":
        d = sweep(a.start, a.count, a.reps)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        np.savez_compressed(a.out, **d)
        print(f"[sweep] wrote {a.out}", flush=True)
    elif a.cmd == "extend":
        d = extend(a.start, a.count, a.reps, base=a.base)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        np.savez_compressed(a.out, **d)
        print(f"[extend] wrote {a.out}", flush=True)
    elif a.cmd == "merge":
        print(merge(a.inputs, a.out))
    elif a.cmd == "train-save":
        out, mlp = evaluate(load(a.data), epochs=a.epochs)
        save_trained(mlp, a.out)
        print(json.dumps(out), flush=True)
    elif a.cmd == "retimed":
        out = retimed(a.count, a.reps, log=sys.stdout)
        print(json.dumps({k: v for k, v in out.items() if k != "rows"}), flush=True)
    else:
        out, _ = evaluate(load(a.data), epochs=a.epochs)
        print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
