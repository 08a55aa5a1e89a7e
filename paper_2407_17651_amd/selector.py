"""Learned configuration selector: sweep records, training and regret.

Section 3.1.2 leaves the outer bandwidth of the split to the user and suggests
choosing it from the bandwidth and density of the reordered matrix.  Here the
choice covers the whole layout configuration (inner band width w_in, outer
boundary t_out, tile height) and is learned:

* ``sweep``: for generated matrices (2D/3D stencils, random geometric graphs,
  Chung-Lu power-law graphs; n log-uniform), the exhaustive autotuner
  (``pars3_autotune``) times every configuration of the default grid on the
  GPU and ``pars3_features`` measures 32 features after reordering.  These
  records are the training data.
* ``targets``: T[m, g] = log(t[m, g] / min_g t[m, g]), masked where a
  configuration failed.
* ``train``: the network (``pars3_mlp``: 32 -> 64 -> 64 -> |G|, ReLU) is
  fitted with the library's own forward, backward and Adam kernels.
* ``evaluate``: regret t(selected) / t(best) - 1 on held-out matrices, for
  the network, the paper's configuration (w_in = 0, t_out = beta - 3, 256-row
  tiles) and the single configuration best on average over the training set.

Command line (GPU):
  python -m paper_2407_17651_amd.selector sweep --start 0 --count 500 --out sweep_0.npz
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
    """(tile_rows, w_in, t_out code) per configuration of a default grid."""
    return np.array([(g.tile_rows, g.w_in, g.t_out) for g in grid], np.int32)


def paper_config_index(grid) -> int:
    """The paper's split (w_in = 0, outer bandwidth 3) with 256-row tiles."""
    for i, g in enumerate(grid):
        if g.tile_rows == 256 and g.w_in == 0 and g.t_out == -1:
            return i
    raise ValueError("grid lacks the paper configuration")


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
        F.append(M.features())
        Tm.append([r["us"] for r in res])
        info = M.info()
        meta.append((start + q, FAMILIES.index(spec["family"]), L.n, L.nnz, info["beta"]))
        M.close()
        print(f"[sweep] {start + q} {spec['family']} n={L.n} nnz={L.nnz} best={best} "
              f"us={res[best]['us']:.1f} elapsed={time.time() - t0:.0f}s", file=log, flush=True)
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
    X = torch.from_numpy(np.ascontiguousarray(features, np.float32)).to(dev)
    Td = torch.from_numpy(T).to(dev)
    Md = torch.from_numpy(Mk).to(dev)
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


def evaluate(d=None, epochs: int = 400, seed: int = 7):
    """Trains on the first matrices, scores regret on the held-out ones."""
    import torch

    d = load() if d is None else d
    tr, te = split(d)
    mlp, hist = train(d["features"][tr], d["times_us"][tr], epochs=epochs, seed=seed)
    X = torch.from_numpy(np.ascontiguousarray(d["features"][te], np.float32)).to("cuda:0")
    valid = torch.from_numpy((d["times_us"][te] > 0).astype(np.float32)).to("cuda:0")
    choice = mlp.select_rows(X, valid).cpu().numpy()
    grid = d["grid"]
    paper = int(np.flatnonzero((grid[:, 0] == 256) & (grid[:, 1] == 0) & (grid[:, 2] == -1))[0])
    single = int(np.argmin(regrets_all(d["times_us"][tr]).mean(0)))
    te_t = d["times_us"][te]
    out = {
        "held_out": int(te.sum()), "trained_on": int(tr.sum()), "epochs": epochs,
        "final_loss": float(hist[-1]) if len(hist) else None,
        "mlp": summary(regrets(te_t, choice)),
        "paper_default": summary(regrets(te_t, np.full(len(te_t), paper))),
        "best_single": summary(regrets(te_t, np.full(len(te_t), single))),
        "best_single_config": grid[single].tolist(), "paper_config": grid[paper].tolist(),
    }
    return out, mlp


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
    a = ap.parse_args(argv)
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    if a.cmd == "sweep":
        d = sweep(a.start, a.count, a.reps)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        np.savez_compressed(a.out, **d)
        print(f"[sweep] wrote {a.out}", flush=True)
    elif a.cmd == "merge":
        print(merge(a.inputs, a.out))
    elif a.cmd == "train-save":
        out, mlp = evaluate(load(a.data), epochs=a.epochs)
        save_trained(mlp, a.out)
        print(json.dumps(out), flush=True)
    else:
        out, _ = evaluate(load(a.data), epochs=a.epochs)
        print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
