"""Host logic of the selector driver: targets, regrets, held-out split,
sweep-file merge and the tuning database (no device work)."""
import os

import numpy as np

import synth
from paper_2407_17651_amd import selector


def test_targets_and_mask():
    t = np.array([[10.0, 20.0, -1.0], [5.0, 5.0, 7.5]])
    T, M = selector.targets(t)
    assert np.array_equal(M, [[1, 1, 0], [1, 1, 1]])
    assert np.allclose(T, [[0.0, np.log(2.0), 0.0], [0.0, 0.0, np.log(1.5)]])


def test_regrets_and_summary():
    t = np.array([[10.0, 20.0, -1.0], [5.0, 6.0, 7.5]])
    r = selector.regrets(t, np.array([1, 0]))
    assert np.allclose(r, [1.0, 0.0])
    assert np.isinf(selector.regrets(t, np.array([2, 0]))[0])  # a failed config is never acceptable
    s = selector.summary([0.0, 0.01, 0.5, 1.0])
    assert s["mean"] == 0.3775 and s["within_2pct"] == 0.5 and s["max"] == 1.0


def test_held_out_split_is_the_last_matrices():
    d = {"meta": np.array([[i, 0, 0, 0, 0] for i in range(10)])}
    tr, te = selector.split(d, held_out=3)
    assert np.array_equal(np.flatnonzero(te), [7, 8, 9]) and tr.sum() == 7


def test_merge_orders_and_rejects_duplicates(tmp_path):
    def part(ids):
        return {"features": np.ones((len(ids), 32)) * np.array(ids)[:, None], "times_us": np.ones((len(ids), 4)),
                "meta": np.array([[i, 1, 2, 3, 4] for i in ids]), "grid": np.zeros((4, 3), np.int32)}
    a, b = tmp_path / "a.npz", tmp_path / "b.npz"
    np.savez(a, **part([3, 4]))
    np.savez(b, **part([0, 1, 2]))
    out = selector.merge([str(a), str(b)], str(tmp_path / "m" / "all.npz"))
    d = selector.load(out)
    assert d["meta"][:, 0].tolist() == [0, 1, 2, 3, 4] and d["features"][4, 0] == 4
    np.savez(b, **part([2, 3]))
    try:
        selector.merge([str(a), str(b)], str(tmp_path / "x.npz"))
        raise AssertionError("duplicates accepted")
    except ValueError:
        pass


def test_tune_db_roundtrip(tmp_path):
    L1, L2 = synth.grid2d(6, 1), synth.grid2d(7, 1)
    db = selector.TuneDB(str(tmp_path / "db.json"))
    assert db.get(L1) is None
    db.put(L1, {"tile_rows": 128}, [{"us": 1.0}])
    db.save()
    db2 = selector.TuneDB(str(tmp_path / "db.json"))
    assert db2.get(L1)["best"] == {"tile_rows": 128} and db2.get(L2) is None
    assert selector.TuneDB.key(L1) == selector.TuneDB.key(synth.grid2d(6, 1, "normal"))  # structure only
    assert selector.TuneDB.key(L1) != selector.TuneDB.key(synth.grid2d(6, 2))
    assert os.path.exists(str(tmp_path / "db.json"))


def test_selector_workload_recipe():
    specs = synth.selector_specs(selector.N_MATRICES)
    assert len(specs) == 2000
    n = np.array([s["n_target"] for s in specs])
    assert n.min() >= 10_000 and n.max() <= 1_000_000
    fam = [s["family"] for s in specs]
    assert set(fam) == set(selector.FAMILIES)
