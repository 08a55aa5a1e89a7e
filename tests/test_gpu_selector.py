"""What the learned selector gains over the method without it: trained with
the library's own kernels on the autotuner sweeps of the first 1,800 generated
matrices, scored by regret t(selected)/t(best) - 1 on the 200 held-out ones,
against the paper's configuration (w_in = 0, t_out = beta - 3, 256-row tiles)
and against the single configuration best on average over the training set.
The sweep records are measured data (timing is the definition; parity of the
timings themselves is unpinned)."""
import json
import os

import numpy as np
import pytest
import torch

import paper_2407_17651_amd as p3
from paper_2407_17651_amd import selector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def data():
    assert os.path.exists(selector.DATA), "sweep records missing"
    return selector.load()


def test_sweep_records_shape(data):
    assert data["features"].shape == (selector.N_MATRICES, 32)
    assert data["times_us"].shape == (selector.N_MATRICES, 40)
    assert np.all(data["times_us"] > 0)
    assert np.array_equal(data["meta"][:, 0], np.arange(selector.N_MATRICES))


def test_selector_beats_paper_default_and_best_single(data):
    out, _ = selector.evaluate(data, epochs=300)
    print("[gpu] selector " + json.dumps(out), flush=True)
    assert out["held_out"] == selector.N_HELD_OUT
    assert out["mlp"]["mean"] < out["paper_default"]["mean"]
    assert out["mlp"]["mean"] < out["best_single"]["mean"]


def test_saved_network_selects_well(data):
    assert os.path.exists(selector.WEIGHTS), "trained weights missing"
    net, grid = selector.load_trained(p3)
    tr, te = selector.split(data)
    X = torch.from_numpy(np.ascontiguousarray(data["features"][te], np.float32)).to("cuda:0")
    choice = net.select_rows(X).cpu().numpy()
    r = selector.regrets(data["times_us"][te], choice)
    g = data["grid"]
    paper = int(np.flatnonzero((g[:, 0] == 256) & (g[:, 1] == 0) & (g[:, 2] == -1))[0])
    rp = selector.regrets(data["times_us"][te], np.full(len(choice), paper))
    assert r.mean() < rp.mean()
