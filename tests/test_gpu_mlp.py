"""The selector network's HIP kernels against the FP64 oracle (oracle/mlp.py):
forward, masked-MSE loss, gradients (|g - g_ref|_inf / |g_ref|_inf <= 1e-4 per
tensor), Adam, the feature scaler, training and selection."""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_17651_amd as p3
import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rand_params(net, rng, scale=0.5):
    return {k: rng.uniform(-scale, scale, shp).astype(np.float32) for k, shp in net.shapes().items()}


def data(rng, n, n_in, n_out, drop=0.2):
    X = rng.normal(0, 1, (n, n_in)).astype(np.float32)
    T = rng.uniform(0, 2, (n, n_out)).astype(np.float32)
    M = (rng.random((n, n_out)) > drop).astype(np.float32)
    return X, T, M


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def f64(params):
    return {k: v.astype(np.float64) for k, v in params.items()}


@pytest.mark.parametrize("sizes,n", [((32, 64, 64, 40), 300), ((5, 7, 3, 4), 17), ((32, 64, 64, 40), 1)])
def test_forward_loss_and_gradients(sizes, n):
    rng = np.random.default_rng(sum(sizes) + n)
    net = p3.MLP(*sizes, seed=3)
    P = rand_params(net, rng)
    net.set_params(P)
    assert all(np.array_equal(net.get_params()[k], P[k]) for k in P)
    X, T, M = data(rng, n, sizes[0], sizes[3])
    out = net.forward(dev(X)).cpu().numpy()
    ref, cache = omlp.forward(f64(P), X)
    assert np.abs(out - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    loss = net.loss_grad(dev(X), dev(T), dev(M))
    lref = omlp.loss(ref, T, M)
    assert abs(loss - lref) <= 1e-5 * max(lref, 1e-12)
    g = net.get_grads()
    gref = omlp.backward(f64(P), cache, ref, T, M)
    for k in omlp.NAMES:
        den = np.abs(gref[k]).max()
        err = np.abs(g[k] - gref[k]).max()
        assert err <= 1e-4 * den + 1e-7, (k, err, den)


def test_adam_steps_match_oracle():
    rng = np.random.default_rng(5)
    net = p3.MLP(8, 16, 16, 6, seed=1)
    P = rand_params(net, rng)
    net.set_params(P)
    X, T, M = data(rng, 64, 8, 6)
    m = {k: np.zeros_like(v, np.float64) for k, v in P.items()}
    v = {k: np.zeros_like(v, np.float64) for k, v in P.items()}
    Pr = f64(P)
    for t in (1, 2, 3):
        net.loss_grad(dev(X), dev(T), dev(M))
        g = {k: a.astype(np.float64) for k, a in net.get_grads().items()}
        net.adam(lr=1e-2)
        Pr, m, v = omlp.adam_step(Pr, g, m, v, t, lr=1e-2)
        got = net.get_params()
        for k in omlp.NAMES:
            assert np.abs(got[k] - Pr[k]).max() <= 2e-6 * max(1.0, np.abs(Pr[k]).max()), (t, k)
        # continue the oracle from the device's rounded parameters
        Pr = f64(got)


def test_scaler_and_standardized_forward():
    rng = np.random.default_rng(9)
    net = p3.MLP(32, 64, 64, 40, seed=2)
    X = (rng.normal(3.0, 5.0, (500, 32)) * rng.uniform(0, 2, 32)).astype(np.float32)
    X[:, 7] = 1.5  # constant feature: std taken as 1
    net.fit_scaler(dev(X))
    mu, sd = net.get_scaler()
    x64 = X.astype(np.float64)
    assert np.abs(mu - x64.mean(0)).max() <= 1e-5 * np.abs(x64).max()
    want_sd = np.where(x64.std(0) > 1e-12, x64.std(0), 1.0)
    assert np.abs(sd - want_sd).max() <= 1e-5 * want_sd.max()
    assert sd[7] == 1.0
    a = net.forward(dev(X), standardize=True).cpu().numpy()
    b = net.forward(dev((X - mu) / sd)).cpu().numpy()
    assert np.abs(a - b).max() <= 1e-5 * max(1.0, np.abs(b).max())


def test_training_fits_a_smooth_target_and_selects_argmin():
    rng = np.random.default_rng(11)
    n, n_in, n_out = 1024, 6, 5
    X = rng.uniform(-1, 1, (n, n_in)).astype(np.float32)
    W = rng.uniform(-1, 1, (n_in, n_out))
    T = (np.abs(X.astype(np.float64) @ W)).astype(np.float32)
    M = np.ones_like(T)
    net = p3.MLP(n_in, 32, 32, n_out, seed=4)
    net.fit_scaler(dev(X))
    hist = net.train(dev(X), dev(T), dev(M), batch=64, epochs=60, lr=3e-3, seed=2)
    assert hist[-1] < 0.1 * hist[0], hist[[0, -1]]
    valid = (rng.random((n, n_out)) > 0.3).astype(np.float32)
    valid[:, 0] = 1
    ch = net.select_rows(dev(X), dev(valid)).cpu().numpy()
    out = net.forward(dev(X), standardize=True).cpu().numpy()
    want = np.argmin(np.where(valid > 0, out, np.inf), 1)
    assert np.array_equal(ch, want)


def test_select_applies_the_chosen_configuration():
    grid = p3.pars3_tune_grid_default(p3.F64)
    net = p3.MLP(32, 64, 64, len(grid), seed=8)
    L = synth.rgg2d(20000, 10.0, 6)
    M = p3.Matrix(L)
    c = p3.pars3_select(M.h, net, grid)
    f = M.features().astype(np.float32)
    out = net.forward(dev(f[None, :]), standardize=True).cpu().numpy()[0]
    assert c == int(np.argmin(out))
    info = M.info()
    g = grid[c]
    assert (info["tile_rows"], info["w_in"]) == (g.tile_rows, g.w_in)
    want_t = max(info["beta"] - 3, 0) if g.t_out == -1 else info["beta"] // 2
    assert info["t_out"] == max(want_t, g.w_in)
    x = synth.vector(L.n, 1)
    B = oracle.permute(L, oracle.rcm(L))
    y = torch.empty(L.n, dtype=torch.float64, device=DEV)
    M.spmv(0.5, dev(x), y)
    torch.cuda.synchronize()
    assert np.abs(y.cpu().numpy() - oracle.spmv(B, 0.5, x)).max() <= 1e-12 * np.abs(oracle.spmv(B, 0.5, x)).max()


def test_select_rejects_size_mismatch():
    grid = p3.pars3_tune_grid_default()
    net = p3.MLP(32, 8, 8, len(grid) - 1, seed=1)
    M = p3.Matrix(synth.grid2d(10, 1))
    with pytest.raises(p3.Pars3Error) as e:
        p3.pars3_select(M.h, net, grid)
    assert e.value.status == p3.EINVAL
