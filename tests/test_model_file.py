"""Model file format of pars3_model_load (include/pars3.h documents it): a file
written here, byte by byte from that description, is read back by the
library on the GPU with the same weights, scaler and grid; damaged files are
refused with EIO before any device work, so those cases run on the CPU."""
import os
import struct

import numpy as np
import pytest

import paper_2407_17651_amd as p3


def fnv1a64(data: bytes) -> int:
    h = 1469598103934665603
    for c in data:
        h = ((h ^ c) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def model_bytes(sizes, grid, mean, std, params, version=2, magic=b"PARS3MLP"):
    """Version 2 stores 7 split parameters per configuration (the last is the
    engine); version 1 stored the first 6."""
    n_in, h1, h2, n_out = sizes
    body = magic + struct.pack("<I", version) + struct.pack("<5i", n_in, h1, h2, n_out, len(grid))
    for g in grid:
        body += struct.pack("<7i", *g) if version == 2 else struct.pack("<6i", *g[:6])
    body += np.asarray(mean, "<f4").tobytes() + np.asarray(std, "<f4").tobytes() + np.asarray(params, "<f4").tobytes()
    return body + struct.pack("<Q", fnv1a64(body))


def example(seed=4, sizes=(32, 8, 6, 5)):
    rng = np.random.default_rng(seed)
    n_in, h1, h2, n_out = sizes
    npar = n_in * h1 + h1 + h1 * h2 + h2 + h2 * n_out + n_out
    grid = [(w, -1, t, 1, 0, 1, int(t == 1024)) for w, t in zip(range(n_out), (64, 128, 256, 512, 1024))]
    return sizes, grid, rng.normal(size=n_in), rng.uniform(0.5, 2, n_in), rng.normal(size=npar)


def load_status(path):
    h = p3._vp()
    return int(p3.lib().pars3_model_load(os.fsencode(path), p3.ctypes.byref(h)))


@pytest.mark.parametrize("damage", ["missing", "magic", "version", "truncated", "checksum", "trailing", "sizes",
                                    "grid_count"])
def test_damaged_files_are_refused(tmp_path, damage):
    sizes, grid, mean, std, params = example()
    b = model_bytes(sizes, grid, mean, std, params)
    if damage == "magic":
        b = model_bytes(sizes, grid, mean, std, params, magic=b"PARS3MLQ")
    elif damage == "version":
        b = model_bytes(sizes, grid, mean, std, params, version=3)
    elif damage == "truncated":
        b = b[:-20]
    elif damage == "checksum":
        b = b[:60] + bytes([b[60] ^ 1]) + b[61:]
    elif damage == "trailing":
        b = b + b"\0"
    elif damage == "sizes":
        b = model_bytes((32, 0, 6, 5), grid, mean, std, params)
    elif damage == "grid_count":
        b = model_bytes(sizes, grid[:4], mean, std, params)
    path = str(tmp_path / "m.p3mlp")
    if damage != "missing":
        with open(path, "wb") as f:
            f.write(b)
    assert load_status(path) == p3.EIO


@pytest.mark.gpu
def test_file_written_from_the_description_loads(tmp_path):
    sizes, grid, mean, std, params = example()
    path = str(tmp_path / "m.p3mlp")
    with open(path, "wb") as f:
        f.write(model_bytes(sizes, grid, mean, std, params))
    m = p3.MLP.load(path)
    assert m.sizes == sizes
    got = np.concatenate([v.ravel() for v in m.get_params().values()])
    assert np.array_equal(got, np.asarray(params, np.float32))
    mu, sd = m.get_scaler()
    assert np.array_equal(mu, np.asarray(mean, np.float32)) and np.array_equal(sd, np.asarray(std, np.float32))
    assert [(g.w_in, g.t_out, g.tile_rows, g.value_dtype, g.keep_fp64, g.permute, g.engine)
            for g in m.get_grid()] == grid
    # and the library writes the same bytes back
    out = str(tmp_path / "again.p3mlp")
    m.save(out)
    with open(path, "rb") as a, open(out, "rb") as b:
        assert a.read() == b.read()


@pytest.mark.gpu
def test_version1_file_loads_with_tile_engine(tmp_path):
    """A version 1 file (6 split parameters per configuration) loads with
    engine PARS3_ENGINE_TILES everywhere and is written back as version 2."""
    sizes, grid, mean, std, params = example()
    grid1 = [g[:6] + (0,) for g in grid]
    path = str(tmp_path / "v1.p3mlp")
    with open(path, "wb") as f:
        f.write(model_bytes(sizes, grid1, mean, std, params, version=1))
    m = p3.MLP.load(path)
    assert [(g.w_in, g.t_out, g.tile_rows, g.value_dtype, g.keep_fp64, g.permute, g.engine)
            for g in m.get_grid()] == grid1
    out = str(tmp_path / "v2.p3mlp")
    m.save(out)
    with open(out, "rb") as f:
        assert f.read() == model_bytes(sizes, grid1, mean, std, params, version=2)
