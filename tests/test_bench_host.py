"""Host logic of bench.py: the refusal of several GPUs, the kernel name, and
the rule that measured traffic is reported only while the kernel sources are
the ones it was measured on (no device work)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_several_gpus_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_kernel_names():
    assert bench.kernel_name("f64") == "p3::k_tile_product<double, double, 1, false, false, unsigned short>"
    assert bench.kernel_name("bf16") == "p3::k_tile_product<unsigned short, float, 1, false, false, unsigned short>"
    assert bench.kernel_name("f32", 512) == "p3::k_tile_product<float, float, 1, false, false, unsigned int>"


def test_algorithmic_bytes():
    n, nnz = 10, 20
    assert bench.skew_bytes(n, nnz, "f64") == nnz * 12 + (n + 1) * 4 + n * 16
    assert bench.skew_bytes(n, nnz, "bf16", 8) == nnz * 6 + (n + 1) * 4 + n * 8 * 8


def test_traffic_only_for_matching_sources(monkeypatch):
    path = os.path.join(ROOT, "profiles", "k_tile_product_3d128_f64_traffic.txt")
    if not os.path.exists(path):
        pytest.skip("no traffic summary committed")
    monkeypatch.setattr(bench, "source_hash", lambda: "0000000000000000")
    assert bench.measured_traffic("f64") is None
    with open(path) as f:
        h = [ln.split(":", 1)[1].strip() for ln in f if ln.startswith("source_sha256:")][0]
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    assert bench.measured_traffic("f64") > 1e8
    # taken on 256-row tiles without an inner band: no figure for other layouts
    assert bench.measured_traffic("f64", tile_rows=512) is None
    assert bench.measured_traffic("f64", w_in=2) is None
    assert bench.measured_traffic("f32") is None or bench.measured_traffic("f32") > 0
