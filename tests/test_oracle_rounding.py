"""Pins of the oracle's precision conversions against library conversions
(numpy's IEEE float32 cast and torch's bfloat16 cast, both round to nearest
even) and hand-picked tie and special cases."""
import numpy as np
import torch

import oracle
import synth


def test_f32_matches_numpy_cast():
    v = np.concatenate([synth.values(20000, 1, "normal") * 1e3, synth.values(1000, 2) * 1e-40,
                        [0.0, -0.0, np.inf, -np.inf, 1.0 + 2.0 ** -24, 1.0 + 3 * 2.0 ** -24, 3.4028235e38]])
    got = oracle.round_f32(v)
    assert np.array_equal(got.view(np.uint32), v.astype(np.float32).view(np.uint32))


def test_bf16_matches_torch_cast():
    f = np.concatenate([synth.values(20000, 3, "normal").astype(np.float32),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 1e-40, 0.0, -0.0,
                                  np.inf, -np.inf, 3.3895314e38], np.float32)])
    got = oracle.round_bf16(f)
    want = torch.from_numpy(f).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, want)


def test_bf16_ties_to_even_and_nan():
    f = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8], np.float32)  # exact ties
    b = oracle.round_bf16(f)
    assert b.tolist() == [0x3F80, 0x3F82]
    nan = np.array([np.float32("nan")], np.float32)
    bn = oracle.round_bf16(nan)[0]
    assert (bn & 0x7F80) == 0x7F80 and (bn & 0x007F) != 0 and (bn & 0x0040)


def test_rounded_values_roundtrip():
    v = synth.values(1000, 4)
    assert np.array_equal(oracle.rounded_values(v, "f64"), v)
    r32 = oracle.rounded_values(v, "f32")
    assert np.abs(r32 - v).max() <= 2 ** -24
    rb = oracle.rounded_values(v, "bf16")
    assert np.abs(rb - v).max() <= 2 ** -8 + 2 ** -24
