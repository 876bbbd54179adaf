"""Pins for the format value tables in oracle.formats against torch's own
float8_e4m3fn and bfloat16 decoders (a library routine, not the same code)."""
import numpy as np
import torch

from oracle import formats


def test_e4m3_table_matches_torch():
    vals, codes = formats.e4m3_nonneg_values()
    t = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(vals, t)
    assert vals[-1] == 448.0 and np.all(np.diff(vals) > 0)
    assert np.isnan(formats.e4m3_value(0x7F))


def test_bf16_table_matches_torch():
    vals, codes = formats.bf16_nonneg_values()
    t = torch.from_numpy(codes.view(np.int16).copy()).view(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(vals, t)
    assert np.all(np.diff(vals) > 0)


def test_least_geq_is_least_upper_value():
    rng = np.random.default_rng(0)
    for vals, _ in (formats.e4m3_nonneg_values(), formats.bf16_nonneg_values()):
        x = np.concatenate([vals[:-1], vals[:-1] * (1 + 1e-7), rng.random(1000) * vals[-1] * 0.99])
        idx = formats.least_geq(x, vals)
        assert np.all(vals[idx] >= x)
        assert np.all((idx == 0) | (vals[np.maximum(idx - 1, 0)] < x))
