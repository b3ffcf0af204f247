"""Pins of the reference BF16 / FP8-E4M3 encoders of the oracle.

Against: the formats' definitions (exhaustive over the 256 E4M3 codes), torch's
CPU dtype conversions (a library routine, compared where it applies: inputs
exactly representable in FP32 and inside the finite range), explicit ties, and
the saturation rule.
"""

import numpy as np
import pytest
import torch

from oracle import quant


def test_e4m3_codes_roundtrip_and_landmarks():
    codes = np.arange(256, dtype=np.uint8)
    vals = quant.e4m3_decode(codes)
    finite = ~np.isnan(vals)
    assert np.isnan(vals[0x7F]) and np.isnan(vals[0xFF]) and finite.sum() == 254
    assert vals[0x7E] == 448.0 and vals[0xFE] == -448.0
    assert vals[0x01] == 2.0 ** -9 and vals[0x08] == 2.0 ** -6 and vals[0x38] == 1.0
    back = quant.e4m3_bits(vals[finite])
    assert np.array_equal(back, codes[finite])   # every finite code, -0 included


def test_e4m3_matches_torch_in_range():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 40, rng.standard_normal(5000) * 0.01,
                        np.ldexp(rng.integers(-80, 80, 2000).astype(np.float64), -10)])
    x = x.astype(np.float32).astype(np.float64)
    x = x[np.abs(x) <= 448.0]
    ours = quant.e4m3_bits(x)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    # torch may keep -0 for negative underflow; compare values of zero codes by magnitude
    assert np.array_equal(ours & 0x7F, ref & 0x7F)
    nz = (ours & 0x7F) != 0
    assert np.array_equal(ours[nz], ref[nz])


def test_e4m3_ties_and_saturation():
    assert quant.e4m3_round(np.array([464.0]))[0] == 448.0   # tie 14.5 quanta -> 14 (even)
    assert quant.e4m3_round(np.array([465.0]))[0] == 448.0   # would be 480: saturates
    assert quant.e4m3_round(np.array([-1e9]))[0] == -448.0
    assert quant.e4m3_round(np.array([1.0625]))[0] == 1.0    # halfway 1 / 1.125 -> even
    assert quant.e4m3_round(np.array([1.1875]))[0] == 1.25   # halfway 1.125 / 1.25 -> even
    assert quant.e4m3_round(np.array([2.0 ** -10]))[0] == 0.0        # half the min subnormal
    assert quant.e4m3_round(np.array([3 * 2.0 ** -10]))[0] == 2.0 ** -8


def test_bf16_matches_torch_for_fp32_inputs():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * np.exp(rng.standard_normal(20000) * 8),
                        np.ldexp(1.0 + np.arange(512) / 512.0, 3)])
    x = x.astype(np.float32).astype(np.float64)
    ours = quant.bf16_bits(x)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).view(torch.int16).numpy()
    assert np.array_equal(ours, ref.astype(np.uint16))


def test_bf16_rounds_fp64_directly():
    # 1 + 2^-8 + 2^-40 lies just above the midpoint of 1 and 1 + 2^-7: direct
    # rounding gives 1 + 2^-7, while rounding through FP32 first would lose
    # 2^-40 and tie to 1.
    v = 1.0 + 2.0 ** -8 + 2.0 ** -40
    assert quant.bf16_round(np.array([v]))[0] == 1.0 + 2.0 ** -7
    assert quant.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert quant.bf16_round(np.array([2.0 ** -133]))[0] == 2.0 ** -133   # subnormal quantum
    assert np.isinf(quant.bf16_round(np.array([3.5e38]))[0])


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_quantize_rows_error_bounds(dtype):
    rng = np.random.default_rng(2)
    X = rng.standard_normal((8, 500)) * np.exp(2.0 * rng.standard_normal(8))[:, None]
    X[3] = 0.0
    codes, s, Xh = quant.quantize_rows(X, dtype)
    rel = np.abs(Xh - X) / np.maximum(np.abs(X), 1e-300)
    if dtype == "bf16":
        assert s is None
        assert np.all(rel[X != 0] <= 2.0 ** -8)
    else:
        assert s[3] == np.float32(1.0)
        big = np.abs(X) >= 2.0 ** -6 * s.astype(np.float64)[:, None]
        assert np.all(rel[big & (X != 0)] <= 2.0 ** -4 * (1 + 1e-6))
        assert np.all(np.abs(Xh) <= 448.0 * s.astype(np.float64)[:, None])
    assert np.all(Xh[3] == 0)
