"""Pins of the oracle's reduced-precision rounding against library dtype
conversions (torch CPU), and of the FP8 block-scale rule."""
import math

import numpy as np
import torch

import oracle as O


def _probe_values(rng, k):
    mag = 2.0 ** rng.uniform(-14, 10, k)
    x = np.concatenate([mag * rng.choice([-1, 1], k), [0.0, 448.0, -448.0, 2 ** -6, 2 ** -9,
                                                       3 * 2 ** -10, 1.0625, 1.1875, 240.0]])
    return x.astype(np.float32)


def test_bf16_rounding_matches_torch():
    x = _probe_values(np.random.default_rng(0), 200000)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.quantise_bf16(x.astype(np.float64)), ref)


def test_fp8_e4m3_rounding_matches_torch_in_range():
    x = _probe_values(np.random.default_rng(1), 200000)
    x = x[np.abs(x) <= 448.0]
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(O.quantise_fp8_e4m3(x.astype(np.float64)), ref)
    # ties to even at a mantissa boundary: 1 + 1/16 lies between 1 and 1.125
    assert O.quantise_fp8_e4m3(np.array([1.0625, 1.1875]))[0] == 1.0
    assert O.quantise_fp8_e4m3(np.array([1.1875]))[0] == 1.25


def test_fp8_block_exponent_is_the_tightest_power_of_two():
    rng = np.random.default_rng(2)
    for a in list(2.0 ** rng.uniform(-30, 30, 5000)) + [448.0, 449.0, 224.0, 896.0, 1.0]:
        e = O.fp8_block_exponent(a)
        assert a <= 448.0 * 2.0 ** e
        assert a > 448.0 * 2.0 ** (e - 1)
    assert O.fp8_block_exponent(0.0) == 0


def test_emulated_reduced_precision_errors_are_in_the_expected_band():
    rng = np.random.default_rng(3)
    B, d, m = 4096, 16, 32
    SX = rng.standard_normal((B, d)) * np.where(np.arange(B) % 64 == 0, 100.0, 1.0)[:, None]
    G = O.gaussian_matrix(4, m, B)
    exact = G @ SX
    e_bf16 = O.rel_frobenius(O.emulate_reduced(G, SX, "bf16"), exact)
    e_fp8 = O.rel_frobenius(O.emulate_reduced(G, SX, "fp8"), exact)
    # relative rounding errors of ~2^-9 (bf16) and ~2^-4 (e4m3) per operand
    assert 1e-4 < e_bf16 < 1e-2
    assert 5e-3 < e_fp8 < 5e-2
    assert math.isfinite(e_fp8)
