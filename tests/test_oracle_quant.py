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


# ---------------------------------------------------------------------------
# A worked case of emulate_reduced, every expected value derived by hand
# from the two format definitions and the block-scale rule (no library
# routine and no other oracle function computes them).
#
# Formats: BF16 keeps 8 significant bits (ulp 2^-7 on [1, 2)); OCP E4M3
# keeps 4 significant bits (ulp 2^-3 on [1, 2)), smallest normal 2^-6,
# subnormal quantum 2^-9, largest finite 448.  Both round to nearest, ties
# to the even significand.
#
# FP8 scales: S X block kb (128 rows of B) is divided by 2^e, e the
# smallest integer with amax <= 448 2^e; G is divided by 2^-6 (times 64).
#
# S X is 256 x 1 (two 128-row blocks), nonzero only at
#   block 0: SX[0] = 448, SX[1] = 1.0625, SX[2] = 1.1875, SX[3] = 2^-9
#   block 1: SX[130] = 2^-10, SX[131] = 3, SX[228] = 449
# G is 4 x 256, nonzero only at
#   row 0: 1 at columns 0, 1, 2, 3, 130, 131, 228
#   row 1: 3 2^-15 at column 0
#   row 2: 5.5 at column 1
#   row 3: 1 + 2^-8 at column 0, 1 + 3 2^-8 at column 3
#
# FP8, block 0: amax 448 = 448 2^0 -> e = 0 (448 > 448 2^-1).
#   448 -> 448 (1.75 2^8, exact); 1.0625 = 1 + 2^-4 lies halfway between
#   1 and 1.125 -> even significand 1.000 -> 1; 1.1875 halfway between
#   1.125 (1.001) and 1.25 (1.010) -> 1.25; 2^-9 is the smallest
#   subnormal -> exact.
# FP8, block 1: amax 449 > 448 -> e = 1 (449 <= 896).  Scaled: 2^-10 / 2 =
#   2^-11, below half a quantum (2^-10) -> 0; 3 / 2 = 1.5 exact -> 3;
#   449 / 2 = 224.5 on [128, 256) with ulp 16, nearest 224 -> 448.
# FP8 of G (times 64): 1 -> 64 exact; 3 2^-15 -> 3 2^-9 = three quanta,
#   exact; 5.5 -> 352 = 1.375 2^8 exact; (1 + 2^-8) 64 = 64.25 and
#   (1 + 3 2^-8) 64 = 64.75 both round to 64 (ulp 8 on [64, 128)) -> 1.
#   Y_fp8[0] = 448 + 1 + 1.25 + 2^-9 + 0 + 3 + 448 = 901.25 + 2^-9
#   Y_fp8[1] = 3 2^-15 * 448 = 1344 2^-15
#   Y_fp8[2] = 5.5 * 1 = 5.5
#   Y_fp8[3] = 1 * 448 + 1 * 2^-9 = 448 + 2^-9
# BF16 (no scale): 448, 1.0625, 1.1875, 2^-9, 2^-10, 3 are exact; 449 =
#   111000001b needs 9 significant bits and is halfway between 448
#   (1.1100000 2^8) and 450 (1.1100001 2^8) -> 448.  G: 1, 3 2^-15, 5.5
#   exact; 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> 1; 1 + 3 2^-8 is
#   halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even) -> 1 + 2^-6.
#   Y_bf16[0] = 448 + 1.0625 + 1.1875 + 2^-9 + 2^-10 + 3 + 448
#             = 901.25 + 2^-9 + 2^-10
#   Y_bf16[1] = 1344 2^-15;  Y_bf16[2] = 5.5 * 1.0625 = 5.84375
#   Y_bf16[3] = 448 + (1 + 2^-6) 2^-9
# Mutations each of these values catches: a 64-row block keeps 2^-10 in
# Y_fp8[0] (its block then has amax 3 and scale 2^-7); the e = E - 8 rule
# for every amax gives block 0 the scale 2 and drops 2^-9 (a tie to 0);
# a G scale of 2^-5 turns 3 2^-15 into 1.5 quanta -> 2^-8 / 32 in
# Y_fp8[1]; a G scale of 2^-7 saturates 5.5 * 128 = 704 at 448 in Y_fp8[2].
WORKED_SX = {0: 448.0, 1: 1.0625, 2: 1.1875, 3: 2.0 ** -9, 130: 2.0 ** -10, 131: 3.0, 228: 449.0}
WORKED_G = {(0, 0): 1.0, (0, 1): 1.0, (0, 2): 1.0, (0, 3): 1.0, (0, 130): 1.0, (0, 131): 1.0,
            (0, 228): 1.0, (1, 0): 3 * 2.0 ** -15, (2, 1): 5.5, (3, 0): 1 + 2.0 ** -8,
            (3, 3): 1 + 3 * 2.0 ** -8}
WORKED_FP8 = [901.25 + 2.0 ** -9, 1344 * 2.0 ** -15, 5.5, 448 + 2.0 ** -9]
WORKED_BF16 = [901.25 + 2.0 ** -9 + 2.0 ** -10, 1344 * 2.0 ** -15, 5.84375,
               448 + (1 + 2.0 ** -6) * 2.0 ** -9]


def _worked_inputs():
    SX = np.zeros((256, 1))
    for b, v in WORKED_SX.items():
        SX[b, 0] = v
    G = np.zeros((4, 256))
    for (i, b), v in WORKED_G.items():
        G[i, b] = v
    return G, SX


def test_emulate_reduced_worked_case():
    G, SX = _worked_inputs()
    assert list(O.emulate_reduced(G, SX, "fp8")[:, 0]) == WORKED_FP8
    assert list(O.emulate_reduced(G, SX, "bf16")[:, 0]) == WORKED_BF16
