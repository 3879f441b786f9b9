"""Pins of the oracle's random source against things other than itself:
published Philox known-answer vectors, the CountSketch structure stated in
Section 1.1, uniformity/independence statistics, and the normal law.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    out = O.philox4x32_10(np.array(ctr, np.uint32), np.array(key, np.uint32))
    assert [int(x) for x in out] == expect


def test_philox_vectorised_matches_scalar_calls():
    rng = np.random.default_rng(7)
    ctr = rng.integers(0, 2 ** 32, size=(50, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(50, 2), dtype=np.uint64).astype(np.uint32)
    batch = O.philox4x32_10(ctr, key)
    for j in range(50):
        assert np.array_equal(batch[j], O.philox4x32_10(ctr[j], key[j]))


def test_seed_key_split():
    assert list(O.seed_key(0x0123456789ABCDEF)) == [0x89ABCDEF, 0x01234567]
    assert list(O.seed_key(2 ** 64 - 1)) == [0xFFFFFFFF, 0xFFFFFFFF]


def test_hash_uses_one_philox_block_per_four_rows():
    seed, rows = 12345, np.arange(64, dtype=np.uint64)
    w = O.hash_words(seed, rows)
    for q in range(16):
        blk = O.philox4x32_10(np.array([q, 0, 0, 0], np.uint32), O.seed_key(seed))
        assert np.array_equal(w[4 * q:4 * q + 4], blk)
    # rows beyond 2^32 * 4 carry the high word of q into counter word 1
    r = np.array([(1 << 34) + 5], dtype=np.uint64)
    blk = O.philox4x32_10(np.array([1, 1, 0, 0], np.uint32), O.seed_key(seed))
    assert O.hash_words(seed, r)[0] == blk[1]


def test_countsketch_structure_one_signed_entry_per_column():
    # Section 1.1: each column of S has a single nonzero, equal to +-1.
    S = O.countsketch_matrix(99, 37, 500)
    nz = S != 0
    assert np.all(nz.sum(axis=0) == 1)
    assert set(np.unique(S[nz])) <= {-1.0, 1.0}


@pytest.mark.parametrize("B", [64, 1000, 65536, 262143])
def test_bucket_range_and_uniformity(B):
    n = 400000
    h, sigma = O.hash_rows(2024, B, np.arange(n, dtype=np.uint64))
    assert h.min() >= 0 and h.max() < B
    # sign balance: mean of n fair signs has sd 1/sqrt(n)
    assert abs(sigma.mean()) * math.sqrt(n) < 4.5
    if B <= 1000:
        counts = np.bincount(h, minlength=B)
        chi2 = ((counts - n / B) ** 2 / (n / B)).sum()
        assert stats.chi2.sf(chi2, B - 1) > 1e-4
    else:
        # coarse uniformity: 64 equal ranges of buckets
        coarse = np.bincount(h * 64 // B, minlength=64)
        expect = np.array([((k + 1) * B + 63) // 64 - (k * B + 63) // 64
                           for k in range(64)]) * n / B
        chi2 = ((coarse - expect) ** 2 / expect).sum()
        assert stats.chi2.sf(chi2, 63) > 1e-4


def test_pairwise_collisions_and_fourwise_sign_products():
    B, n = 997, 1 << 18
    h, sigma = O.hash_rows(31337, B, np.arange(n, dtype=np.uint64))
    rng = np.random.default_rng(0)
    pairs = 2_000_000
    a = rng.integers(0, n, pairs)
    b = rng.integers(0, n, pairs)
    ok = a != b
    coll = (h[a[ok]] == h[b[ok]]).mean()
    se = math.sqrt((1 / B) * (1 - 1 / B) / ok.sum())
    assert abs(coll - 1 / B) / se < 4.5
    # products of four distinct signs have mean zero (independence)
    idx = rng.integers(0, n, (1_000_000, 4))
    distinct = np.array([len(set(r)) == 4 for r in idx[:200000]])
    idx = idx[:200000][distinct]
    prod = sigma[idx].prod(axis=1)
    assert abs(prod.mean()) * math.sqrt(len(prod)) < 4.5
    # and pairs of signs within one Philox block (rows 4q..4q+3) too
    s4 = sigma[: n - n % 4].reshape(-1, 4)
    for i in range(4):
        for j in range(i + 1, 4):
            assert abs((s4[:, i] * s4[:, j]).mean()) * math.sqrt(len(s4)) < 4.5


def test_uniform_map_is_open_interval_and_exact():
    w = np.array([0, 511, 512, 0xFFFFFFFF, 0x80000000], np.uint32)
    u = O.uniforms_from_words(w)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24
    assert u[2] == 3 * 2.0 ** -24
    assert u[3] == 1 - 2.0 ** -24
    assert np.all((u > 0) & (u < 1))
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_box_muller_pairs_share_a_radius_and_carry_the_angle():
    # The (z0, z1) and (z2, z3) pairs are polar coordinates: radius^2 is
    # -2 ln u0 (resp. u2) and the angle is 2 pi u1 (resp. u3).
    seed, m, b0, nb = 77, 12, 1000, 40
    G = O.gaussian_block(seed, m, b0, nb)
    for q in range(m // 4):
        for j in range(nb):
            ctr = np.array([b0 + j, q, 1, 0], np.uint32)
            w = O.philox4x32_10(ctr, O.seed_key(seed))
            u = O.uniforms_from_words(w)
            z = G[4 * q:4 * q + 4, j]
            assert math.isclose(z[0] ** 2 + z[1] ** 2, -2 * math.log(u[0]), rel_tol=1e-12)
            assert math.isclose(z[2] ** 2 + z[3] ** 2, -2 * math.log(u[2]), rel_tol=1e-12)
            a0 = math.atan2(z[1], z[0]) % (2 * math.pi)
            a1 = math.atan2(z[3], z[2]) % (2 * math.pi)
            assert math.isclose(a0, 2 * math.pi * u[1], rel_tol=1e-9, abs_tol=1e-12)
            assert math.isclose(a1, 2 * math.pi * u[3], rel_tol=1e-9, abs_tol=1e-12)


def test_gaussian_entries_follow_standard_normal():
    G = O.gaussian_matrix(4242, 64, 16384)
    assert stats.kstest(G.ravel(), "norm").pvalue > 1e-3
    for t in range(4):   # each of the four Box-Muller outputs on its own
        assert stats.kstest(G[t::4].ravel(), "norm").pvalue > 1e-3
    assert np.abs(G).max() <= O.GAUSS_ABS_MAX
    # rows are uncorrelated (unit covariance)
    C = np.cov(G[:8])
    assert np.max(np.abs(C - np.eye(8))) < 4.5 / math.sqrt(G.shape[1])


def test_gaussian_nesting_and_independence_of_shape():
    big = O.gaussian_matrix(5, 64, 300)
    assert np.array_equal(O.gaussian_block(5, 13, 17, 100), big[:13, 17:117])
    assert np.array_equal(O.gaussian_matrix(5, 7, 300), big[:7])
    assert not np.array_equal(O.gaussian_matrix(6, 7, 300), big[:7])


def test_dense_comparison_gaussian_is_normal_and_distinct_stream():
    Gt = O.dense_gaussian_block(11, 32, (1 << 33) - 5, 20000)
    assert stats.kstest(Gt.ravel(), "norm").pvalue > 1e-3
    G = O.gaussian_block(11, 32, 0, 20000)
    assert abs(np.corrcoef(G.ravel(), O.dense_gaussian_block(11, 32, 0, 20000).ravel())[0, 1]) < 0.01
