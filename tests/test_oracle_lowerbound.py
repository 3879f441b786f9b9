"""Pins of the Section 7 quantities in oracle/lowerbound.py against what
the mathematics fixes.

* KL(N(0, I) || N(0, M)) against a Monte Carlo estimate of E_p[ln p - ln q]
  with scipy's multivariate normal log-density, and against numerical
  quadrature of the integral in one dimension.
* Pinsker's bound is at least the exact total variation (quadrature) in
  one dimension.
* The pair statistic on a hand-worked Y, and its distribution for G~ U
  (2-stability: ||G~ U (e_i + e_j)||^2 / 2 is chi-square with m degrees of
  freedom for orthonormal U).
* The lower-bound lemma's identity: after exactly one collision between
  rows a, b of two columns' blocks, ||S U (e_i* + e_j*)||^2 = 2 +
  (2 / L) sigma_a sigma_b, and M has exactly that one nonzero pair.
* The expected ||I - M||_F^2 closed form against a Monte Carlo mean over
  seeds.
"""
import math

import numpy as np
from scipy import integrate, stats

import oracle as O
from oracle import lowerbound as LB
from paper_1606_05732_amd import workloads as W


def test_kl_matches_quadrature_in_one_dimension():
    for s2 in (0.3, 1.0, 1.7, 4.0):
        p = stats.norm(0, 1).pdf
        q = stats.norm(0, math.sqrt(s2)).pdf
        val, _ = integrate.quad(lambda x: p(x) * (math.log(p(x)) - math.log(q(x))), -12, 12)
        assert abs(LB.kl_to_standard(np.array([[s2]])) - val) < 1e-9


def test_kl_matches_monte_carlo_in_four_dimensions():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((4, 4))
    M = np.eye(4) + 0.3 * (A + A.T) / 2
    x = rng.standard_normal((400_000, 4))
    diff = (stats.multivariate_normal(np.zeros(4), np.eye(4)).logpdf(x)
            - stats.multivariate_normal(np.zeros(4), M).logpdf(x))
    mc, se = diff.mean(), diff.std() / math.sqrt(len(diff))
    assert abs(LB.kl_to_standard(M) - mc) < 5 * se
    assert LB.kl_to_standard(np.eye(4)) == 0.0
    assert LB.kl_to_standard(np.diag([1.0, 0.0, 1.0, 1.0])) == math.inf


def test_pinsker_bound_is_above_exact_tv():
    for s2 in (0.2, 0.8, 1.3, 3.0):
        p = stats.norm(0, 1).pdf
        q = stats.norm(0, math.sqrt(s2)).pdf
        tv, _ = integrate.quad(lambda x: 0.5 * abs(p(x) - q(x)), -15, 15, limit=200)
        assert tv <= LB.pinsker_tv_bound(LB.kl_to_standard(np.array([[s2]])), 1) + 1e-12
    assert LB.pinsker_tv_bound(math.inf, 5) == 1.0
    assert LB.pinsker_tv_bound(0.02, 2) == math.sqrt(0.02)


def test_pair_deviation_hand_worked():
    # columns (1, 0), (2, 1), (0, 3) with m = 2:
    # pair (0, 1): (3, 1) -> 10; (0, 2): (1, 3) -> 10; (1, 2): (2, 4) -> 20;
    # deviations from 2 m = 4: 6, 6, 16
    Y = np.array([[1.0, 2.0, 0.0], [0.0, 1.0, 3.0]])
    P = LB.pair_norms(Y)
    assert (P[0, 1], P[0, 2], P[1, 2]) == (10.0, 10.0, 20.0)
    assert LB.pair_deviation(Y, 2) == 16.0
    assert LB.pair_deviation(np.ones((3, 1)), 3) == 0.0


def test_pair_norms_of_gaussian_projection_are_scaled_chi_square():
    d, L, m = 4, 3, 20
    rp, ci, v, n = W.block_orthonormal(d, L)
    q = []
    for s in range(500):
        Y = O.gaussian_product_csr(rp, ci, v, n, d, m, 40_000 + s)
        q.append(LB.pair_norms(Y)[1, 3] / 2.0)
    assert stats.kstest(q, "chi2", args=(m,)).pvalue > 1e-3


def test_unique_collision_moves_one_pair_by_two_over_L():
    d, L, B = 6, 4, 700
    rp, ci, v, n = W.block_orthonormal(d, L)
    seen = 0
    for seed in range(2000):
        pairs = LB.colliding_pairs(seed, B, d, L)
        if len(pairs) != 1:
            continue
        (a, b), = pairs
        h, sigma = O.hash_rows(seed, B, np.arange(n, dtype=np.uint64))
        # no collision inside a block either, so every other pair keeps norm 2
        if len(np.unique(h)) != n - 1:
            continue
        SU = O.sx_csr(rp, ci, v, n, d, seed, B)
        i, j = a // L, b // L
        P = LB.pair_norms(SU)
        assert abs(P[i, j] - (2.0 + 2.0 / L * sigma[a] * sigma[b])) < 1e-12
        others = [P[x, y] for x in range(d) for y in range(x + 1, d) if (x, y) != (i, j)]
        assert np.allclose(others, 2.0, atol=1e-12)
        M = SU.T @ SU
        off = np.abs(M[np.triu_indices(d, 1)]) > 1e-9
        assert off.sum() == 1
        seen += 1
        if seen >= 5:
            break
    assert seen >= 5


def test_expected_frobenius_gap_matches_monte_carlo():
    d, L, B = 5, 6, 400
    rp, ci, v, n = W.block_orthonormal(d, L)
    U = O.csr_to_dense(rp, ci, v, n, d)
    gaps = [LB.frobenius_gap(O.sx_csr(rp, ci, v, n, d, 77_000 + s, B).T
                             @ O.sx_csr(rp, ci, v, n, d, 77_000 + s, B)) for s in range(3000)]
    pred = LB.expected_frobenius_gap(U, B)
    assert abs(pred - (d * d + d - 2.0 * d / L) / B) < 1e-12
    assert abs(np.mean(gaps) - pred) < 4.5 * np.std(gaps) / math.sqrt(len(gaps))


def test_pinsker_bound_of_identity_covariance_is_zero():
    # M = I up to rounding: KL may come out a hair below zero
    assert LB.pinsker_tv_bound(-4e-31, 100) == 0.0
    assert LB.pinsker_tv_bound(LB.kl_to_standard(np.eye(7)), 100) == 0.0
