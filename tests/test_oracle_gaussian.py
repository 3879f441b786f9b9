"""Pins of the oracle's dense Gaussian projection G~ X (the product that
T X stands in for: Section 1.1 "Our Results"; Theorem 1 compares G S U
with G~ U), against what the mathematics fixes rather than against the
oracle itself.

* Every entry of G~ X is N(0, ||X[:, j]||^2) (2-stability of the Gaussian,
  used the same way in the proof of the lower-bound lemma, Section 7), so
  the standardized entries pass a KS test against N(0, 1) over seeds, and
  ||G~ x||^2 / ||x||^2 follows chi-square with m degrees of freedom.
* The rows of G~ X have covariance X^T X (unit-variance G~).
* The CSR form equals scipy.sparse's own product of its CSR matrix with the
  explicit G~ (no shared row expansion), and the chunked dense form equals
  the explicit matrix product, at any row offset (chunking by rows)."""
import math

import numpy as np
import scipy.sparse as sp
from scipy import stats

import oracle as O
from paper_1606_05732_amd import workloads as W


def _rng(k):
    return np.random.Generator(np.random.PCG64(7100 + k))


def test_entries_are_normal_with_column_norm_variance():
    X = _rng(0).standard_normal((300, 3)) * np.array([1.0, 10.0, 0.01])
    m, R = 16, 400
    z = np.empty((R, m, 3))
    for s in range(R):
        z[s] = O.gaussian_product_dense(X, m, 90_000 + s) / np.linalg.norm(X, axis=0)
    for j in range(3):
        assert stats.kstest(z[:, :, j].ravel(), "norm").pvalue > 1e-3


def test_squared_norm_is_chi_square_m():
    x = _rng(1).standard_normal((500, 1))
    m, R = 24, 600
    q = np.array([float(np.sum(O.gaussian_product_dense(x, m, 91_000 + s) ** 2)) for s in range(R)])
    q /= float(np.sum(x ** 2))
    assert stats.kstest(q, "chi2", args=(m,)).pvalue > 1e-3


def test_row_covariance_is_XtX():
    X = _rng(2).standard_normal((60, 4))
    m, R = 8, 2500
    C = X.T @ X
    acc = np.empty((R, 4, 4))
    for s in range(R):
        Y = O.gaussian_product_dense(X, m, 92_000 + s)
        acc[s] = Y.T @ Y / m
    z = (acc.mean(0) - C) / (acc.std(0, ddof=1) / math.sqrt(R))
    assert np.max(np.abs(z)) < 4.5


def test_dense_chunking_and_row_offset_match_the_explicit_product():
    X = _rng(3).standard_normal((5000, 6))
    for off in (0, (1 << 32) - 7):
        Gt = O.dense_gaussian_block(17, 11, off, 5000)
        ref = Gt @ X
        for chunk in (1, 333, 1 << 15):
            got = O.gaussian_product_dense(X, 11, 17, row_offset=off, chunk=chunk)
            assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
        # two row blocks with their global offsets add up to the whole
        top = O.gaussian_product_dense(X[:1234], 11, 17, row_offset=off)
        bot = O.gaussian_product_dense(X[1234:], 11, 17, row_offset=off + 1234)
        assert np.abs(top + bot - ref).max() < 1e-12 * np.abs(ref).max()


def test_csr_form_matches_scipy_sparse_product():
    rng = _rng(4)
    n, d, m = 7000, 9, 13
    rp, ci, v = W.csr_bernoulli(rng, n, d, 0.07, dtype=np.float64)
    Xs = sp.csr_matrix((v, ci, rp), shape=(n, d))
    for off in (0, 5 << 32):
        Gt = O.dense_gaussian_block(23, m, off, n)
        ref = np.asarray((Xs.T @ Gt.T).T)
        for chunk in (50, 1 << 15):
            got = O.gaussian_product_csr(rp, ci, v, n, d, m, 23, row_offset=off, chunk=chunk)
            assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_columns_in_any_order_match_the_block():
    rows = np.array([5, 0, (1 << 33) + 2, 77, 3], dtype=np.uint64)
    got = O.dense_gaussian_columns(3, 10, rows)
    for k, r in enumerate(rows):
        assert np.array_equal(got[:, k], O.dense_gaussian_block(3, 10, int(r), 1)[:, 0])


def test_row_quads_on_their_own_match_the_block():
    full = O.dense_gaussian_block(9, 22, 100, 50)
    for q0 in range(6):
        assert np.array_equal(O.dense_gaussian_block(9, 22, 100, 50, q0=q0), full[4 * q0:])
