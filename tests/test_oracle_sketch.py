"""Pins of the oracle's S.X, G.(S.X) and adjoint against what the paper and
the mathematics fix: the explicit product, the CountSketch special case
that is an exact isometry, the worked identity in the proof of the
lower-bound lemma (Section 7), the exact second moment of M - X^T X, the
covariance statement behind Theorem 1, and the adjoint/finite differences.
"""
import math

import numpy as np
from scipy import linalg, stats

import oracle as O
from paper_1606_05732_amd.workloads import csr_bernoulli


def _rng(s):
    return np.random.default_rng(s)


def test_three_formulations_agree():
    X = _rng(1).standard_normal((300, 5))
    ys = [O.sketch_dense(X, 7, 50, 123, method=k) for k in ("brute", "scatter", "outer")]
    for y in ys[1:]:
        assert O.rel_frobenius(y, ys[0]) < 1e-13


def test_brute_force_is_the_textbook_triple_product():
    # Y = G S X with S and G explicit; check entrywise with plain loops.
    X = _rng(2).standard_normal((20, 3))
    m, B, seed = 5, 6, 8
    S = O.countsketch_matrix(seed, B, 20)
    G = O.gaussian_matrix(seed, m, B)
    Y = O.sketch_dense(X, m, B, seed)
    for i in range(m):
        for j in range(3):
            acc = 0.0
            for b in range(B):
                for r in range(20):
                    acc += G[i, b] * S[b, r] * X[r, j]
            assert math.isclose(Y[i, j], acc, rel_tol=1e-12, abs_tol=1e-12)


def test_csr_matches_dense_and_row_offset_chunking():
    rng = _rng(3)
    rp, ci, v = csr_bernoulli(rng, 2000, 12, 0.1, dtype=np.float64)
    Xd = O.csr_to_dense(rp, ci, v, 2000, 12)
    yc = O.sketch_csr(rp, ci, v, 2000, 12, 9, 300, 77)
    yd = O.sketch_dense(Xd, 9, 300, 77)
    assert O.rel_frobenius(yc, yd) < 1e-13
    # linearity over row chunks with global row indices
    y2 = O.sketch_dense(Xd[:777], 9, 300, 77) + O.sketch_dense(Xd[777:], 9, 300, 77, row_offset=777)
    assert O.rel_frobenius(y2, yd) < 1e-13


def test_injective_hash_gives_an_exact_isometry():
    # If every row lands in its own bucket, S is a signed partial
    # permutation, so (SX)^T (SX) = X^T X exactly and T.X = G' X with G'
    # a column-signed selection of G (Section 2 intuition: M = U^T S^T S U).
    n, B = 24, 1 << 16
    seed = next(s for s in range(1000)
                if len(set(O.hash_rows(s, B, np.arange(n, dtype=np.uint64))[0])) == n)
    X = _rng(4).standard_normal((n, 5))
    SX = O.sx_dense(X, seed, B)
    assert np.allclose(SX.T @ SX, X.T @ X, rtol=0, atol=1e-12)
    h, sigma = O.hash_rows(seed, B, np.arange(n, dtype=np.uint64))
    G = O.gaussian_matrix(seed, 6, B)
    assert np.allclose(O.sketch_dense(X, 6, B, seed), (G[:, h] * sigma) @ X, atol=1e-12)


def test_lower_bound_lemma_single_collision_identity():
    # Proof of the lower-bound lemma (Section 7): U has L = ceil(sqrt(B)/d)
    # entries 1/sqrt(L) per column in disjoint row blocks.  If exactly one
    # pair of rows (a, b) from two distinct columns i*, j* collides, then
    # ||S U (e_i* + e_j*)||^2 = 2 + (2/L) sigma_a sigma_b, and every other
    # pair of columns keeps ||S U (e_i + e_j)||^2 = 2.
    B, d = 4096, 8
    L = math.ceil(math.sqrt(B) / d)
    n = L * d
    U = np.zeros((n, d))
    for i in range(d):
        U[L * i:L * (i + 1), i] = 1 / math.sqrt(L)
    assert np.allclose(U.T @ U, np.eye(d))
    seen_signs = set()
    for seed in range(2000):
        h, sigma = O.hash_rows(seed, B, np.arange(n, dtype=np.uint64))
        _, inv, cnt = np.unique(h, return_inverse=True, return_counts=True)
        if (cnt > 1).sum() != 1 or cnt.max() != 2:
            continue
        a, b = np.nonzero(cnt[inv] == 2)[0]
        ia, ib = a // L, b // L
        if ia == ib:
            continue
        SU = O.sx_dense(U, seed, B)
        for i in range(d):
            for j in range(i + 1, d):
                v = SU[:, i] + SU[:, j]
                expect = 2 + 2 / L * sigma[a] * sigma[b] if {i, j} == {ia, ib} else 2.0
                assert math.isclose(v @ v, expect, rel_tol=1e-12)
        seen_signs.add(sigma[a] * sigma[b])
        if seen_signs == {1.0, -1.0}:
            break
    assert seen_signs == {1.0, -1.0}


def test_exact_second_moment_of_M_minus_C():
    # Setting of the Frobenius-norm lemma (Section 7): M = X^T S^T S X.
    # For pairwise-uniform h and 4-wise independent signs,
    #   E ||M - C||_F^2 = [(tr C)^2 + ||C||_F^2 - 2 sum_r ||x_r||^4] / B,
    # with C = X^T X (derived from M - C = sum_{r != s} [h(r)=h(s)]
    # sigma_r sigma_s x_r x_s^T).  Monte Carlo over seeds must match it.
    X = np.abs(_rng(5).standard_normal((64, 3)))    # nonnegative, NMF-like
    B, R = 16, 4000
    C = X.T @ X
    pred = (np.trace(C) ** 2 + np.sum(C * C) - 2 * np.sum(np.sum(X * X, 1) ** 2)) / B
    vals = np.empty(R)
    for s in range(R):
        SX = O.sx_dense(X, 10_000 + s, B)
        vals[s] = np.sum((SX.T @ SX - C) ** 2)
    se = vals.std(ddof=1) / math.sqrt(R)
    assert abs(vals.mean() - pred) / se < 4.5


def test_row_covariance_matches_XtX_over_seeds():
    # Theorem 1's content: rows of T X are distributed like rows of G~ X,
    # whose covariance is X^T X; S^T S is the identity in expectation.
    X = _rng(6).standard_normal((40, 3))
    m, B, R = 8, 32, 3000
    C = X.T @ X
    stats_ = np.empty((R, 3, 3))
    ctrl = np.empty((R, 3, 3))
    for s in range(R):
        Y = O.sketch_dense(X, m, B, 50_000 + s)
        stats_[s] = Y.T @ Y / m
        Yt = O.dense_gaussian_block(50_000 + s, m, 0, 40) @ X
        ctrl[s] = Yt.T @ Yt / m
    for arr in (stats_, ctrl):
        z = (arr.mean(0) - C) / (arr.std(0, ddof=1) / math.sqrt(R))
        assert np.max(np.abs(z)) < 4.5


def test_conditional_rows_are_gaussian_with_covariance_M():
    # Proof of Theorem 1: for fixed S the rows of G S X are i.i.d.
    # N(0, M) with M = (SX)^T (SX).  Whitening by M^{-1/2} gives N(0, 1).
    X = _rng(7).standard_normal((2000, 4))
    m, B, seed = 4096, 256, 31
    Y = O.sketch_dense(X, m, B, seed)
    SX = O.sx_dense(X, seed, B)
    W = Y @ np.real(linalg.inv(linalg.sqrtm(SX.T @ SX)))
    assert stats.kstest(W.ravel(), "norm").pvalue > 1e-3
    assert abs(np.mean(W.ravel() ** 2) - 1) < 4.5 * math.sqrt(2 / W.size)


def test_adjoint_identity_dense_and_csr():
    rng = _rng(8)
    n, d, m, B, seed = 500, 6, 9, 77, 5
    X = rng.standard_normal((n, d))
    dY = rng.standard_normal((m, d))
    lhs = np.sum(dY * O.sketch_dense(X, m, B, seed))
    rhs = np.sum(O.adjoint_dense(dY, n, d, m, B, seed) * X)
    assert math.isclose(lhs, rhs, rel_tol=1e-12)
    rp, ci, v = csr_bernoulli(rng, n, d, 0.2, dtype=np.float64)
    lhs = np.sum(dY * O.sketch_csr(rp, ci, v, n, d, m, B, seed))
    rhs = np.sum(O.adjoint_csr(rp, ci, dY, n, d, m, B, seed) * v)
    assert math.isclose(lhs, rhs, rel_tol=1e-12)


def test_adjoint_matches_central_differences():
    rng = _rng(9)
    n, d, m, B, seed = 40, 3, 5, 16, 21
    X = rng.standard_normal((n, d))
    dY = rng.standard_normal((m, d))

    def loss(Z):
        return np.sum(dY * O.sketch_dense(Z, m, B, seed))

    entries = [(r, c) for r in range(n) for c in range(d)]
    fd = O.central_fd(loss, X, entries, 1e-3)
    adj = O.adjoint_dense(dY, n, d, m, B, seed)
    assert np.allclose(fd, [adj[r, c] for r, c in entries], rtol=1e-8, atol=1e-9)

    # quadratic loss ||T (X w - y)||^2 of an n-vector: gradient in w is
    # X^T (T^T (2 T r)), r = X w - y; central differences are exact.
    w = rng.standard_normal(d)
    y = rng.standard_normal(n)

    def lw(wv):
        r = (X @ wv - y)[:, None]
        return float(np.sum(O.sketch_dense(r, m, B, seed) ** 2))

    r = (X @ w - y)[:, None]
    grad = X.T @ O.adjoint_dense(2 * O.sketch_dense(r, m, B, seed), n, 1, m, B, seed)[:, 0]
    fdw = O.central_fd(lambda W: lw(W[0]), w[None, :], [(0, c) for c in range(d)], 1e-3)
    assert np.allclose(fdw, grad, rtol=1e-7)


def _scipy_countsketch(seed, B, n, row_offset=0):
    # S (B x n) as a scipy.sparse matrix straight from the hash: column r
    # holds sigma(r) at row h(r)
    from scipy import sparse
    h, sigma = O.hash_rows(seed, B, np.arange(n, dtype=np.uint64) + np.uint64(row_offset))
    return sparse.csr_matrix((sigma, (h, np.arange(n))), shape=(B, n))


def _csr_cases():
    rng = _rng(11)
    yield csr_bernoulli(rng, 3000, 17, 0.05, dtype=np.float64), 3000, 17, 500, 0
    yield csr_bernoulli(rng, 1000, 64, 0.3, dtype=np.float64, absolute=True), 1000, 64, 4096, 5
    # empty rows at both ends and duplicate columns inside a row
    rp = np.array([0, 0, 3, 3, 6, 6], np.int32)
    ci = np.array([1, 1, 2, 0, 2, 2], np.int32)
    v = np.array([1.5, -2.0, 0.25, 3.0, -1.0, 4.0])
    yield (rp, ci, v), 5, 3, 7, 2 ** 33 + 1


def test_csr_oracle_matches_scipy_sparse_product():
    # S X with scipy.sparse doing the CSR expansion and the product, none of
    # the oracle's own CSR handling involved
    from scipy import sparse
    for (rp, ci, v), n, d, B, off in _csr_cases():
        seed = 40 + n
        Xs = sparse.csr_matrix((v, ci, rp), shape=(n, d))
        ref = (_scipy_countsketch(seed, B, n, off) @ Xs).toarray()
        got = O.sx_csr(rp, ci, v, n, d, seed, B, row_offset=off)
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)
        assert np.allclose(O.csr_to_dense(rp, ci, v, n, d), Xs.toarray(), rtol=0, atol=0)
        y = O.sketch_csr(rp, ci, v, n, d, 6, B, seed, row_offset=off)
        assert np.allclose(y, O.gaussian_matrix(seed, 6, B) @ ref, rtol=1e-12, atol=1e-12)


def test_csr_adjoint_matches_scipy_sparse_transpose():
    # dvals[k] = (S^T Z)[row of k, col_idx[k]], rows from scipy's expansion
    from scipy import sparse
    for (rp, ci, v), n, d, B, off in _csr_cases():
        seed, m = 90 + n, 5
        dY = _rng(n).standard_normal((m, d))
        Z = O.gaussian_matrix(seed, m, B).T @ dY
        dense_grad = np.asarray(_scipy_countsketch(seed, B, n, off).T @ Z)
        coo = sparse.csr_matrix((np.arange(1, len(v) + 1, dtype=np.float64), ci, rp),
                                shape=(n, d)).tocoo()
        order = np.argsort(coo.data)         # back to stored-entry order
        ref = dense_grad[coo.row[order], coo.col[order]]
        got = O.adjoint_csr(rp, ci, dY, n, d, m, B, seed, row_offset=off)
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_touched_columns_formulation_matches_the_full_product():
    # generating only the columns of G that rows hash to changes nothing
    X = _rng(12).standard_normal((200, 4))
    for B, off in ((50, 0), (3000, 7), (1 << 20, 2 ** 33 + 2)):
        ref = O.sketch_dense(X, 9, B, 606, row_offset=off, method="brute" if B < 5000 else "scatter")
        assert O.rel_frobenius(O.sketch_touched(X, 9, B, 606, row_offset=off), ref) < 1e-13
