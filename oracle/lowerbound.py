"""Quantities of the paper's Section 7 (Theorem 1's proof and the
lower-bound lemma), in FP64 (test infrastructure only, like the rest of
oracle/).

For an n x d matrix U with orthonormal columns and a CountSketch S, the
rows of G S U are i.i.d. N(0, M) given S, with M = (S U)^T (S U), while the
rows of G~ U are N(0, I).  The proof of Theorem 1 bounds
  KL(N(0, I) || N(0, M)) = 1/2 tr(M^-1 - I) + 1/2 ln det M
(the claim on the KL divergence between Gaussians) through
||I - M||_F^2 = O(d^2 / B), and the total variation of the m rows through
Pinsker's inequality and additivity of KL: TV <= sqrt(m KL / 2).  The
lower-bound lemma builds U from disjoint blocks of L = ceil(sqrt(B) / d)
rows per column and distinguishes the two distributions by the squared
norms ||Y (e_i + e_j)||^2, which are near 2 m for G~ U and, after a unique
collision between two columns' blocks, near m (2 + (2 / L) sigma_a sigma_b)
for T U.
"""
import math

import numpy as np

from .countgauss import hash_rows

__all__ = ["pair_norms", "pair_deviation", "kl_to_standard", "pinsker_tv_bound",
           "frobenius_gap", "expected_frobenius_gap", "colliding_pairs"]


def pair_norms(Y):
    """||Y (e_i + e_j)||^2 for every pair i < j of columns of Y, as a
    d x d matrix (upper triangle; the rest is NaN)."""
    Y = np.asarray(Y, dtype=np.float64)
    d = Y.shape[1]
    out = np.full((d, d), np.nan)
    for i in range(d):
        for j in range(i + 1, d):
            v = Y[:, i] + Y[:, j]
            out[i, j] = float(v @ v)
    return out


def pair_deviation(Y, m):
    """max over pairs i < j of | ||Y (e_i + e_j)||^2 - 2 m |: the lemma's
    distinguishing statistic for U with orthonormal columns (0 for d < 2)."""
    P = pair_norms(Y)
    vals = P[np.isfinite(P)]
    return float(np.max(np.abs(vals - 2.0 * m))) if vals.size else 0.0


def kl_to_standard(M):
    """KL(N(0, I) || N(0, M)) = 1/2 tr(M^-1 - I) + 1/2 ln det M for a
    symmetric positive definite M; +inf if M is not positive definite."""
    M = np.asarray(M, dtype=np.float64)
    d = M.shape[0]
    w = np.linalg.eigvalsh(M)
    if w.min() <= 0.0:
        return math.inf
    return 0.5 * (float(np.sum(1.0 / w)) - d) + 0.5 * float(np.sum(np.log(w)))


def pinsker_tv_bound(kl, m):
    """Pinsker's inequality with KL additive over m independent rows:
    TV <= sqrt(m KL / 2), capped at 1.  KL is nonnegative (Gibbs); a value
    a rounding below zero (M equal to I up to rounding) counts as zero."""
    if not math.isfinite(kl):
        return 1.0
    return min(1.0, math.sqrt(m * max(kl, 0.0) / 2.0))


def frobenius_gap(M):
    """||I - M||_F^2."""
    M = np.asarray(M, dtype=np.float64)
    return float(np.sum((np.eye(M.shape[0]) - M) ** 2))


def expected_frobenius_gap(U, B):
    """E_S ||U^T S^T S U - U^T U||_F^2 for a CountSketch with independent
    uniform buckets and signs: every unordered pair of rows {r, s} collides
    with probability 1/B and then contributes sigma_r sigma_s
    (u_r u_s^T + u_s u_r^T), whose squared norm is
    2 ((u_r . u_s)^2 + ||u_r||^2 ||u_s||^2); different pairs are
    uncorrelated.  Summed over the pairs:
    ((tr C)^2 + ||C||_F^2 - 2 sum_r ||u_r||^4) / B with C = U^T U."""
    U = np.asarray(U, dtype=np.float64)
    C = U.T @ U
    r4 = float(np.sum(np.sum(U * U, axis=1) ** 2))
    return (float(np.trace(C)) ** 2 + float(np.sum(C * C)) - 2.0 * r4) / B


def colliding_pairs(seed, B, d, L, row_offset=0):
    """The pairs (a, b), a < b, of rows of the block matrix U (rows of
    column i: L i .. L i + L - 1) in distinct blocks that S puts into the
    same bucket.  The lemma's event is that there is exactly one."""
    n = L * d
    h, _ = hash_rows(seed, B, np.arange(n, dtype=np.uint64) + np.uint64(row_offset))
    pairs = []
    for a in range(n):
        for b in range(a + 1, n):
            if a // L != b // L and h[a] == h[b]:
                pairs.append((a, b))
    return pairs
