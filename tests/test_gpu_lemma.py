"""Section 7 statistics on the GPU (cg_lemma_stats) against the oracle:
the lower-bound lemma's pair statistic of T U and G~ U, and, from S U, the
Frobenius gap, KL divergence, Pinsker bound, off-diagonal count and
positive definiteness of M = (S U)^T (S U), for the lemma's block matrix U."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle import lowerbound as LB
import paper_1606_05732_amd as cg
from paper_1606_05732_amd import workloads as W
from tests.gpu_util import csr_to_gpu, say

pytestmark = pytest.mark.gpu


def _close(a, b, rtol):
    if math.isinf(b):
        return math.isinf(a)
    return abs(a - b) <= rtol * max(1.0, abs(b))


@pytest.mark.parametrize("dtype,rtol", [(np.float64, 1e-10), (np.float32, 1e-4)])
@pytest.mark.parametrize("d,L,m,B", [(16, 4, 64, 1024), (8, 1, 64, 64), (32, 3, 100, 9000),
                                     (64, 2, 40, 5000), (5, 2, 3, 4)])
def test_stats_match_oracle(cuda, dtype, rtol, d, L, m, B):
    rp, ci, v, n = W.block_orthonormal(d, L, dtype=dtype)
    X = csr_to_gpu(rp, ci, v, n, d)
    for seed in (3, 4, 5):
        say("lemma stats", dtype.__name__, d, L, m, B, seed)
        SU = torch.empty((B, d), dtype=X.vals.dtype, device=cuda)
        Y = cg.sketch(X, m, B, seed, algo="atomic", sx_out=SU)
        got = cg.lemma_stats(Y, SU).cpu().numpy()
        Yt = cg.gaussian(torch.from_numpy(O.csr_to_dense(rp, ci, v, n, d).astype(dtype)).to(cuda),
                         m, seed)
        got_t = cg.lemma_stats(Yt).cpu().numpy()
        torch.cuda.synchronize()
        y, su, yt = Y.cpu().numpy(), SU.cpu().numpy(), Yt.cpu().numpy()
        M = su.astype(np.float64).T @ su.astype(np.float64)
        kl = LB.kl_to_standard(M)
        assert _close(got[0], LB.pair_deviation(y, m), rtol)
        assert _close(got[1], LB.frobenius_gap(M), rtol)
        if math.isinf(kl) or not np.all(np.linalg.eigvalsh(M) > 1e-6):
            assert got[5] == 0.0 or got[2] > 1e6
        else:
            assert _close(got[2], kl, 1e3 * rtol)
            # Pinsker's bound is sqrt(m KL / 2): compare its square, which
            # carries the KL tolerance (the root magnifies a KL near zero)
            tv = LB.pinsker_tv_bound(kl, m)
            assert abs(got[3] ** 2 - tv ** 2) <= m / 2 * 1e3 * rtol * max(1.0, abs(kl))
            assert got[5] == 1.0
        assert got[4] == float(np.sum(np.abs(M[np.triu_indices(d, 1)]) > 1e-9))
        assert _close(got_t[0], LB.pair_deviation(yt, m), rtol)
        assert np.all(np.isnan(got_t[1:]))


def test_singular_covariance_is_flagged(cuda):
    # U = I (L = 1) with fewer buckets than columns: two columns of S U
    # coincide up to sign, so M is singular
    d, m, B = 12, 8, 5
    rp, ci, v, n = W.block_orthonormal(d, 1)
    X = csr_to_gpu(rp, ci, v, n, d)
    SU = torch.empty((B, d), dtype=torch.float64, device=cuda)
    Y = cg.sketch(X, m, B, 1, algo="atomic", sx_out=SU)
    got = cg.lemma_stats(Y, SU).cpu().numpy()
    assert got[5] == 0.0 and math.isinf(got[2]) and got[3] == 1.0
