"""Per-cell accuracy of the binned CSR S X, whose cells are summed in
two-word 64-bit fixed point with one scale per bucket range.

Columns of very different magnitude share every bucket range here (1e4,
1e-8, and values spread over 2^-30 .. 2^10 within one column), so a
single-word fixed point scaled to the range's largest value would round
the small columns to a few significant bits.  Each column of S X must match
the FP64 oracle at FP32-summation accuracy, and each column of Y at the
FP32 bar, while the sums stay bitwise reproducible.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1606_05732_amd as cg
from paper_1606_05732_amd import workloads as W
from tests.gpu_util import csr_to_gpu, rel, say

pytestmark = pytest.mark.gpu


def _mixed_magnitude_csr(n, d, p, seed):
    rng = np.random.default_rng(seed)
    rp, ci, v = W.csr_bernoulli(rng, n, d, p, dtype=np.float64)
    v = v.copy()
    v[ci == 0] *= 1e4
    v[ci == 1] *= 1e-8
    wide = ci == 2
    v[wide] = np.sign(v[wide]) * np.exp2(rng.uniform(-30.0, 10.0, int(wide.sum())))
    return rp, ci, v.astype(np.float32)


@pytest.mark.parametrize("n,d,p,m,B", [(200000, 8, 0.5, 16, 4096), (60000, 33, 0.2, 20, 20000)])
def test_binned_cells_keep_fp32_accuracy_across_magnitudes(cuda, n, d, p, m, B):
    seed = 77 + d
    rp, ci, v = _mixed_magnitude_csr(n, d, p, seed)
    say("binned mixed magnitudes", n, d, p, m, B)
    X = csr_to_gpu(rp, ci, v, n, d)
    SX = torch.empty((B, d), dtype=torch.float32, device=cuda)
    Y = cg.sketch(X, m, B, seed, algo="binned", sx_out=SX)
    SX2 = torch.empty_like(SX)
    Y2 = cg.sketch(X, m, B, seed, algo="binned", sx_out=SX2)
    torch.cuda.synchronize()
    sx, y = SX.cpu().numpy(), Y.cpu().numpy()
    assert np.array_equal(sx.view(np.uint32), SX2.cpu().numpy().view(np.uint32))
    assert np.array_equal(y.view(np.uint32), Y2.cpu().numpy().view(np.uint32))
    v64 = v.astype(np.float64)
    sx_ref = O.sx_csr(rp, ci, v64, n, d, seed, B)
    y_ref = O.sketch_csr(rp, ci, v64, n, d, m, B, seed)
    for j in range(d):
        # an FP32 sum of a cell's few values is within a few ulp of the cell
        assert rel(sx[:, j], sx_ref[:, j]) < 1e-6, (j, rel(sx[:, j], sx_ref[:, j]))
        assert rel(y[:, j], y_ref[:, j]) < 1e-5, (j, rel(y[:, j], y_ref[:, j]))
