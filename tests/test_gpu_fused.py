"""The fused single pass (CG_SX_FUSED): each bucket range's S X slice is
summed in LDS and multiplied at once by G's columns of those buckets, so
S X never reaches memory.  Against the FP64 oracle (FP32 1e-5), the binned
route, bitwise reproducibility, and its rejections; the FP32 CSR workload
at full size."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1606_05732_amd as cg
from paper_1606_05732_amd import workloads as W
from tests.gpu_util import csr_to_gpu, rel, say

pytestmark = pytest.mark.gpu

# d across the 16-column blocks and past 64 (column groups), m across the
# 64-row groups, B with ragged last ranges and B = 1
SHAPES = [(1, 1, 1.0, 1, 1), (3000, 10, 0.05, 20, 2000), (70001, 32, 0.05, 64, 65536),
          (4099, 17, 0.3, 65, 777), (20000, 64, 0.05, 130, 5000), (900, 300, 0.1, 33, 1000),
          (5000, 7, 0.0, 16, 100), (40000, 65, 0.02, 9, 3000)]


@pytest.mark.parametrize("n,d,p,m,B", SHAPES)
def test_fused_parity_and_determinism(cuda, n, d, p, m, B):
    rp, ci, v = W.csr_bernoulli(np.random.default_rng(n + d), n, d, p, dtype=np.float32,
                                absolute=True)
    seed = 5100 + n
    say("fused", n, d, p, m, B)
    X = csr_to_gpu(rp, ci, v, n, d)
    Y = cg.sketch(X, m, B, seed, algo="fused")
    Y2 = cg.sketch(X, m, B, seed, algo="fused")
    Yb = cg.sketch(X, m, B, seed, algo="binned")
    torch.cuda.synchronize()
    y = Y.cpu().numpy()
    assert np.array_equal(y.view(np.uint32), Y2.cpu().numpy().view(np.uint32))
    ref = O.sketch_csr(rp, ci, v.astype(np.float64), n, d, m, B, seed)
    if len(v) == 0:
        assert np.all(y == 0)
        return
    assert rel(y, ref) < 1e-5
    assert rel(y, Yb.cpu().numpy()) < 2e-6


def test_fused_keeps_fp32_accuracy_with_mixed_magnitudes(cuda):
    # the second pass of the fixed-point sums (remainders) on the fused path
    from tests.test_gpu_binned_precision import _mixed_magnitude_csr
    n, d, p, m, B = 200000, 8, 0.5, 16, 4096
    rp, ci, v = _mixed_magnitude_csr(n, d, p, 85)
    say("fused mixed magnitudes")
    Y = cg.sketch(csr_to_gpu(rp, ci, v, n, d), m, B, 85, algo="fused")
    torch.cuda.synchronize()
    ref = O.sketch_csr(rp, ci, v.astype(np.float64), n, d, m, B, 85)
    y = Y.cpu().numpy()
    for j in range(d):
        assert rel(y[:, j], ref[:, j]) < 1e-5


def test_fused_rejections(cuda):
    rp, ci, v = W.csr_bernoulli(np.random.default_rng(1), 100, 4, 0.5, dtype=np.float64)
    X64 = csr_to_gpu(rp, ci, v, 100, 4)
    with pytest.raises(cg.CountGaussError):
        cg.sketch(X64, 8, 16, 1, algo="fused")
    X32 = csr_to_gpu(rp, ci, v.astype(np.float32), 100, 4)
    with pytest.raises(cg.CountGaussError):
        cg.sketch(X32, 8, 16, 1, algo="fused", sx_out=torch.empty((16, 4), device=cuda))
    with pytest.raises(cg.CountGaussError):
        cg.sketch(X32, 8, 16, 1, algo="fused", precision="bf16")
    with pytest.raises(cg.CountGaussError):
        cg.sketch(torch.ones((10, 4), device=cuda), 8, 16, 1, algo="fused")


def test_fused_full_size_workload(cuda):
    w = W.workload2()
    c = w.csr
    say("fused full size", c.n, c.d, c.nnz)
    Y = cg.sketch(csr_to_gpu(c.row_ptr, c.col_idx, c.vals, c.n, c.d), w.m, w.B, w.seed, algo="fused")
    torch.cuda.synchronize()
    ref = O.sketch_csr(c.row_ptr, c.col_idx, c.vals, c.n, c.d, w.m, w.B, w.seed)
    assert rel(Y.cpu().numpy(), ref) < 1e-5
