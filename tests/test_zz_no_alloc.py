"""The allocation-free forward (cg_sketch_csr_noalloc) against cg_sketch_csr.

Both are called through the C ABI on the same seeded CSR inputs.  Two calls
in a row share the static scratch buffer, the second on a smaller input, so
that leftovers of the first call cannot leak into the second.  FP32 data
takes the binned S X (bitwise reproducible), so the two entry points must
agree bit for bit; FP64 data takes the atomic S X, whose summation order
varies, so they must agree to 1e-12 relative (and each match the oracle).
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import paper_1606_05732_amd as cg
from paper_1606_05732_amd import _lib as L
from paper_1606_05732_amd import workloads as W
from tests.gpu_util import csr_to_gpu, rel, say

pytestmark = pytest.mark.gpu

CASES = [  # (n, d, density, m, B, seed): the second of each pair is smaller
    ((200000, 32, 0.05, 64, 32768, 11), (30001, 17, 0.1, 70, 5000, 12)),
    ((100000, 10, 0.02, 20, 2000, 21), (4099, 3, 0.3, 9, 777, 22)),
]


def _noalloc(X, m, B, seed, dtype_code, stream):
    lib = L.load()
    Y = torch.empty((m, X.d), dtype=X.vals.dtype, device=X.vals.device)
    opts = L.make_opts(stream=stream)
    st = lib.cg_sketch_csr_noalloc(
        ctypes.c_void_p(X.row_ptr.data_ptr()), ctypes.c_void_p(X.col_idx.data_ptr()),
        ctypes.c_void_p(X.vals.data_ptr()), dtype_code, X.n, X.d, X.nnz, m, B,
        ctypes.c_uint64(seed), ctypes.c_void_p(Y.data_ptr()), ctypes.byref(opts))
    L.check(st, "cg_sketch_csr_noalloc")
    return Y


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("pair", CASES)
def test_noalloc_matches_cg_sketch_csr_twice(cuda, dtype, pair):
    stream = ctypes.c_void_p(torch.cuda.current_stream(cuda).cuda_stream)
    code = L.CG_DTYPE_F32 if dtype == np.float32 else L.CG_DTYPE_F64
    for (n, d, p, m, B, seed) in pair:
        say("noalloc", dtype.__name__, n, d, p, m, B, seed)
        rp, ci, v = W.csr_bernoulli(np.random.default_rng(seed), n, d, p, dtype=dtype)
        X = csr_to_gpu(rp, ci, v, n, d)
        y_na = _noalloc(X, m, B, seed, code, stream)
        y_ws = cg.sketch(X, m, B, seed)
        torch.cuda.synchronize()
        a, b = y_na.cpu().numpy(), y_ws.cpu().numpy()
        ref = O.sketch_csr(rp, ci, v.astype(np.float64), n, d, m, B, seed)
        if dtype == np.float32:
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
            assert rel(a, ref) < 1e-5
        else:
            assert rel(a, b) < 1e-12
            assert rel(a, ref) < 1e-12
