"""The measured choice of the S X algorithm: it times every algorithm the
library accepts, returns the fastest, and that algorithm's result agrees
with the oracle like any other."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1606_05732_amd as cg
from paper_1606_05732_amd import autotune
from paper_1606_05732_amd import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,d,p,m,B,dtype", [(20000, 16, 0.05, 32, 4096, np.float32),
                                             (5000, 8, 0.1, 20, 500, np.float64)])
def test_choose_algo_picks_an_accepted_algorithm(cuda, n, d, p, m, B, dtype):
    say("choose_algo", n, d, p, m, B, dtype.__name__)
    rp, ci, v = W.csr_bernoulli(np.random.default_rng(3), n, d, p, dtype=dtype, absolute=True)
    X = cg.CsrMatrix(torch.from_numpy(rp).to(cuda), torch.from_numpy(ci).to(cuda),
                     torch.from_numpy(v).to(cuda), n, d)
    res = autotune.choose_algo(X, m, B, 11, reps=2, warmup=1)
    assert res["algo"] in res["ms"]
    assert all(t > 0 for t in res["ms"].values())
    assert set(res["ms"]) | set(res["rejected"]) == {"binned", "atomic", "rows", "fused", "sorted"}
    if dtype == np.float64:
        # FP64 data: the FP32-only routes say so instead of running
        assert {"rows", "fused"} <= set(res["rejected"])
    Y = cg.sketch(X, m, B, 11, algo=res["algo"]).cpu().numpy()
    ref = O.sketch_csr(rp, ci, v, n, d, m, B, 11)
    tol = 1e-12 if dtype == np.float64 else 1e-5
    assert np.linalg.norm(Y - ref) <= tol * np.linalg.norm(ref)
