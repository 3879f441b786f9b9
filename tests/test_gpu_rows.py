"""The rows route (no S X: Y summed over the nonempty rows of CSR X as
sigma(r) G[:, h(r)] x_r^T) against the FP64 oracle, against the binned S X
route, and for bitwise reproducibility."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1606_05732_amd as cg
from paper_1606_05732_amd import workloads as W

from tests.gpu_util import csr_to_gpu, rel, say

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _csr(n, d, p, seed, absolute=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    return W.csr_bernoulli(rng, n, d, p, dtype=np.float32, absolute=absolute)


# n spans several 8192-row parts with a ragged tail; d crosses 16-column
# blocks and 64-column groups; m crosses half and full 64-row groups of G
@pytest.mark.parametrize("n,d,p,m,B", [
    (1, 1, 1.0, 1, 1), (100, 3, 0.3, 5, 7), (9000, 8, 0.01, 32, 2048), (20000, 33, 0.004, 32, 50000),
    (40000, 64, 0.002, 70, 131072), (17000, 100, 0.01, 130, 8192), (3000, 16, 0.0, 8, 100),
    (70001, 24, 0.05, 64, 4096),
])
def test_rows_route_matches_oracle(cuda, n, d, p, m, B):
    rp, ci, v = _csr(n, d, p, n + d)
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    say("rows", n, d, p, m, B, "nnz", len(ci))
    Y = cg.sketch(X, m, B, 11 + d, algo="rows")
    torch.cuda.synchronize()
    ref = O.sketch_csr(rp, ci, v, n, d, m, B, 11 + d)
    if len(ci):
        assert rel(Y.cpu().numpy(), ref) < TOL
    else:
        assert np.all(Y.cpu().numpy() == 0)


def test_long_rows_and_duplicate_columns(cuda):
    """A row holding every column (its entries spread over many lanes and
    over steps), rows next to it empty, and a row that names one column
    twice (duplicates add, as in the oracle)."""
    n, d, m, B, seed = 5000, 1000, 40, 3000, 3
    rows = {7: np.arange(d), 8: np.array([5, 5, 17]), 4095: np.arange(0, d, 3), 4999: np.array([999])}
    rng = np.random.default_rng(1)
    counts = np.zeros(n, np.int64)
    for r, c in rows.items():
        counts[r] = len(c)
    rp = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    ci = np.concatenate([rows[r] for r in sorted(rows)]).astype(np.int32)
    v = rng.standard_normal(ci.size).astype(np.float32)
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    say("rows long/duplicate")
    Y = cg.sketch(X, m, B, seed, algo="rows")
    torch.cuda.synchronize()
    assert rel(Y.cpu().numpy(), O.sketch_csr(rp, ci, v, n, d, m, B, seed)) < TOL


def test_rows_route_is_bitwise_reproducible_and_agrees_with_binned(cuda):
    n, d, m, B, seed = 300000, 64, 32, 131072, 21
    rp, ci, v = _csr(n, d, 0.003, 5)
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    say("rows reproducible")
    ys = [cg.sketch(X, m, B, seed, algo="rows") for _ in range(3)]
    yb = cg.sketch(X, m, B, seed, algo="binned")
    torch.cuda.synchronize()
    assert torch.equal(ys[0], ys[1]) and torch.equal(ys[0], ys[2])
    assert rel(ys[0].cpu().numpy(), yb.cpu().numpy()) < 2e-6
    assert rel(ys[0].cpu().numpy(), O.sketch_csr(rp, ci, v, n, d, m, B, seed)) < TOL


@pytest.mark.parametrize("m_small,m_big", [(32, 64), (9, 64), (96, 128)])
def test_rows_half_groups_equal_full_groups(cuda, m_small, m_big):
    """Half groups of G (at most 32 rows) on the rows route: the rows that
    exist are bit for bit those of a full group (same parts for any m)."""
    n, d, B, seed = 30000, 40, 20000, 8
    rp, ci, v = _csr(n, d, 0.01, 9)
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    say("rows half groups", m_small, m_big)
    small = cg.sketch(X, m_small, B, seed, algo="rows")
    big = cg.sketch(X, m_big, B, seed, algo="rows")
    torch.cuda.synchronize()
    assert torch.equal(small, big[:m_small])


def test_rows_route_row_offset_chunks_add_up(cuda):
    n, d, m, B, seed = 50001, 16, 24, 9999, 13
    rp, ci, v = _csr(n, d, 0.02, 4)
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    cut = 20003   # not a multiple of four: the two-block hash at the seam
    a = cg.CsrMatrix(X.row_ptr[:cut + 1], X.col_idx, X.vals, cut, d)
    rp_b = X.row_ptr[cut:] - X.row_ptr[cut]
    b = cg.CsrMatrix(rp_b.contiguous(), X.col_idx[int(rp[cut]):], X.vals[int(rp[cut]):], n - cut, d)
    say("rows row_offset")
    full = cg.sketch(X, m, B, seed, algo="rows")
    parts = cg.sketch(a, m, B, seed, algo="rows") + cg.sketch(b, m, B, seed, algo="rows", row_offset=cut)
    torch.cuda.synchronize()
    ref = O.sketch_csr(rp, ci, v, n, d, m, B, seed)
    assert rel(full.cpu().numpy(), ref) < TOL
    assert rel(parts.cpu().numpy(), ref) < TOL


def test_nan_and_inf_on_the_rows_route(cuda):
    n, d, m, B, seed = 4000, 8, 16, 500, 2
    rp, ci, v = _csr(n, d, 0.05, 6)
    v = v.copy()
    v[3] = np.inf
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    say("rows inf")
    Y = cg.sketch(X, m, B, seed, algo="rows").cpu().numpy()
    ref = O.sketch_csr(rp, ci, v, n, d, m, B, seed)
    assert np.array_equal(np.isnan(Y), np.isnan(ref)) and np.array_equal(np.isinf(Y), np.isinf(ref))


def test_auto_takes_the_rows_route_where_it_pays(cuda):
    """AUTO picks the rows route for a sparse X with a large B (the result
    equals an explicit rows call bit for bit) and keeps S X for config-2
    shapes scaled down (the result equals the binned call)."""
    rp, ci, v = _csr(200000, 64, 0.002, 7)
    X = csr_to_gpu(rp, ci, v, 200000, 64, cuda)
    say("auto rows")
    y_auto = cg.sketch(X, 32, 131072, 5)
    y_rows = cg.sketch(X, 32, 131072, 5, algo="rows")
    rp2, ci2, v2 = _csr(200000, 32, 0.05, 8, absolute=True)
    X2 = csr_to_gpu(rp2, ci2, v2, 200000, 32, cuda)
    y2_auto = cg.sketch(X2, 64, 4096, 5)
    y2_bin = cg.sketch(X2, 64, 4096, 5, algo="binned")
    torch.cuda.synchronize()
    assert torch.equal(y_auto, y_rows)
    assert torch.equal(y2_auto, y2_bin)


@pytest.mark.parametrize("case", ["fp64", "sx_out", "bf16"])
def test_rows_route_rejects_what_it_cannot_do(cuda, case):
    rp, ci, v = _csr(1000, 8, 0.1, 2)
    if case == "fp64":
        X = csr_to_gpu(rp, ci, v.astype(np.float64), 1000, 8, cuda)
        kw = {}
    else:
        X = csr_to_gpu(rp, ci, v, 1000, 8, cuda)
        kw = {"sx_out": torch.empty((64, 8), device=cuda)} if case == "sx_out" else {"precision": "bf16"}
    with pytest.raises(cg.CountGaussError, match="rows route"):
        cg.sketch(X, 4, 64, 1, algo="rows", **kw)
