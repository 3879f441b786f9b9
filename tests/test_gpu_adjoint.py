"""The adjoint kernels (Z = G^T dY on MFMA, then the signed row gather) and
the autograd binding, against the oracle's FP64 adjoint, the adjoint
identity and central finite differences of the oracle forward."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1606_05732_amd as cg
from paper_1606_05732_amd import workloads as W
from tests.gpu_util import csr_to_gpu, rel, say

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-5, torch.float64: 1e-12}
NPD = {torch.float32: np.float32, torch.float64: np.float64}


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
# d multiple of 4 takes the 16-byte gather (8, 12, 64, 132: two to 33
# lanes per row), the others the scalar one
@pytest.mark.parametrize("n,d,m,B", [(1, 1, 1, 1), (3000, 10, 20, 2000), (5003, 64, 128, 4096),
                                     (999, 17, 70, 333), (500, 130, 9, 100), (7001, 8, 16, 1000),
                                     (3001, 12, 40, 777), (600, 132, 24, 300)])
def test_dense_adjoint_parity(cuda, dtype, n, d, m, B):
    rng = np.random.default_rng(n + m)
    dY = rng.standard_normal((m, d)).astype(NPD[dtype])
    seed = 41
    say("adjoint dense", dtype, n, d, m, B)
    dX = cg.sketch_adjoint(torch.from_numpy(dY).to(cuda), n, m, B, seed)
    torch.cuda.synchronize()
    ref = O.adjoint_dense(dY.astype(np.float64), n, d, m, B, seed)
    assert rel(dX.cpu().numpy(), ref) < TOL[dtype]


@pytest.mark.parametrize("pad,shift", [(4, 0), (3, 1)])
def test_dense_adjoint_into_strided_output(cuda, pad, shift):
    """dX written into a wider buffer: row stride d + pad, starting `shift`
    floats in (16-byte aligned rows take the vector gather, the rest the
    scalar one); the columns around it stay untouched."""
    n, d, m, B, seed = 4099, 64, 32, 2048, 17
    rng = np.random.default_rng(5)
    dY = rng.standard_normal((m, d)).astype(np.float32)
    buf = torch.full((n, d + pad), 7.0, device=cuda)
    out = buf[:, shift:shift + d]
    say("adjoint strided out", pad, shift)
    cg.sketch_adjoint(torch.from_numpy(dY).to(cuda), n, m, B, seed, out=out)
    torch.cuda.synchronize()
    ref = O.adjoint_dense(dY.astype(np.float64), n, d, m, B, seed)
    assert rel(out.cpu().numpy(), ref) < TOL[torch.float32]
    rest = torch.cat([buf[:, :shift], buf[:, shift + d:]], dim=1)
    assert torch.all(rest == 7.0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_csr_adjoint_parity_and_identity(cuda, dtype):
    rng = np.random.default_rng(5)
    n, d, m, B, seed = 7000, 24, 40, 900, 3
    rp, ci, v = W.csr_bernoulli(rng, n, d, 0.1, dtype=NPD[dtype])
    dY = rng.standard_normal((m, d)).astype(NPD[dtype])
    say("adjoint csr", dtype)
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    dv = cg.sketch_adjoint_csr(X, torch.from_numpy(dY).to(cuda), m, B, seed)
    Y = cg.sketch(X, m, B, seed)
    torch.cuda.synchronize()
    ref = O.adjoint_csr(rp, ci, dY.astype(np.float64), n, d, m, B, seed)
    assert rel(dv.cpu().numpy(), ref) < TOL[dtype]
    lhs = float(np.sum(dY.astype(np.float64) * Y.cpu().numpy()))
    rhs = float(np.sum(dv.cpu().numpy().astype(np.float64) * v))
    assert abs(lhs - rhs) <= 10 * TOL[dtype] * (abs(lhs) + 1)


@pytest.mark.parametrize("case", ["long_rows", "mixed", "sparse_offset"])
def test_csr_adjoint_row_shapes(cuda, case):
    """The CSR gather on rows of about 100 entries (a row spans several of
    a wavefront's 64-entry windows), on short rows with a few long ones, and
    on very sparse rows (mostly empty) with a row offset, against the
    oracle's FP64 adjoint."""
    rng = np.random.default_rng(23)
    row_offset = 0
    if case == "long_rows":
        n, d, m, B, seed = 3001, 200, 24, 700, 8
        rp, ci, v = W.csr_bernoulli(rng, n, d, 0.5, dtype=np.float32)
    elif case == "mixed":
        n, d, m, B, seed = 9000, 160, 20, 1500, 9
        mask = rng.random((n, d)) < 0.02
        mask[rng.choice(n, 12, replace=False)] = rng.random((12, d)) < 0.9
        rp = np.concatenate([[0], np.cumsum(mask.sum(axis=1))]).astype(np.int32)
        ci = np.nonzero(mask)[1].astype(np.int32)
        v = rng.standard_normal(ci.size).astype(np.float32)
    else:
        n, d, m, B, seed = 20003, 16, 16, 4000, 10
        rp, ci, v = W.csr_bernoulli(rng, n, d, 0.01, dtype=np.float32)
        row_offset = 123457
    dY = rng.standard_normal((m, d)).astype(np.float32)
    say("adjoint csr row shapes", case, len(ci))
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    dv = cg.sketch_adjoint_csr(X, torch.from_numpy(dY).to(cuda), m, B, seed, row_offset=row_offset)
    torch.cuda.synchronize()
    ref = O.adjoint_csr(rp, ci, dY.astype(np.float64), n, d, m, B, seed, row_offset=row_offset)
    assert rel(dv.cpu().numpy(), ref) < TOL[torch.float32]


def test_finite_differences_on_slice(cuda):
    """X[0:4096, 0:8] of the gradient workload as its own input, m = 128,
    B = 2^19: the GPU adjoint equals the oracle's FP64 adjoint on every
    entry, and central differences (h = 1e-3) of the oracle's forward on
    every one of the 32768 entries (L = <dY, T X> is linear, so the
    differences are exact up to rounding)."""
    n, d, m, B, seed = 4096, 8, 128, 1 << 19, 2004
    rng = np.random.default_rng(1004)
    X = rng.standard_normal((n, d))
    dY = rng.standard_normal((m, d))
    say("fd slice")
    dX = cg.sketch_adjoint(torch.from_numpy(dY).to(cuda), n, m, B, seed)
    torch.cuda.synchronize()
    dX = dX.cpu().numpy()
    assert rel(dX, O.adjoint_dense(dY, n, d, m, B, seed)) < 1e-12
    # the forward restricted to the buckets the slice touches (G is
    # independent of X, so this is the same function of X): S X by a
    # scatter of the signed rows, then <dY, G S X> = <G^T dY, S X> with
    # G^T dY formed once, so that each of the 65536 evaluations costs one
    # scatter of the perturbed X
    h, sigma = O.hash_rows(seed, B, np.arange(n, dtype=np.uint64))
    used = np.unique(h)
    Gu = np.concatenate([O.gaussian_block(seed, m, int(b), 1) for b in used], axis=1)
    P = (Gu.T @ dY).ravel()
    cell = (np.searchsorted(used, h)[:, None] * d + np.arange(d)[None, :]).ravel()
    sig = np.repeat(sigma.astype(np.float64), d)

    def loss(Z):
        SX = np.bincount(cell, weights=sig * Z.ravel(), minlength=len(used) * d)
        return float(P @ SX)

    entries = [(r, c) for r in range(n) for c in range(d)]
    fd = O.central_fd(loss, X, entries, 1e-3)
    got = dX.ravel()
    assert np.allclose(got, fd, rtol=1e-7, atol=1e-8)


def test_autograd_linear_and_quadratic(cuda):
    rng = np.random.default_rng(8)
    n, d, m, B, seed = 6000, 16, 32, 777, 12
    X = torch.from_numpy(rng.standard_normal((n, d))).to(cuda).requires_grad_(True)
    dY = torch.from_numpy(rng.standard_normal((m, d))).to(cuda)
    say("autograd")
    Y = cg.countgauss(X, m, B, seed)
    (Y * dY).sum().backward()
    torch.cuda.synchronize()
    ref = O.adjoint_dense(dY.cpu().numpy(), n, d, m, B, seed)
    assert rel(X.grad.cpu().numpy(), ref) < 1e-12
    # L(w) = ||T (X w - y)||^2, T acting on an n-vector
    Xn = X.detach()
    w = torch.from_numpy(rng.standard_normal(d)).to(cuda).requires_grad_(True)
    y = torch.from_numpy(rng.standard_normal(n)).to(cuda)
    r = (Xn @ w - y)[:, None]
    loss = (cg.countgauss(r, m, B, seed) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    rn = (Xn.cpu().numpy() @ w.detach().cpu().numpy() - y.cpu().numpy())[:, None]
    g_ref = Xn.cpu().numpy().T @ O.adjoint_dense(2 * O.sketch_dense(rn, m, B, seed), n, 1, m, B,
                                                 seed)[:, 0]
    assert rel(w.grad.cpu().numpy(), g_ref) < 1e-12
    assert abs(loss.item() - float(np.sum(O.sketch_dense(rn, m, B, seed) ** 2))) < 1e-9 * loss.item()


def test_autograd_through_csr_values(cuda):
    """countgauss on a CSR matrix differentiates with respect to its stored
    values: against the oracle's CSR adjoint (FP64), central differences of
    the oracle forward over every stored entry, and the quadratic loss
    ||T X||^2 whose gradient is 2 T^T (T X)."""
    rng = np.random.default_rng(19)
    n, d, m, B, seed = 2000, 8, 16, 500, 23
    rp, ci, v = W.csr_bernoulli(rng, n, d, 0.1, dtype=np.float64)
    dY = rng.standard_normal((m, d))
    say("autograd csr", n, d, len(v))
    vals = torch.from_numpy(v.copy()).to(cuda).requires_grad_(True)
    X = cg.CsrMatrix(torch.from_numpy(rp).to(cuda), torch.from_numpy(ci).to(cuda), vals, n, d)
    Y = cg.countgauss(X, m, B, seed)
    (Y * torch.from_numpy(dY).to(cuda)).sum().backward()
    torch.cuda.synchronize()
    g = vals.grad.cpu().numpy()
    assert rel(g, O.adjoint_csr(rp, ci, dY, n, d, m, B, seed)) < 1e-12

    def loss(V):
        return float(np.sum(dY * O.sketch_csr(rp, ci, V[:, 0], n, d, m, B, seed)))

    fd = O.central_fd(loss, v[:, None], [(k, 0) for k in range(len(v))], 1e-3)
    assert np.allclose(g, fd, rtol=1e-7, atol=1e-8)
    vals.grad = None
    Y = cg.countgauss(X, m, B, seed)
    (Y ** 2).sum().backward()
    torch.cuda.synchronize()
    y_ref = O.sketch_csr(rp, ci, v, n, d, m, B, seed)
    assert rel(vals.grad.cpu().numpy(), O.adjoint_csr(rp, ci, 2 * y_ref, n, d, m, B, seed)) < 1e-12
    # FP32 values through the same path
    v32 = torch.from_numpy(v.astype(np.float32)).to(cuda).requires_grad_(True)
    X32 = cg.CsrMatrix(X.row_ptr, X.col_idx, v32, n, d)
    (cg.countgauss(X32, m, B, seed) * torch.from_numpy(dY.astype(np.float32)).to(cuda)).sum().backward()
    torch.cuda.synchronize()
    assert rel(v32.grad.cpu().numpy(), O.adjoint_csr(rp, ci, dY.astype(np.float32).astype(np.float64),
                                                     n, d, m, B, seed)) < 1e-5


def test_workload4_full_size_adjoint(cuda):
    """n = 2^22, d = 64, m = 128, B = 2^19, FP32 upstream dY ~ N(0,1): the
    whole dX against the oracle, plus the gradient of ||T (X w - y)||^2."""
    w = W.workload4()
    dY = w.extra["dY"].astype(np.float32)
    say("workload4 adjoint full")
    dX = cg.sketch_adjoint(torch.from_numpy(dY).to(cuda), w.n, w.m, w.B, w.seed)
    torch.cuda.synchronize()
    ref = O.adjoint_dense(dY.astype(np.float64), w.n, w.d, w.m, w.B, w.seed)
    assert rel(dX.cpu().numpy(), ref) < 1e-5
    del dX
    Xg = torch.from_numpy(w.dense).to(cuda)
    wt = torch.from_numpy(w.extra["w"].astype(np.float32)).to(cuda).requires_grad_(True)
    y = torch.from_numpy(w.extra["y"].astype(np.float32)).to(cuda)
    r = (Xg @ wt - y)[:, None]
    loss = (cg.countgauss(r, w.m, w.B, w.seed) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    rn = (w.dense.astype(np.float64) @ w.extra["w"].astype(np.float32).astype(np.float64)
          - w.extra["y"].astype(np.float32))[:, None]
    g_ref = w.dense.astype(np.float64).T @ O.adjoint_dense(
        2 * O.sketch_dense(rn, w.m, w.B, w.seed), w.n, 1, w.m, w.B, w.seed)[:, 0]
    assert rel(wt.grad.cpu().numpy(), g_ref) < 1e-4
