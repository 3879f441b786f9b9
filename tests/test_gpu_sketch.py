"""Parity of the HIP forward path with the FP64 oracle.

Tolerances (relative Frobenius error against FP64): FP64 data 1e-12, FP32
1e-5.  S X itself is compared too: the atomic FP32 path sums each bucket's
contributions in a run-dependent order, so it matches to rounding; the
sorted path must give the same bits on every run.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1606_05732_amd as cg
from paper_1606_05732_amd import workloads as W
from tests.gpu_util import csr_to_gpu, rel, say

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-5, torch.float64: 1e-12}
SXTOL = {torch.float32: 2e-6, torch.float64: 1e-13}
NPD = {torch.float32: np.float32, torch.float64: np.float64}


def _dense_case(n, d, seed, dtype):
    X = np.random.default_rng(seed).standard_normal((n, d)).astype(NPD[dtype])
    return X


# n spans several 1024-row workgroups with a ragged tail; d crosses the
# 8/16/32/64 lane-group boundaries and the wide path; m crosses 64-row
# groups of G; B includes 1 and non-powers of two.
SHAPES = [
    (1, 1, 1, 1), (5, 3, 7, 2), (3000, 10, 20, 2000), (5000, 32, 64, 4096),
    (4099, 17, 65, 777), (2500, 64, 130, 5000), (1500, 65, 9, 300), (700, 300, 33, 1000),
    (2000, 40, 64, 700),
]


def _binned_applies(dtype, d, csr):
    return dtype == torch.float32 and (csr or d <= 64)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n,d,m,B", SHAPES)
@pytest.mark.parametrize("algo", ["atomic", "sorted", "binned", "auto"])
def test_dense_parity(cuda, dtype, n, d, m, B, algo):
    X = _dense_case(n, d, n + d, dtype)
    seed = 1234 + n
    say("dense", dtype, n, d, m, B, algo)
    Xg = torch.from_numpy(X).to(cuda)
    SX = torch.empty((B, d), dtype=dtype, device=cuda)
    if algo == "binned" and not _binned_applies(dtype, d, False):
        with pytest.raises(cg.CountGaussError):
            cg.sketch(Xg, m, B, seed, algo=algo)
        return
    Y = cg.sketch(Xg, m, B, seed, algo=algo, sx_out=SX)
    torch.cuda.synchronize()
    sx_ref = O.sx_dense(X.astype(np.float64), seed, B)
    y_ref = O.sketch_dense(X.astype(np.float64), m, B, seed)
    assert rel(SX.cpu().numpy(), sx_ref) < SXTOL[dtype]
    assert rel(Y.cpu().numpy(), y_ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n,d,p,m,B", [
    (1, 1, 1.0, 1, 1), (4097, 10, 0.01, 20, 2000), (20000, 32, 0.05, 64, 4096),
    (3001, 17, 0.3, 70, 555), (1000, 200, 0.2, 16, 64), (777, 8, 0.0, 5, 100),
])
@pytest.mark.parametrize("algo", ["atomic", "sorted", "binned", "auto"])
def test_csr_parity(cuda, dtype, n, d, p, m, B, algo):
    rng = np.random.default_rng(n * 7 + d)
    rp, ci, v = W.csr_bernoulli(rng, n, d, p, dtype=NPD[dtype], absolute=True)
    seed = 99 + d
    say("csr", dtype, n, d, p, m, B, algo, "nnz", len(ci))
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    SX = torch.empty((B, d), dtype=dtype, device=cuda)
    if algo == "binned" and not _binned_applies(dtype, d, True):
        with pytest.raises(cg.CountGaussError):
            cg.sketch(X, m, B, seed, algo=algo)
        return
    Y = cg.sketch(X, m, B, seed, algo=algo, sx_out=SX)
    torch.cuda.synchronize()
    sx_ref = O.sx_csr(rp, ci, v, n, d, seed, B)
    y_ref = O.sketch_csr(rp, ci, v, n, d, m, B, seed)
    assert rel(SX.cpu().numpy(), sx_ref) < SXTOL[dtype]
    if len(ci):
        assert rel(Y.cpu().numpy(), y_ref) < TOL[dtype]
    else:
        assert np.all(Y.cpu().numpy() == 0)


def test_row_offset_chunks_add_up(cuda):
    X = _dense_case(10001, 12, 5, torch.float64)
    Xg = torch.from_numpy(X).to(cuda)
    m, B, seed = 24, 999, 77
    say("row_offset chunks")
    full = cg.sketch(Xg, m, B, seed)
    parts = cg.sketch(Xg[:3333], m, B, seed) + cg.sketch(Xg[3333:], m, B, seed, row_offset=3333)
    torch.cuda.synchronize()
    ref = O.sketch_dense(X, m, B, seed)
    assert rel(full.cpu().numpy(), ref) < 1e-12
    assert rel(parts.cpu().numpy(), ref) < 1e-12
    # an offset that is not a multiple of four exercises the two-block hash
    ref2 = O.sketch_dense(X[:501], m, B, seed, row_offset=2 ** 32 + 3)
    got = cg.sketch(Xg[:501], m, B, seed, row_offset=2 ** 32 + 3)
    assert rel(got.cpu().numpy(), ref2) < 1e-12


# A 64-row group of G holding at most 32 rows (m <= 32, or the last group
# of a larger m) draws each Philox block once per two column steps and
# moves half of the normals across lanes.  The MFMA operands for the rows
# that exist are those of a full group, and G for m rows is the top rows of
# G for more rows, so these rows must equal the first rows of a larger m
# bit for bit (same split: kc is fixed, and both m have as many groups).
# S X must be the same bits in both calls: the sorted path for dense X,
# the binned path (fixed point) for CSR X.
@pytest.mark.parametrize("m_small,m_big", [(32, 64), (1, 64), (17, 64), (96, 128), (70, 128)])
@pytest.mark.parametrize("kind", ["dense64", "dense32", "csr32"])
def test_half_group_rows_equal_full_group_rows(cuda, m_small, m_big, kind):
    B, seed, kc = 5000, 41, 64   # B is not a multiple of the chunk: a ragged last chunk
    if kind == "csr32":
        rng = np.random.Generator(np.random.PCG64(9))
        X = csr_to_gpu(*W.csr_bernoulli(rng, 6000, 64, 0.05, dtype=np.float32), 6000, 64)
        algo = "binned"
    else:
        dt = torch.float64 if kind == "dense64" else torch.float32
        X = torch.from_numpy(_dense_case(3000, 40, 8, dt)).to(cuda)
        algo = "sorted"
    say("half group", kind, m_small, m_big)
    small = cg.sketch(X, m_small, B, seed, kc=kc, algo=algo)
    big = cg.sketch(X, m_big, B, seed, kc=kc, algo=algo)
    torch.cuda.synchronize()
    assert torch.equal(small, big[:m_small])


def test_strided_dense_input(cuda):
    X = np.random.default_rng(3).standard_normal((2000, 40))
    Xg = torch.from_numpy(X).to(cuda)[:, 5:29]        # row stride 40, d = 24
    say("strided")
    Y = cg.sketch(Xg, 16, 300, 8)
    torch.cuda.synchronize()
    assert rel(Y.cpu().numpy(), O.sketch_dense(X[:, 5:29], 16, 300, 8)) < 1e-12


@pytest.mark.parametrize("shift", [0, 1, 2, 3])
def test_binned_csr_any_alignment(cuda, shift):
    """row_ptr, col_idx and vals starting 4 * shift bytes into their buffers
    (the binned kernels use 16-byte loads only where every start is 16-byte
    aligned), with ragged tiles, several input chunks per round and rows
    that straddle chunk boundaries."""
    n, d, m, B, seed = 70001, 32, 40, 8192, 4242
    rng = np.random.Generator(np.random.PCG64(77 + shift))
    rp, ci, v = W.csr_bernoulli(rng, n, d, 0.2, dtype=np.float32)
    say("binned alignment", shift)

    def at(a):
        buf = torch.zeros(a.size + 4, dtype=torch.from_numpy(a).dtype, device=cuda)
        buf[shift:shift + a.size] = torch.from_numpy(a).to(cuda)
        return buf[shift:shift + a.size]

    X = cg.CsrMatrix(at(rp), at(ci), at(v), n, d)
    SX = torch.empty((B, d), dtype=torch.float32, device=cuda)
    Y = cg.sketch(X, m, B, seed, algo="binned", sx_out=SX)
    torch.cuda.synchronize()
    assert rel(SX.cpu().numpy(), O.sx_csr(rp, ci, v, n, d, seed, B)) < SXTOL[torch.float32]
    assert rel(Y.cpu().numpy(), O.sketch_csr(rp, ci, v, n, d, m, B, seed)) < TOL[torch.float32]


@pytest.mark.parametrize("shift,ld", [(0, 64), (1, 65), (4, 68), (0, 66)])
def test_binned_dense_any_alignment(cuda, shift, ld):
    """Dense X at a 4 * shift byte offset with row stride ld (16-byte row
    loads apply only when both keep rows 16-byte aligned)."""
    n, d, m, B, seed = 30011, 64, 32, 4096, 99
    X = np.random.default_rng(5).standard_normal((n, ld + 8)).astype(np.float32)
    Xg = torch.from_numpy(X).to(cuda).reshape(-1)[shift:shift + (n - 1) * (ld + 8) + d]
    Xv = Xg.as_strided((n, d), (ld + 8, 1))
    say("binned dense alignment", shift, ld)
    SX = torch.empty((B, d), dtype=torch.float32, device=cuda)
    Y = cg.sketch(Xv, m, B, seed, algo="binned", sx_out=SX)
    torch.cuda.synchronize()
    Xh = X.reshape(-1)[shift:shift + (n - 1) * (ld + 8) + d]
    Xh = np.lib.stride_tricks.as_strided(Xh, (n, d), ((ld + 8) * 4, 4)).copy()
    assert rel(SX.cpu().numpy(), O.sx_dense(Xh, seed, B)) < SXTOL[torch.float32]
    assert rel(Y.cpu().numpy(), O.sketch_dense(Xh, m, B, seed)) < TOL[torch.float32]


@pytest.mark.parametrize("kind", ["csr", "dense"])
def test_binned_csr_is_bitwise_reproducible(cuda, kind):
    if kind == "dense":
        pytest.skip("dense binned sums in FP32 in a run-dependent order (documented)")
    rng = np.random.default_rng(12)
    n, d, m, B, seed = 200000, 32, 64, 65536, 6
    rp, ci, v = W.csr_bernoulli(rng, n, d, 0.05, dtype=np.float32, absolute=True)
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    say("binned determinism")
    sxs = []
    for _ in range(3):
        SX = torch.empty((B, d), dtype=torch.float32, device=cuda)
        cg.sketch(X, m, B, seed, algo="binned", sx_out=SX)
        sxs.append(SX)
    torch.cuda.synchronize()
    assert torch.equal(sxs[0], sxs[1]) and torch.equal(sxs[0], sxs[2])
    assert rel(sxs[0].cpu().numpy(), O.sx_csr(rp, ci, v, n, d, seed, B)) < 2e-7


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_dense_wide_atomic_many_rows(cuda, dtype):
    """Dense X wider than 64 columns on the atomic path: 64-column groups
    along the grid's second dimension and, for this n, about a hundred rows
    per wavefront (a ragged last run); S X and Y against the oracle."""
    n, d, m, B = 150001, 130, 16, 2500
    X = _dense_case(n, d, 77, dtype)
    seed = 4321
    say("dense wide atomic", dtype, n, d)
    Xg = torch.from_numpy(X).to(cuda)
    SX = torch.empty((B, d), dtype=dtype, device=cuda)
    Y = cg.sketch(Xg, m, B, seed, algo="atomic", sx_out=SX)
    torch.cuda.synchronize()
    assert rel(SX.cpu().numpy(), O.sx_dense(X.astype(np.float64), seed, B)) < SXTOL[dtype]
    assert rel(Y.cpu().numpy(), O.sketch_dense(X.astype(np.float64), m, B, seed)) < TOL[dtype]


def _mixed_density_csr(rng, n, d, block, dense_p, sparse_p, long_rows):
    """CSR whose 1024-row blocks alternate between dense_p and sparse_p
    density, plus the given rows made (almost) full: rounds of both kinds
    in one tile, and long rows inside otherwise sparse rounds."""
    rows = []
    for b0 in range(0, n, block):
        nb = min(block, n - b0)
        p = dense_p if (b0 // block) % 2 == 0 else sparse_p
        mask = rng.random((nb, d)) < p
        rows.extend(mask)
    mask = np.array(rows)
    for r in long_rows:
        mask[r, :] = rng.random(d) < 0.8
    row_ptr = np.concatenate([[0], np.cumsum(mask.sum(axis=1))]).astype(np.int32)
    col_idx = np.nonzero(mask)[1].astype(np.int32)
    vals = rng.standard_normal(col_idx.size).astype(np.float32)
    return row_ptr, col_idx, vals


@pytest.mark.parametrize("d,long_rows", [(32, []), (500, [1024 + 7, 5 * 1024 + 1023, 9 * 1024]),
                                         (64, [3 * 1024 + 500])])
def test_binned_csr_sparse_and_dense_rounds(cuda, d, long_rows):
    """Rounds with few entries take the scatter's sparse path (no stage);
    tiles that mix both kinds of round, and long rows inside sparse rounds
    (their entries spread over the wavefront), must give the oracle's S X,
    the same bits on every run."""
    rng = np.random.default_rng(31 + d)
    n, m, B, seed = 40000, 24, 20000, 5
    # about 2048 entries in a dense round (staged for d = 32 and 64, direct
    # stores for d = 500, whose 1250 ranges leave a small stage), about 50
    # in a sparse one
    rp, ci, v = _mixed_density_csr(rng, n, d, 1024, 2.0 / d, 0.05 / d, long_rows)
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    say("binned sparse/dense rounds", d, len(ci))
    sxs = []
    for _ in range(3):
        SX = torch.empty((B, d), dtype=torch.float32, device=cuda)
        Y = cg.sketch(X, m, B, seed, algo="binned", sx_out=SX)
        sxs.append(SX)
    torch.cuda.synchronize()
    assert torch.equal(sxs[0], sxs[1]) and torch.equal(sxs[0], sxs[2])
    assert rel(sxs[0].cpu().numpy(), O.sx_csr(rp, ci, v, n, d, seed, B)) < SXTOL[torch.float32]
    assert rel(Y.cpu().numpy(), O.sketch_csr(rp, ci, v, n, d, m, B, seed)) < TOL[torch.float32]


@pytest.mark.parametrize("aligned", [True, False])
def test_binned_csr_sparse_rounds_short_rows(cuda, aligned):
    """Sparse rounds whose rows hold 0 to 3 entries: a wavefront whose rows
    all hold at most two entries lets each lane take its own rows' entries,
    one with a 3-entry row spreads the entries over the lanes instead; both
    kinds, and row_ptr with and without 16-byte alignment (the row starts
    then go through LDS), must give the oracle's S X bit-identically."""
    rng = np.random.default_rng(57)
    n, d, m, B, seed = 70000, 16, 20, 30000, 9
    # about 0.4 entries per row: rows of length 0, 1, 2, and 3 in about one
    # wavefront in two (256 rows of 1 in 300 chance each)
    lens = rng.choice([0, 1, 2, 3], size=n, p=[0.7, 0.2, 0.097, 0.003])
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col_idx = np.concatenate([np.sort(rng.choice(d, size=k, replace=False)) for k in lens]).astype(np.int32)
    vals = rng.standard_normal(col_idx.size).astype(np.float32)
    rp_t = torch.from_numpy(row_ptr).to(cuda)
    if not aligned:
        # the same values at a 4-byte offset from a 16-byte boundary
        buf = torch.empty(n + 2, dtype=torch.int32, device=cuda)
        buf[1:].copy_(rp_t)
        rp_t = buf[1:]
        assert rp_t.data_ptr() % 16 != 0
    X = cg.CsrMatrix(rp_t, torch.from_numpy(col_idx).to(cuda), torch.from_numpy(vals).to(cuda), n, d)
    say("binned sparse rounds, short rows", aligned, len(col_idx))
    sxs = []
    for _ in range(3):
        SX = torch.empty((B, d), dtype=torch.float32, device=cuda)
        Y = cg.sketch(X, m, B, seed, algo="binned", sx_out=SX)
        sxs.append(SX)
    torch.cuda.synchronize()
    assert torch.equal(sxs[0], sxs[1]) and torch.equal(sxs[0], sxs[2])
    assert rel(sxs[0].cpu().numpy(), O.sx_csr(row_ptr, col_idx, vals, n, d, seed, B)) < SXTOL[torch.float32]
    assert rel(Y.cpu().numpy(), O.sketch_csr(row_ptr, col_idx, vals, n, d, m, B, seed)) < TOL[torch.float32]


@pytest.mark.parametrize("algo", ["atomic", "binned", "sorted"])
def test_nan_and_inf_reach_their_bucket(cuda, algo):
    rng = np.random.default_rng(13)
    n, d, m, B, seed = 5000, 8, 16, 512, 7
    rp, ci, v = W.csr_bernoulli(rng, n, d, 0.3, dtype=np.float32)
    v[10] = np.nan
    v[20] = np.inf
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    say("nonfinite", algo)
    SX = torch.empty((B, d), dtype=torch.float32, device=cuda)
    Y = cg.sketch(X, m, B, seed, algo=algo, sx_out=SX)
    torch.cuda.synchronize()
    with np.errstate(invalid="ignore"):
        sx_ref = O.sx_csr(rp, ci, v, n, d, seed, B)
        y_ref = O.gaussian_matrix(seed, m, B) @ sx_ref
    got = SX.cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(sx_ref))
    assert np.array_equal(np.isinf(got), np.isinf(sx_ref))
    fin = np.isfinite(sx_ref)
    assert rel(got[fin], sx_ref[fin]) < 2e-6
    assert np.array_equal(np.isfinite(Y.cpu().numpy()), np.isfinite(y_ref))


@pytest.mark.parametrize("kind", ["csr", "dense"])
def test_sorted_path_is_bitwise_reproducible(cuda, kind):
    rng = np.random.default_rng(11)
    n, d, m, B, seed = 30000, 32, 64, 4096, 5
    say("sorted determinism", kind)
    if kind == "csr":
        rp, ci, v = W.csr_bernoulli(rng, n, d, 0.05, dtype=np.float32, absolute=True)
        X = csr_to_gpu(rp, ci, v, n, d, cuda)
    else:
        X = torch.from_numpy(rng.standard_normal((n, d)).astype(np.float32)).to(cuda)
    outs, sxs = [], []
    for _ in range(3):
        SX = torch.empty((B, d), dtype=torch.float32, device=cuda)
        outs.append(cg.sketch(X, m, B, seed, algo="sorted", sx_out=SX))
        sxs.append(SX)
    atomic = cg.sketch(X, m, B, seed, algo="atomic")
    torch.cuda.synchronize()
    for k in (1, 2):
        assert torch.equal(outs[0], outs[k])
        assert torch.equal(sxs[0], sxs[k])
    assert rel(atomic.cpu().numpy(), outs[0].cpu().numpy()) < 1e-5


@pytest.mark.parametrize("algo", ["binned", "atomic", "sorted"])
def test_stage_events_any_subset(cuda, algo):
    """Stage events may be given for any subset of the boundaries (None
    skips one); the result does not depend on them (bit for bit where the
    algorithm is reproducible; the atomic path's order varies), and the
    recorded ones are ordered."""
    import ctypes
    rt = None
    for name in ("libamdhip64.so.7", "libamdhip64.so"):
        try:
            rt = ctypes.CDLL(name)
            break
        except OSError:
            continue
    assert rt is not None, "HIP runtime library not found"
    rt.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                       ctypes.c_void_p]
    rt.hipEventDestroy.argtypes = [ctypes.c_void_p]
    rng = np.random.default_rng(14)
    n, d, m, B, seed = 40000, 16, 32, 8192, 9
    rp, ci, v = W.csr_bernoulli(rng, n, d, 0.1, dtype=np.float32, absolute=True)
    X = csr_to_gpu(rp, ci, v, n, d, cuda)
    plan = cg.SketchPlan(X, m, B, seed, algo=algo)
    plan.run()
    torch.cuda.synchronize()
    ref = plan.Y.clone()
    evs = []
    for _ in range(5):
        h = ctypes.c_void_p()
        assert rt.hipEventCreate(ctypes.byref(h)) == 0
        evs.append(h.value)
    say("stage events", algo)
    for mask in ([1, 0, 1, 0, 0], [0, 0, 0, 0, 1], [1, 1, 1, 1, 1], [0, 0, 0, 0, 0]):
        plan.set_stage_events([h if k else None for h, k in zip(evs, mask)])
        plan.run()
        torch.cuda.synchronize()
        if algo == "atomic":
            assert rel(plan.Y.cpu().numpy(), ref.cpu().numpy()) < TOL[torch.float32]
        else:
            assert torch.equal(plan.Y, ref)
    plan.set_stage_events(None)
    t = ctypes.c_float()
    for a, b in ((0, 1), (1, 2), (2, 3), (3, 4)):
        assert rt.hipEventElapsedTime(ctypes.byref(t), ctypes.c_void_p(evs[a]),
                                      ctypes.c_void_p(evs[b])) == 0
        assert t.value >= 0.0
    for h in evs:
        rt.hipEventDestroy(ctypes.c_void_p(h))


def test_workload1_full_size(cuda):
    """CSR n = 10^6, d = 10, density 1%, m = 20, B = 2000: FP64 and FP32."""
    w = W.workload1()
    c = w.csr
    say("workload1 full")
    ref = O.sketch_csr(c.row_ptr, c.col_idx, c.vals, c.n, c.d, w.m, w.B, w.seed)
    X64 = csr_to_gpu(c.row_ptr, c.col_idx, c.vals, c.n, c.d, cuda)
    X32 = csr_to_gpu(c.row_ptr, c.col_idx, c.vals.astype(np.float32), c.n, c.d, cuda)
    y64 = cg.sketch(X64, w.m, w.B, w.seed)
    y64s = cg.sketch(X64, w.m, w.B, w.seed, algo="sorted")
    y32 = cg.sketch(X32, w.m, w.B, w.seed)
    torch.cuda.synchronize()
    assert rel(y64.cpu().numpy(), ref) < 1e-12
    assert rel(y64s.cpu().numpy(), ref) < 1e-12
    ref32 = O.sketch_csr(c.row_ptr, c.col_idx, c.vals.astype(np.float32), c.n, c.d, w.m, w.B,
                         w.seed)
    assert rel(y32.cpu().numpy(), ref32) < 1e-5


def test_workload2_full_size_csr(cuda):
    """CSR n = 2^24, d = 32, density 5% (27M entries), m = 64, B = 65536,
    FP32, in the launch configuration the benchmark times."""
    w = W.workload2()
    c = w.csr
    say("workload2 full csr", c.nnz)
    X = csr_to_gpu(c.row_ptr, c.col_idx, c.vals, c.n, c.d, cuda)
    SX = torch.empty((w.B, c.d), dtype=torch.float32, device=cuda)
    sx_ref = O.sx_csr(c.row_ptr, c.col_idx, c.vals, c.n, c.d, w.seed, w.B)
    ref = O.gaussian_matrix(w.seed, w.m, w.B) @ sx_ref
    for algo in ("auto", "atomic", "binned", "sorted"):
        y = cg.sketch(X, w.m, w.B, w.seed, sx_out=SX, algo=algo)
        torch.cuda.synchronize()
        assert rel(SX.cpu().numpy(), sx_ref) < 2e-6, algo
        assert rel(y.cpu().numpy(), ref) < 1e-5, algo


def test_workload2_full_size_dense(cuda):
    """Dense n = 2^22, d = 32, FP32, m = 64, B = 65536."""
    w = W.workload2_dense()
    say("workload2 full dense")
    ref = O.sketch_dense(w.dense, w.m, w.B, w.seed)
    Xg = torch.from_numpy(w.dense).to(cuda)
    for algo in ("auto", "atomic", "binned", "sorted"):
        y = cg.sketch(Xg, w.m, w.B, w.seed, algo=algo)
        torch.cuda.synchronize()
        assert rel(y.cpu().numpy(), ref) < 1e-5, algo


@pytest.mark.parametrize("B", [1 << 24, (1 << 26) + 3])
def test_sorted_path_with_far_more_buckets_than_entries(cuda, B):
    """Bucket offsets of the sorted path for B far above the entry count:
    every empty bucket between two keys still gets its offset (one binary
    search per bucket)."""
    n, d, m, seed = 1000, 4, 8, 91
    rp, ci, v = W.csr_bernoulli(np.random.default_rng(7), n, d, 0.5, dtype=np.float32)
    say("sorted B >> count", B)
    X = csr_to_gpu(rp, ci, v, n, d)
    Y = cg.sketch(X, m, B, seed, algo="sorted")
    torch.cuda.synchronize()
    ref = O.sketch_touched(O.csr_to_dense(rp, ci, v, n, d), m, B, seed)
    assert rel(Y.cpu().numpy(), ref) < 1e-5
