"""Batched instances (cg_sketch_batched) against the FP64 oracle, against
single-instance calls, under other tuning tables, and on the batched
workload (512 instances of uneven n, d, density)."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1606_05732_amd as cg
from paper_1606_05732_amd import autotune
from paper_1606_05732_amd import workloads as W

from tests.gpu_util import csr_to_gpu, rel, say

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5

# (n, d, density, m, B, row_offset): ragged tiles, B = 1, B > n, empty rows,
# an empty matrix, d = 1, d not a power of two, d > 64 (two column groups),
# m > 64 (two row groups), a row offset
MIXED = [
    (1, 1, 1.0, 1, 1, 0), (100, 3, 0.3, 5, 7, 0), (5000, 8, 0.05, 32, 1250, 3),
    (40000, 64, 0.02, 70, 10000, 0), (17000, 33, 0.1, 32, 4096, 1 << 33),
    (2000, 16, 0.0, 8, 100, 0), (30000, 16, 0.005, 32, 8192, 0),
    (1000, 100, 0.2, 16, 5000, 0), (65536 + 77, 32, 0.05, 64, 16384, 0),
]


def _instances(specs, seed0=500):
    out = []
    for k, (n, d, p, m, B, off) in enumerate(specs):
        rng = np.random.Generator(np.random.PCG64(seed0 + k))
        rp, ci, v = W.csr_bernoulli(rng, n, d, p, dtype=np.float32, absolute=(k % 2 == 0))
        out.append(((rp, ci, v, n, d), m, B, 900 + 13 * k, off))
    return out


def _to_gpu(inst):
    return [(csr_to_gpu(*x), m, B, s, off) for (x, m, B, s, off) in inst]


def _oracle(x, m, B, s, off):
    rp, ci, v, n, d = x
    return O.sketch_csr(rp, ci, v, n, d, m, B, s, row_offset=off)


@pytest.fixture(autouse=True)
def _default_tuning():
    cg.set_tuning()
    yield
    cg.set_tuning()


def test_mixed_batch_matches_oracle(cuda):
    inst = _instances(MIXED)
    say("batched mixed", len(inst))
    Ys = cg.sketch_batched(_to_gpu(inst))
    torch.cuda.synchronize()
    for k, (it, Y) in enumerate(zip(inst, Ys)):
        ref = _oracle(*it)
        assert Y.shape == ref.shape
        assert rel(Y.cpu().numpy(), ref) < FP32_TOL, (k, MIXED[k])


def test_batch_equals_single_calls(cuda):
    inst = _instances(MIXED)
    g = _to_gpu(inst)
    say("batched vs single")
    Ys = cg.sketch_batched(g)
    for k, (X, m, B, s, off) in enumerate(g):
        Y1 = cg.sketch(X, m, B, s, row_offset=off)
        torch.cuda.synchronize()
        # same S X (bitwise, fixed point); the contraction differs only in
        # its split order
        assert rel(Ys[k].cpu().numpy(), Y1.cpu().numpy()) < 2e-6, k


def test_batch_is_bitwise_reproducible(cuda):
    g = _to_gpu(_instances(MIXED))
    plan = cg.BatchedSketch(g)
    say("batched reproducible")
    a = [y.clone() for y in plan.run()]
    for _ in range(3):
        b = plan.run()
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y)


@pytest.mark.parametrize("rows,kc", [(1024, 16), (4096, 128), (32768, 2048), (1 << 20, 64)])
def test_other_tuning_tables(cuda, rows, kc):
    inst = _instances(MIXED)
    cg.set_tuning([rows] * 11, [kc] * 11)
    say("batched tuning", rows, kc)
    plan = cg.BatchedSketch(_to_gpu(inst))
    assert plan.plan_fields(3)["tile_rows"] == rows and plan.plan_fields(3)["kc"] == kc
    Ys = plan.run()
    torch.cuda.synchronize()
    for it, Y in zip(inst, Ys):
        assert rel(Y.cpu().numpy(), _oracle(*it)) < FP32_TOL


def test_stale_plan_is_rejected(cuda):
    g = _to_gpu(_instances(MIXED[:3]))
    plan = cg.BatchedSketch(g)
    _, kc = cg.get_tuning()
    cg.set_tuning(None, [2 * k for k in kc])   # any table other than the one planned with
    with pytest.raises(cg.CountGaussError):
        plan.run()


def test_autotuner_keeps_results_exact(cuda):
    inst = _instances(MIXED)
    g = _to_gpu(inst)
    say("autotune small")
    res = autotune.autotune_batched(g, rows_candidates=(4096, 16384), kc_candidates=(128, 1024),
                                    reps=2, warmup=1)
    assert res["ms_after"] <= res["ms_before"]
    assert cg.get_tuning() == (res["rows_per_item"], res["kc_per_item"])
    Ys = cg.sketch_batched(g)
    torch.cuda.synchronize()
    for it, Y in zip(inst, Ys):
        assert rel(Y.cpu().numpy(), _oracle(*it)) < FP32_TOL


def _check_sample(ws, Ys, picks):
    for k in picks:
        w = ws[k]
        c = w.csr
        ref = O.sketch_csr(c.row_ptr, c.col_idx, c.vals, c.n, c.d, w.m, w.B, w.seed)
        assert rel(Ys[k].cpu().numpy(), ref) < FP32_TOL, (k, c.n, c.d, w.B)


def test_workload5_reduced_scale(cuda):
    ws = W.workload5(scale=0.02)
    g = [(csr_to_gpu(w.csr.row_ptr, w.csr.col_idx, w.csr.vals, w.csr.n, w.csr.d), w.m, w.B, w.seed)
         for w in ws]
    say("workload5 x0.02", len(g))
    Ys = cg.sketch_batched(g)
    torch.cuda.synchronize()
    _check_sample(ws, Ys, range(len(ws)))


def test_workload5_full_size(cuda):
    ws = W.workload5()
    g = [(csr_to_gpu(w.csr.row_ptr, w.csr.col_idx, w.csr.vals, w.csr.n, w.csr.d), w.m, w.B, w.seed)
         for w in ws]
    say("workload5 full", len(g), sum(w.csr.nnz for w in ws))
    Ys = cg.sketch_batched(g)
    torch.cuda.synchronize()
    _check_sample(ws, Ys, range(len(ws)))
