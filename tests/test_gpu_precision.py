"""The precision ladder of the G (S X) contraction: FP32, BF16 and FP8-E4M3
(power-of-two scale per 128-wide block of B) inputs with FP32 accumulation,
each against the FP64 oracle: FP32 <= 1e-5, BF16 <= 1e-2, FP8 <= 5e-2
relative Frobenius error.  The GPU error must also track the oracle's
emulation of the same rounding (within a factor of two either way)."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1606_05732_amd as cg
from paper_1606_05732_amd import workloads as W
from tests.gpu_util import rel, say

pytestmark = pytest.mark.gpu

LIMIT = {"native": 1e-5, "bf16": 1e-2, "fp8": 5e-2}


@pytest.mark.parametrize("n,d,m,B", [(20000, 64, 64, 4096), (9000, 17, 70, 1000),
                                     (3000, 8, 5, 300), (5000, 100, 33, 640),
                                     (4000, 40, 48, 800)])
@pytest.mark.parametrize("prec", ["native", "bf16", "fp8"])
def test_ladder_small(cuda, n, d, m, B, prec):
    rng = np.random.default_rng(n + d)
    X = rng.standard_normal((n, d)).astype(np.float32)
    X[::64] *= 100.0
    seed = 17
    say("ladder", n, d, m, B, prec)
    SX = torch.empty((B, d), dtype=torch.float32, device=cuda)
    Y = cg.sketch(torch.from_numpy(X).to(cuda), m, B, seed, precision=prec, sx_out=SX)
    torch.cuda.synchronize()
    sx = O.sx_dense(X, seed, B)
    G = O.gaussian_matrix(seed, m, B)
    exact = G @ sx
    err = rel(Y.cpu().numpy(), exact)
    assert err < LIMIT[prec], err
    if prec != "native":
        emu = rel(O.emulate_reduced(G, SX.cpu().numpy(), prec), exact)
        assert emu / 2 < err < emu * 2, (err, emu)


@pytest.mark.parametrize("prec", ["native", "bf16", "fp8"])
def test_ladder_workload3_full_size(cuda, prec):
    """Dense n = 2^22, d = 64, every 64th row x100, m = 64, B = 262144."""
    w = _w3()
    say("ladder workload3 full", prec)
    Y = cg.sketch(torch.from_numpy(w.dense).to(cuda), w.m, w.B, w.seed, precision=prec)
    torch.cuda.synchronize()
    err = rel(Y.cpu().numpy(), _w3_ref())
    print(f"workload3 {prec}: relative Frobenius error {err:.3e}")
    assert err < LIMIT[prec]


_cache = {}


def _w3():
    if "w" not in _cache:
        _cache["w"] = W.workload3()
    return _cache["w"]


def _w3_ref():
    if "ref" not in _cache:
        w = _w3()
        _cache["ref"] = O.sketch_dense(w.dense, w.m, w.B, w.seed)
    return _cache["ref"]
