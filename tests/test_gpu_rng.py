"""The device random source against the oracle: Philox words and hashes
bit for bit, Gaussians within rounding."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1606_05732_amd as cg
from tests.gpu_util import say, u32

pytestmark = pytest.mark.gpu

SEEDS = [0, 1, 2002, 0x0123456789ABCDEF, 2 ** 64 - 1]


@pytest.mark.parametrize("seed", SEEDS)
def test_philox_words_bit_exact(cuda, seed):
    rng = np.random.default_rng(seed % 1000)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:8] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [0xFFFFFFFF, 0, 0, 0], [0, 0xFFFFFFFF, 0, 0],
               [1, 0, 1, 0], [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
               [123, 456, 1, 0], [7, 0, 0, 0xFFFFFFFF]]
    say("philox", seed)
    out = cg.debug_philox(seed, torch.from_numpy(ctr.view(np.int32)).to(cuda))
    torch.cuda.synchronize()
    ref = O.philox4x32_10(ctr, O.seed_key(seed))
    assert np.array_equal(u32(out), ref)


def test_philox_published_vectors_on_device(cuda):
    ctr = np.array([[0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344]], np.uint32)
    seed = (0x299F31D0 << 32) | 0xA4093822
    out = u32(cg.debug_philox(seed, torch.from_numpy(ctr.view(np.int32)).to(cuda)))
    assert [int(x) for x in out[0]] == [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("B", [1, 7, 2000, 65536, 262143, 2 ** 31 - 1])
@pytest.mark.parametrize("row0", [0, 3, 2 ** 32 - 2, 2 ** 34 + 1])
def test_hash_bit_exact(cuda, seed, B, row0):
    count = 3001
    say("hash", seed, B, row0)
    h, s = cg.debug_hash(seed, B, row0, count, device=cuda)
    torch.cuda.synchronize()
    rows = np.arange(row0, row0 + count, dtype=np.uint64)
    hr, sr = O.hash_rows(seed, B, rows)
    assert np.array_equal(h.cpu().numpy().astype(np.int64), hr)
    assert np.array_equal(s.cpu().numpy().astype(np.float64), sr)


@pytest.mark.parametrize("m,b0,nb", [(64, 0, 4096), (13, 65530, 300), (130, 2 ** 31 - 201, 200),
                                     (64, 1 << 20, 65536)])
def test_gaussian_matches_oracle(cuda, m, b0, nb):
    say("gaussian", m, b0, nb)
    G32 = cg.debug_gaussian(2003, m, b0, nb, torch.float32, cuda).cpu().numpy().astype(np.float64)
    G64 = cg.debug_gaussian(2003, m, b0, nb, torch.float64, cuda).cpu().numpy()
    ref = O.gaussian_block(2003, m, b0, nb)
    # FP64 device Box-Muller: library log/sqrt/sincospi vs numpy; a few ulp
    assert np.max(np.abs(G64 - ref)) < 1e-13
    # FP32: u is exact; the hardware log2/sqrt/sin/cos and the products add
    # a few ulp of a value bounded by 5.77 (largest error seen over 2^22
    # pairs: 8.5e-7) -> 1.5e-6 absolute
    err = np.abs(G32 - ref)
    assert np.max(err) < 1.5e-6, np.max(err)
    assert np.max(np.abs(G32)) <= O.GAUSS_ABS_MAX


@pytest.mark.parametrize("m,B", [(4, 1), (64, 4096), (8, 262145)])
def test_normals_probe_draws_g(cuda, m, B):
    """The generator-only probe draws exactly the normals of G: its
    per-thread sums add up to the sum of the device's G (FP32, different
    order: a rounding-level tolerance) and of the oracle's."""
    say("normals probe", m, B)
    sink = cg.debug_normals(77, m, B, cuda).cpu().numpy().astype(np.float64)
    G = cg.debug_gaussian(77, m, 0, B, torch.float32, cuda).cpu().numpy().astype(np.float64)
    ref = O.gaussian_block(77, m, 0, B)
    tol = 1e-5 * np.sum(np.abs(ref)) + 1e-6
    assert abs(sink.sum() - G.sum()) < tol
    assert abs(sink.sum() - ref.sum()) < tol
