"""Helpers for the gpu-marked tests: move seeded inputs to the device and
compare with the oracle."""
import sys

import numpy as np
import torch

from paper_1606_05732_amd import CsrMatrix


def say(*a):
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def csr_to_gpu(rp, ci, v, n, d, dev="cuda"):
    return CsrMatrix(torch.from_numpy(np.ascontiguousarray(rp)).to(dev),
                     torch.from_numpy(np.ascontiguousarray(ci)).to(dev),
                     torch.from_numpy(np.ascontiguousarray(v)).to(dev), n, d)


def rel(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(a - ref) / (den if den > 0 else 1.0))


def u32(t):
    return t.cpu().numpy().view(np.uint32)
