"""Seeded synthetic inputs of the paper's shape (n >> d, sparse nonnegative
or dense Gaussian X).

This module holds data generators only -- none of the transform's
arithmetic -- so that both the HIP path and the CPU oracle can be fed the
same matrices.  It depends on numpy alone.

Workloads (data seed 1000 + k for workload k, sketch seed 2000 + k):

  k=1  CSR   n=10^6,  d=10, density 1%,  values N(0,1) (float64); m=20,  B=2000
  k=2  CSR   n=2^24,  d=32, density 5%,  values |N(0,1)| (float32); m=64, B=65536
  k=2d dense n=2^22,  d=32, N(0,1) float32;                         m=64, B=65536
  k=3  dense n=2^22,  d=64, N(0,1) float32, rows r % 64 == 0 scaled x100;
             m=64, B=262144 (precision ladder)
  k=4  dense n=2^22,  d=64, N(0,1) float32 plus w, w*, y = X w* + 0.1 N(0,1)
             and an upstream dY ~ N(0,1) (m x d); m=128, B=2^19
  k=5  512 CSR instances, n log-uniform in [1e4, 1e6], d in {8,16,32,64},
       density log-uniform in [0.1%, 10%], values |N(0,1)| float32; m=32,
       B = min(32 d^2, n // 4), sketch seed 5_000_000 + i.

CSR structure: every entry is nonzero independently with probability p,
generated as the positions of a Bernoulli(p) process over the row-major
index space (geometric gaps), so columns come out sorted within each row.
"""
from dataclasses import dataclass, field

import numpy as np


def csr_bernoulli(rng, n, d, p, dtype=np.float32, absolute=False):
    """CSR (row_ptr int32[n+1], col_idx int32[nnz], vals dtype[nnz]) with
    i.i.d. Bernoulli(p) sparsity over an n x d matrix, values N(0,1) (or
    |N(0,1)| when absolute)."""
    total = n * d
    if p <= 0.0:
        pos = np.zeros(0, np.int64)
    elif p >= 1.0:
        pos = np.arange(total, dtype=np.int64)
    else:
        pieces = []
        last = -1
        while True:
            want = max(1024, int((total - last) * p * 1.02) + 64)
            gaps = rng.geometric(p, size=want).astype(np.int64)
            cum = last + np.cumsum(gaps)
            keep = cum[cum < total]
            pieces.append(keep)
            if len(keep) < len(cum):
                break
            last = int(cum[-1])
        pos = np.concatenate(pieces) if pieces else np.zeros(0, np.int64)
    rows = pos // d
    cols = (pos - rows * d).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    vals = rng.standard_normal(len(pos), dtype=np.float64)
    if absolute:
        vals = np.abs(vals)
    return row_ptr.astype(np.int32), cols, vals.astype(dtype)


def dense_normal(rng, n, d, dtype=np.float32, chunk=1 << 20):
    X = np.empty((n, d), dtype=dtype)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        X[r0:r1] = rng.standard_normal((r1 - r0, d), dtype=np.float32).astype(dtype)
    return X


@dataclass
class CsrInput:
    row_ptr: np.ndarray
    col_idx: np.ndarray
    vals: np.ndarray
    n: int
    d: int

    @property
    def nnz(self):
        return int(self.row_ptr[-1])


@dataclass
class Workload:
    name: str
    m: int
    B: int
    seed: int
    csr: CsrInput = None
    dense: np.ndarray = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.csr.n if self.csr is not None else self.dense.shape[0]

    @property
    def d(self):
        return self.csr.d if self.csr is not None else self.dense.shape[1]

    @property
    def nnz(self):
        return self.csr.nnz if self.csr is not None else self.dense.size


def workload1(n=10 ** 6, d=10, p=0.01):
    rng = np.random.Generator(np.random.PCG64(1001))
    rp, ci, v = csr_bernoulli(rng, n, d, p, dtype=np.float64)
    return Workload("csr_n1e6_d10_p0.01_m20_B2000", 20, 2000, 2001,
                    csr=CsrInput(rp, ci, v, n, d))


def workload2(n=1 << 24, d=32, p=0.05, m=64, B=65536):
    rng = np.random.Generator(np.random.PCG64(1002))
    rp, ci, v = csr_bernoulli(rng, n, d, p, dtype=np.float32, absolute=True)
    return Workload(f"csr_n{n}_d{d}_p{p}_m{m}_B{B}", m, B, 2002,
                    csr=CsrInput(rp, ci, v, n, d))


def workload2_dense(n=1 << 22, d=32, m=64, B=65536):
    rng = np.random.Generator(np.random.PCG64(10021))
    return Workload(f"dense_n{n}_d{d}_m{m}_B{B}", m, B, 2002,
                    dense=dense_normal(rng, n, d))


def workload3(n=1 << 22, d=64, m=64, B=262144, spike_every=64, spike=100.0):
    rng = np.random.Generator(np.random.PCG64(1003))
    X = dense_normal(rng, n, d)
    X[::spike_every] *= np.float32(spike)
    return Workload(f"dense_spiky_n{n}_d{d}_m{m}_B{B}", m, B, 2003, dense=X)


def workload4(n=1 << 22, d=64, m=128, B=1 << 19):
    rng = np.random.Generator(np.random.PCG64(1004))
    X = dense_normal(rng, n, d)
    w = rng.standard_normal(d)
    w_star = rng.standard_normal(d)
    y = X.astype(np.float64) @ w_star + 0.1 * rng.standard_normal(n)
    dY = rng.standard_normal((m, d))
    return Workload(f"dense_grad_n{n}_d{d}_m{m}_B{B}", m, B, 2004, dense=X,
                    extra={"w": w, "w_star": w_star, "y": y, "dY": dY})


def workload5_specs(count=512, m=32, seed=1005):
    """Shapes of the batched workload: list of (n, d, p, B, sketch_seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for i in range(count):
        n = int(round(10.0 ** rng.uniform(4.0, 6.0)))
        d = int(rng.choice([8, 16, 32, 64]))
        p = float(10.0 ** rng.uniform(-3.0, -1.0))
        B = int(min(32 * d * d, n // 4))
        specs.append((n, d, p, B, 5_000_000 + i))
    return specs


def workload5(count=512, m=32, seed=1005, scale=1.0):
    """The batched instances; `scale` < 1 shrinks every n (test sizes)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    out = []
    for (n, d, p, B, s) in workload5_specs(count, m, seed):
        n = max(16, int(n * scale))
        B = int(min(32 * d * d, max(1, n // 4)))
        rp, ci, v = csr_bernoulli(rng, n, d, p, dtype=np.float32, absolute=True)
        out.append(Workload(f"batched_{len(out)}", m, B, s, csr=CsrInput(rp, ci, v, n, d)))
    return out


def separable_nmf(rng, features, points, k, dtype=np.float64):
    """A k-separable nonnegative matrix (the exact-recovery experiment of the
    paper's Section 6): X = U V^T, features x points, with U (features x k)
    i.i.d. uniform on [0, 1] and V (points x k) holding the identity in its
    first k rows and i.i.d. uniform [0, 1] entries below, every row of V
    scaled to unit l1 norm, so that every column of X is a convex
    combination of its first k columns (the anchors).  Returns (X, anchors)."""
    U = rng.uniform(0.0, 1.0, size=(features, k))
    V = np.empty((points, k))
    V[:k] = np.eye(k)
    V[k:] = rng.uniform(0.0, 1.0, size=(points - k, k))
    V /= V.sum(axis=1, keepdims=True)
    return (U @ V.T).astype(dtype), np.arange(k)


def block_orthonormal(d, L, dtype=np.float64):
    """The matrix U of the lower-bound lemma (Section 7) as CSR: n = L d rows,
    d columns, column i holding the value 1/sqrt(L) in rows L i .. L i + L - 1
    (disjoint blocks, so the columns are orthonormal).  Every row has exactly
    one stored entry.  Returns (row_ptr, col_idx, vals, n)."""
    n = L * d
    row_ptr = np.arange(n + 1, dtype=np.int32)
    col_idx = (np.arange(n) // L).astype(np.int32)
    vals = np.full(n, 1.0 / np.sqrt(L), dtype=dtype)
    return row_ptr, col_idx, vals, n
