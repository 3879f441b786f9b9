"""FP64 reference for the CountGauss transform (test infrastructure only).

The method (Section 1.1 "A New Randomized Transform" and Section 2 of the
paper): for an n x d matrix X, T.X = G.(S.X) where

* S (B x n) is a CountSketch: column r has a single nonzero, at row h(r),
  equal to sigma(r) in {+1,-1}; all choices independent (Section 1.1, and the
  restatement at the start of the proof of Theorem 1, Section 7, which also
  names the position h(k) and value sigma(k) in the lower-bound lemma);
* G (m x B) has i.i.d. unit-variance Gaussian entries (Theorem 1);
* S.X costs O(nnz(X)); G.(S.X) is a dense m x B by B x d product (Sec. 1.1).

The paper leaves the random source unspecified ("uniformly random", "+1 or -1
with probability 1/2", "i.i.d. Gaussians").  The reading used here, and on
the GPU, is a counter-based generator so that S and G are pure functions of
(seed, index):

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11), key = (lo32(seed), hi32(seed)).
* Hash of global row r (counter tag 0): q = r >> 2, counter
  (lo32(q), hi32(q), 0, 0), word w = out[r & 3];
  sigma(r) = +1 if bit 31 of w is clear else -1;
  h(r) = ((w & 0x7fffffff) * B) >> 31  (multiply-shift range reduction).
* Gaussian G[i, b] (counter tag 1): counter (b, i >> 2, 1, 0), words
  w0..w3, u_k = ((w_k >> 9) + 1/2) * 2^-23 (exact in FP32 and FP64),
  Box-Muller (Box & Muller 1958): rho0 = sqrt(-2 ln u0), rho1 = sqrt(-2 ln u2),
  z = (rho0 cos 2 pi u1, rho0 sin 2 pi u1, rho1 cos 2 pi u3, rho1 sin 2 pi u3),
  G[i, b] = z[i & 3].
* Dense comparison Gaussian G~[i, r] (m x n, tag 2, oracle only): counter
  (lo32(r), i >> 2, 2, hi32(r)), same Box-Muller map.

No 1/sqrt(m) scaling: Theorem 1 uses unit-variance Gaussians.
"""
import math

import numpy as np

__all__ = [
    "PHILOX_M0", "PHILOX_M1", "PHILOX_W0", "PHILOX_W1",
    "philox4x32_10", "seed_key", "hash_words", "hash_rows",
    "uniforms_from_words", "box_muller", "gaussian_block", "gaussian_matrix",
    "dense_gaussian_block", "dense_gaussian_columns", "gaussian_product_dense",
    "gaussian_product_csr", "countsketch_matrix", "row_of_nonzero",
    "sx_dense", "sx_csr", "sketch_dense", "sketch_csr", "sketch_touched", "csr_to_dense",
    "adjoint_dense", "adjoint_csr", "central_fd", "round_to_format",
    "quantise_bf16", "quantise_fp8_e4m3", "fp8_block_exponent",
    "emulate_reduced", "rel_frobenius", "GAUSS_ABS_MAX",
]

# Philox4x32 constants (Salmon et al. 2011): round multipliers and the
# Weyl increments added to the key between rounds.
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)

# Largest |G| the Box-Muller map above can produce: u >= 2^-24.
GAUSS_ABS_MAX = math.sqrt(-2.0 * math.log(2.0 ** -24))


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.

    ctr: uint32 array (..., 4); key: uint32 array (..., 2), broadcastable.
    Each round multiplies c0 and c2 by the two constants into 64-bit
    products, then outputs (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key
    is advanced by the Weyl increments before every round but the first.
    Returns uint32 (..., 4).
    """
    ctr = np.asarray(ctr, dtype=np.uint32)
    key = np.asarray(key, dtype=np.uint32)
    c0, c1, c2, c3 = (ctr[..., j].astype(np.uint64) for j in range(4))
    k0 = key[..., 0].astype(np.uint64)
    k1 = key[..., 1].astype(np.uint64)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK32
        p0 = np.uint64(PHILOX_M0) * c0          # < 2^64, exact in uint64
        p1 = np.uint64(PHILOX_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def seed_key(seed):
    """Philox key (lo32, hi32) of a 64-bit seed."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)


def hash_words(seed, rows):
    """Philox word w(r) of each global row index r (tag 0 counters)."""
    rows = np.asarray(rows, dtype=np.uint64)
    q = rows >> np.uint64(2)
    ctr = np.zeros(rows.shape + (4,), dtype=np.uint32)
    ctr[..., 0] = (q & _MASK32).astype(np.uint32)
    ctr[..., 1] = (q >> np.uint64(32)).astype(np.uint32)
    out = philox4x32_10(ctr, seed_key(seed))
    lane = (rows & np.uint64(3)).astype(np.int64)
    return np.take_along_axis(out, lane[..., None], axis=-1)[..., 0]


def hash_rows(seed, B, rows):
    """Bucket h(r) in [0, B) and sign sigma(r) in {+1, -1} of each row r.

    This is the CountSketch column r of S (Section 1.1): its one nonzero
    sits at row h(r) with value sigma(r).
    """
    w = hash_words(seed, rows).astype(np.uint64)
    sigma = np.where((w >> np.uint64(31)) == 0, 1.0, -1.0)
    h = ((w & np.uint64(0x7FFFFFFF)) * np.uint64(B)) >> np.uint64(31)
    return h.astype(np.int64), sigma


def uniforms_from_words(w):
    """u = ((w >> 9) + 1/2) * 2^-23, strictly inside (0, 1)."""
    w = np.asarray(w, dtype=np.uint32)
    return ((w >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(words):
    """Four normals from four Philox words (last axis), FP64."""
    u = uniforms_from_words(words)
    rho0 = np.sqrt(-2.0 * np.log(u[..., 0]))
    rho1 = np.sqrt(-2.0 * np.log(u[..., 2]))
    t0 = 2.0 * np.pi * u[..., 1]
    t1 = 2.0 * np.pi * u[..., 3]
    return np.stack([rho0 * np.cos(t0), rho0 * np.sin(t0),
                     rho1 * np.cos(t1), rho1 * np.sin(t1)], axis=-1)


def gaussian_block(seed, m, b0, nb):
    """Columns [b0, b0+nb) of the m x B Gaussian G (tag 1), FP64 (m, nb)."""
    nq = (m + 3) // 4
    b = np.arange(b0, b0 + nb, dtype=np.uint64)
    q = np.arange(nq, dtype=np.uint64)
    ctr = np.zeros((nq, nb, 4), dtype=np.uint32)
    ctr[..., 0] = b[None, :].astype(np.uint32)
    ctr[..., 1] = q[:, None].astype(np.uint32)
    ctr[..., 2] = 1
    z = box_muller(philox4x32_10(ctr, seed_key(seed)))     # (nq, nb, 4)
    G = np.transpose(z, (0, 2, 1)).reshape(nq * 4, nb)      # row 4q+t
    return G[:m]


def gaussian_matrix(seed, m, B):
    """The whole m x B Gaussian G, FP64."""
    return gaussian_block(seed, m, 0, B)


def dense_gaussian_block(seed, m, r0, nr, q0=0):
    """Columns [r0, r0+nr) of the m x n dense Gaussian G~ (tag 2), FP64;
    rows 4 q0 .. m-1 only when q0 > 0."""
    nq = (m + 3) // 4
    r = np.arange(r0, r0 + nr, dtype=np.uint64)
    q = np.arange(q0, nq, dtype=np.uint64)
    nq -= q0
    ctr = np.zeros((nq, nr, 4), dtype=np.uint32)
    ctr[..., 0] = (r & _MASK32).astype(np.uint32)[None, :]
    ctr[..., 1] = q[:, None].astype(np.uint32)
    ctr[..., 2] = 2
    ctr[..., 3] = (r >> np.uint64(32)).astype(np.uint32)[None, :]
    z = box_muller(philox4x32_10(ctr, seed_key(seed)))
    return np.transpose(z, (0, 2, 1)).reshape(nq * 4, nr)[:m - 4 * q0]


def dense_gaussian_columns(seed, m, rows):
    """Columns `rows` (global row indices of X, any order) of the m x n
    dense Gaussian G~ (tag 2), FP64 (m, len(rows))."""
    nq = (m + 3) // 4
    r = np.asarray(rows, dtype=np.uint64)
    q = np.arange(nq, dtype=np.uint64)
    ctr = np.zeros((nq, len(r), 4), dtype=np.uint32)
    ctr[..., 0] = (r & _MASK32).astype(np.uint32)[None, :]
    ctr[..., 1] = q[:, None].astype(np.uint32)
    ctr[..., 2] = 2
    ctr[..., 3] = (r >> np.uint64(32)).astype(np.uint32)[None, :]
    z = box_muller(philox4x32_10(ctr, seed_key(seed)))
    return np.transpose(z, (0, 2, 1)).reshape(nq * 4, len(r))[:m]


def gaussian_product_dense(X, m, seed, row_offset=0, chunk=1 << 15):
    """G~ X (m x d, FP64): the dense Gaussian projection that T X stands in
    for (Section 1.1, "Our Results": O(nnz(X) m) time; Theorem 1 compares the
    distributions of G S U and G~ U).  Row chunks of X times the matching
    columns of G~."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    Y = np.zeros((m, d))
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        Y += dense_gaussian_block(seed, m, row_offset + r0, r1 - r0) @ X[r0:r1]
    return Y


def gaussian_product_csr(row_ptr, col_idx, vals, n, d, m, seed, row_offset=0, chunk=1 << 15):
    """G~ X for CSR X (m x d, FP64): only the columns of G~ of nonempty rows
    contribute."""
    row = row_of_nonzero(row_ptr)
    col = np.asarray(col_idx, np.int64)
    v = np.asarray(vals, np.float64)
    rows = np.unique(row)
    Y = np.zeros((m, d))
    for k0 in range(0, len(rows), chunk):
        sel = rows[k0:k0 + chunk]
        Xs = np.zeros((len(sel), d))
        mask = (row >= sel[0]) & (row <= sel[-1])
        np.add.at(Xs, (np.searchsorted(sel, row[mask]), col[mask]), v[mask])
        Y += dense_gaussian_columns(seed, m, sel.astype(np.uint64) + np.uint64(row_offset)) @ Xs
    return Y


def countsketch_matrix(seed, B, n, row_offset=0):
    """S as an explicit dense B x n FP64 matrix (brute force, tiny n*B)."""
    h, sigma = hash_rows(seed, B, np.arange(n, dtype=np.uint64) + np.uint64(row_offset))
    S = np.zeros((B, n))
    S[h, np.arange(n)] = sigma
    return S


def row_of_nonzero(row_ptr):
    """Local row index of every stored entry of a CSR matrix."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    return np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))


def csr_to_dense(row_ptr, col_idx, vals, n, d):
    X = np.zeros((n, d))
    np.add.at(X, (row_of_nonzero(row_ptr), np.asarray(col_idx, np.int64)),
              np.asarray(vals, np.float64))
    return X


def sx_dense(X, seed, B, row_offset=0, chunk=1 << 20):
    """S.X for dense X: (SX)[b, :] = sum over rows r with h(r) = b of
    sigma(r) X[r, :] (the per-bucket sum written out in the proof of the
    lower-bound lemma, Section 7).  FP64 scatter-add, row chunks."""
    X = np.asarray(X)
    n, d = X.shape
    SX = np.zeros((B, d))
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        rows = np.arange(r0, r1, dtype=np.uint64) + np.uint64(row_offset)
        h, sigma = hash_rows(seed, B, rows)
        np.add.at(SX, h, sigma[:, None] * X[r0:r1].astype(np.float64))
    return SX


def sx_csr(row_ptr, col_idx, vals, n, d, seed, B, row_offset=0):
    """S.X for CSR X: every stored entry (r, c, v) adds sigma(r) v to
    SX[h(r), c].  O(nnz) as stated in Section 1.1.  FP64 (bincount)."""
    row = row_of_nonzero(row_ptr)
    h, sigma = hash_rows(seed, B, np.arange(n, dtype=np.uint64) + np.uint64(row_offset))
    flat = h[row] * d + np.asarray(col_idx, np.int64)
    w = sigma[row] * np.asarray(vals, np.float64)
    return np.bincount(flat, weights=w, minlength=B * d).reshape(B, d)


def _sketch_from_sx(SX, m, seed):
    B = SX.shape[0]
    return gaussian_matrix(seed, m, B) @ SX


def sketch_dense(X, m, B, seed, row_offset=0, method="scatter"):
    """Y = G.S.X (m x d, FP64) for dense X.

    method="brute":   explicit dense S and G, then G @ (S @ X);
    method="scatter": S.X by scatter-add, then G @ SX;
    method="outer":   T = G.S column by column (T[:, r] = sigma(r) G[:, h(r)])
                      and Y = T @ X in row chunks.
    """
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    if method == "brute":
        S = countsketch_matrix(seed, B, n, row_offset)
        return gaussian_matrix(seed, m, B) @ (S @ X)
    if method == "scatter":
        return _sketch_from_sx(sx_dense(X, seed, B, row_offset), m, seed)
    if method == "outer":
        G = gaussian_matrix(seed, m, B)
        Y = np.zeros((m, d))
        for r0 in range(0, n, 1 << 16):
            r1 = min(n, r0 + (1 << 16))
            rows = np.arange(r0, r1, dtype=np.uint64) + np.uint64(row_offset)
            h, sigma = hash_rows(seed, B, rows)
            Y += (G[:, h] * sigma[None, :]) @ X[r0:r1]
        return Y
    raise ValueError(method)


def sketch_touched(X, m, B, seed, row_offset=0):
    """Y = sum over the rows r of sigma(r) G[:, h(r)] X[r, :] (the streamed
    formulation of G.S.X, Section 1.1: S puts row r into column h(r) of
    S.X with sign sigma(r)), with only the columns of G that some row
    hashes to generated: for B far larger than n.  FP64."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    h, sigma = hash_rows(seed, B, np.arange(n, dtype=np.uint64) + np.uint64(row_offset))
    Y = np.zeros((m, d))
    for b in np.unique(h):
        rows = h == b
        Y += gaussian_block(seed, m, int(b), 1) @ (sigma[rows] @ X[rows])[None, :]
    return Y


def sketch_csr(row_ptr, col_idx, vals, n, d, m, B, seed, row_offset=0):
    """Y = G.S.X (m x d, FP64) for CSR X, via the O(nnz) scatter."""
    return _sketch_from_sx(sx_csr(row_ptr, col_idx, vals, n, d, seed, B, row_offset),
                           m, seed)


def adjoint_dense(dY, n, d, m, B, seed, row_offset=0):
    """T^T dY = S^T (G^T dY): Z = G^T dY (B x d), then row r of the result
    is sigma(r) Z[h(r), :].  T = G.S is linear (Section 1.1), so this is the
    gradient of <dY, T X> with respect to X."""
    dY = np.asarray(dY, dtype=np.float64)
    Z = gaussian_matrix(seed, m, B).T @ dY
    h, sigma = hash_rows(seed, B, np.arange(n, dtype=np.uint64) + np.uint64(row_offset))
    return sigma[:, None] * Z[h]


def adjoint_csr(row_ptr, col_idx, dY, n, d, m, B, seed, row_offset=0):
    """Gradient of <dY, T X> with respect to the stored values of CSR X."""
    dY = np.asarray(dY, dtype=np.float64)
    Z = gaussian_matrix(seed, m, B).T @ dY
    row = row_of_nonzero(row_ptr)
    h, sigma = hash_rows(seed, B, np.arange(n, dtype=np.uint64) + np.uint64(row_offset))
    return sigma[row] * Z[h[row], np.asarray(col_idx, np.int64)]


def central_fd(f, X, entries, step):
    """Central differences (f(X + step e) - f(X - step e)) / (2 step) of a
    scalar function f at the listed (row, col) entries of X."""
    X = np.array(X, dtype=np.float64, copy=True)
    out = np.empty(len(entries))
    for k, (r, c) in enumerate(entries):
        x0 = X[r, c]
        X[r, c] = x0 + step
        fp = f(X)
        X[r, c] = x0 - step
        fm = f(X)
        X[r, c] = x0
        out[k] = (fp - fm) / (2.0 * step)
    return out


def round_to_format(x, mant_bits, emin, max_finite):
    """Round FP64 values to a binary floating-point format with `mant_bits`
    stored significand bits, minimum normal exponent `emin` (subnormals
    below it) and largest finite value `max_finite`; round to nearest, ties
    to even; saturate at max_finite."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    with np.errstate(divide="ignore"):
        _, e2 = np.frexp(a)                    # a = f 2^e2, f in [0.5, 1)
    e = np.maximum(e2 - 1, emin)               # floor(log2 a), clamped
    quantum = np.ldexp(1.0, e - mant_bits)
    q = np.rint(a / quantum) * quantum         # np.rint: ties to even
    q = np.minimum(q, max_finite)
    return np.where(a == 0, 0.0, np.copysign(q, x))


def quantise_bf16(x):
    """bfloat16: 7 stored bits, emin -126."""
    return round_to_format(x, 7, -126, (2.0 - 2.0 ** -7) * 2.0 ** 127)


def quantise_fp8_e4m3(x):
    """OCP FP8 E4M3 ("fn"): 3 stored bits, bias 7, emin -6, max 448."""
    return round_to_format(x, 3, -6, 448.0)


def fp8_block_exponent(amax):
    """Smallest integer e with amax <= 448 * 2^e (so the block scaled by
    2^-e fits E4M3), decided exactly from amax's binary exponent;
    0 for amax == 0."""
    amax = float(amax)
    if amax == 0.0:
        return 0
    f, E = math.frexp(amax)                    # amax = f 2^E, f in [0.5, 1)
    return E - 9 if f <= 0.875 else E - 8      # 448 = 0.875 * 2^9


def emulate_reduced(G, SX, precision, kblock=128):
    """Y ~= G.SX with both operands rounded to `precision` ("bf16" or
    "fp8") per 128-wide block along B; FP64 accumulation.  For fp8 each SX
    block gets the power-of-two scale 2^fp8_block_exponent(amax) and G the
    constant 2^-6 (|G| <= 5.77 < 7).  Inputs are first rounded to FP32, as
    the GPU holds them.  The paper fixes no precision: this is the reading
    the reduced-precision contraction follows."""
    G32 = np.asarray(G, np.float32).astype(np.float64)
    S32 = np.asarray(SX, np.float32).astype(np.float64)
    m, B = G32.shape
    Y = np.zeros((m, S32.shape[1]))
    for k0 in range(0, B, kblock):
        g = G32[:, k0:k0 + kblock]
        s = S32[k0:k0 + kblock]
        if precision == "bf16":
            Y += quantise_bf16(g) @ quantise_bf16(s)
        elif precision == "fp8":
            sg = 2.0 ** -6
            sx = 2.0 ** fp8_block_exponent(np.max(np.abs(s)) if s.size else 0.0)
            Y += (quantise_fp8_e4m3(g / sg) @ quantise_fp8_e4m3(s / sx)) * (sg * sx)
        else:
            raise ValueError(precision)
    return Y


def rel_frobenius(a, ref):
    """||a - ref||_F / ||ref||_F."""
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(a - ref) / (den if den > 0 else 1.0))
