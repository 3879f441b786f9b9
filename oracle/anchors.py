"""Algorithm 1 of the paper (CountGauss NMF, Section 4) and its Gaussian
baseline, in FP64 (test infrastructure only, like the rest of oracle/).

The separable NMF setting (Section 2): the columns of a nonnegative X lie in
the cone of k of its columns, the anchors.  Algorithm 1 forms Z = T X with
T = G S and returns, for every row of Z, the column where it is largest
(I_max) and where it is smallest (I_min).  A linear function over a polytope
is extremal at an extreme point, so every index returned names an anchor
when the extremum is unique (Section 4).  The baseline it is compared with
(Damle and Sun; "GP" in Section 6) does the same with a dense Gaussian
G~ X.  Ties, on which the paper is silent, go to the lowest column index.

Here X is features x points, as in Section 4: T sketches the feature rows
and the anchors are columns.
"""
import numpy as np

from .countgauss import gaussian_product_dense, sketch_dense

__all__ = ["row_extrema", "countgauss_anchors", "gaussian_anchors", "recovers"]


def row_extrema(Z):
    """For each row i of Z: the lowest column index where Z[i] is largest,
    and the lowest where it is smallest (step 3 of Algorithm 1).  NaN
    entries never win; a row of NaNs gives -1.  Written as a plain scan."""
    Z = np.asarray(Z, dtype=np.float64)
    m, d = Z.shape
    imax = np.full(m, -1, dtype=np.int64)
    imin = np.full(m, -1, dtype=np.int64)
    for i in range(m):
        best_hi = best_lo = None
        for j in range(d):
            z = Z[i, j]
            if z != z:
                continue
            if best_hi is None or z > best_hi:
                best_hi, imax[i] = z, j
            if best_lo is None or z < best_lo:
                best_lo, imin[i] = z, j
    return imax, imin


def countgauss_anchors(X, m, B, seed):
    """Algorithm 1: Z = G S X (the oracle's T X), then its row extrema."""
    return row_extrema(sketch_dense(X, m, B, seed))


def gaussian_anchors(X, m, seed):
    """The Gaussian baseline: Z = G~ X, then its row extrema."""
    return row_extrema(gaussian_product_dense(X, m, seed))


def recovers(imax, imin, anchors):
    """Whether I_max and I_min together contain every anchor."""
    found = set(np.asarray(imax).tolist()) | set(np.asarray(imin).tolist())
    return set(np.asarray(anchors).tolist()) <= found
