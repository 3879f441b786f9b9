"""Pins of the Algorithm 1 oracle (row extrema of Z = T X, Section 4).

* row_extrema against a hand-worked fixture with ties, signed zeros and
  NaNs (tests/golden/row_extrema.txt), and against numpy's argmax/argmin
  (which also return the first occurrence) on random matrices.
* Separable data (X = U V^T with the rows of V on the simplex): the maximum
  and the minimum of a linear function over the polytope spanned by the
  columns are attained at its vertices, so every extremum that is unique
  names an anchor, whatever the projection -- T X, G~ X or any other.
* With m rows the extraction sees at most 2 m indices; with enough rows all
  anchors are found (the exact-recovery behaviour of Section 6).
"""
import os

import numpy as np

import oracle as O
from paper_1606_05732_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "row_extrema.txt")


def _fixture():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        vals, idx = line.split("|")
        rows.append(([float(t) for t in vals.split()], [int(t) for t in idx.split()]))
    return rows


def test_row_extrema_hand_worked_fixture():
    rows = _fixture()
    assert len(rows) >= 8
    for vals, (emax, emin) in rows:
        imax, imin = O.row_extrema(np.array([vals]))
        assert (int(imax[0]), int(imin[0])) == (emax, emin), vals


def test_row_extrema_matches_numpy_first_occurrence():
    rng = np.random.default_rng(3)
    Z = rng.integers(-3, 4, size=(200, 37)).astype(np.float64)   # many ties
    imax, imin = O.row_extrema(Z)
    assert np.array_equal(imax, np.argmax(Z, axis=1))
    assert np.array_equal(imin, np.argmin(Z, axis=1))


def _unique_extrema(Z):
    s = np.sort(Z, axis=1)
    return (s[:, -1] > s[:, -2]), (s[:, 0] < s[:, 1])


def test_unique_extrema_of_separable_data_are_anchors():
    rng = np.random.default_rng(11)
    for k in (3, 8, 20):
        X, anchors = W.separable_nmf(rng, 300, 200, k)
        for Z in (O.sketch_dense(X, 24, 120, 7 + k), O.gaussian_product_dense(X, 24, 9 + k),
                  rng.standard_normal((24, 300)) @ X):
            imax, imin = O.row_extrema(Z)
            umax, umin = _unique_extrema(Z)
            assert set(imax[umax].tolist()) <= set(anchors.tolist())
            assert set(imin[umin].tolist()) <= set(anchors.tolist())


def test_enough_rows_recover_every_anchor():
    rng = np.random.default_rng(12)
    X, anchors = W.separable_nmf(rng, 400, 150, 6)
    assert O.recovers(*O.countgauss_anchors(X, 64, 320, 5), anchors)
    assert O.recovers(*O.gaussian_anchors(X, 64, 5), anchors)
    # one row can name at most two anchors
    imax, imin = O.countgauss_anchors(X, 1, 5, 5)
    assert not O.recovers(imax, imin, anchors)


def test_block_orthonormal_has_orthonormal_columns():
    for d, L in ((4, 1), (5, 3), (16, 7)):
        rp, ci, v, n = W.block_orthonormal(d, L)
        U = O.csr_to_dense(rp, ci, v, n, d)
        assert np.abs(U.T @ U - np.eye(d)).max() < 1e-15
        assert np.array_equal(np.diff(rp), np.ones(n, dtype=np.int32))
