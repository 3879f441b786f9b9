"""Plain CPU FP64 oracle for the CountGauss transform T.X = G.(S.X).

TEST INFRASTRUCTURE ONLY.  This package is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``.
The product path (the HIP library and its Python binding) never imports,
calls, links or executes anything here, and this package imports nothing
from the product path.  The two share no code: the random-number and hash
specification is written out independently on each side.

Every function is written for clarity, not speed: FP64 throughout, whole
matrices materialised where that makes the definition visible.

Parity status per function (what pins it against something other than
itself is listed in tests/test_oracle_*.py):
  philox4x32_10      pinned: published known-answer vectors (Salmon et al.)
  hash_rows          pinned: structure of S (Section 1.1), uniformity and
                     collision statistics, Lemma lb worked identity (Sec. 7)
  gaussian_block     pinned: Box-Muller radius/angle identities, KS vs the
                     normal CDF, bound, nesting
  sketch_*           pinned: brute-force dense product, injective special
                     case, closed-form E||M-C||_F^2, covariance over seeds,
                     conditional whitening KS (Theorem 1 setting)
  sx_csr, csr_to_dense, sketch_csr
                     pinned also against scipy.sparse's own CSR expansion
                     and sparse product S @ X
  sketch_touched     pinned: equals the full product (brute force, scatter)
  adjoint_*          pinned: adjoint identity and central differences;
                     adjoint_csr also against scipy.sparse S^T Z
  quantise_bf16/fp8  pinned: torch CPU dtype conversions (library routines)
  emulate_reduced    pinned: a hand-worked BF16 / E4M3 case (ties to even,
                     the 448 edge, subnormals, 128-row blocks, the G scale),
                     each expected value derived from the format definitions
  gaussian_product_* pinned: 2-stability (entries N(0, ||x_j||^2), squared
                     norms chi-square m), row covariance X^T X, scipy.sparse
                     product with the explicit G~, chunk / offset invariance
  row_extrema        pinned: hand-worked fixture with ties and NaNs
                     (tests/golden/row_extrema.txt), numpy argmax/argmin
  *_anchors          pinned: on separable data every unique extremum is an
                     anchor (extreme points of the polytope, Section 4)
  lowerbound.*       pinned: KL against quadrature and Monte Carlo (scipy
                     densities), Pinsker against exact TV, hand-worked pair
                     statistic, chi-square law under G~, the lemma's
                     unique-collision identity, E||I-M||_F^2 by Monte Carlo
"""
from .countgauss import *  # noqa: F401,F403
from .anchors import *  # noqa: F401,F403
from . import lowerbound  # noqa: F401
