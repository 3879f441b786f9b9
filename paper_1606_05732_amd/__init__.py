"""MI355X (gfx950) CountGauss transform T.X = G.(S.X).

The transform of Kapralov, Potluru and Woodruff ("How to Fake Multiply by a
Gaussian Matrix"): a seeded CountSketch S followed by an m x B Gaussian G,
computed by hand-written HIP kernels in libcountgauss.so (C ABI in
include/countgauss.h).  This package is a thin binding: torch provides
device memory and streams.
"""
from .api import (anchors, BatchedSketch, CsrMatrix, CountGaussCsrFn, CountGaussFn, countgauss,  # noqa: F401
                  debug_gaussian, debug_hash, debug_normals, debug_philox, gaussian, get_tuning,
                  lemma_stats, LEMMA_STATS,
                  row_extrema, set_tuning, sketch,
                  sketch_adjoint, sketch_adjoint_csr, sketch_batched, sketch_csr_noalloc,
                  SketchPlan)
from ._lib import CountGaussError, LIB_PATH  # noqa: F401
