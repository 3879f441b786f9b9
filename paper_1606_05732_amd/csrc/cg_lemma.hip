// Diagnostics of the paper's Section 7 on the GPU, for an n x d matrix U
// with orthonormal columns (d <= 64), from Y = T U (or G~ U) and optionally
// S U:
//  * max over column pairs i < j of | ||Y (e_i + e_j)||^2 - 2 m |: the
//    statistic with which the lower-bound lemma tells T U from G~ U (a
//    unique collision between two columns' blocks moves one pair's squared
//    norm to about m (2 + (2 / L) sigma_a sigma_b));
//  * with M = (S U)^T (S U) -- the covariance of each row of T U given S --
//    ||I - M||_F^2 (O(d^2 / B) in expectation), the number of nonzero
//    off-diagonal pairs of M (one after a unique cross-block collision),
//    KL(N(0, I) || N(0, M)) = 1/2 tr(M^-1 - I) + 1/2 ln det M (the claim on
//    Gaussian KL divergences) and Pinsker's bound sqrt(m KL / 2) on the
//    total variation of the m rows given S.
// Gram matrices are summed in FP64: per-workgroup partials over row chunks,
// added in a fixed order (bitwise reproducible); M is factored by Cholesky
// in LDS by one workgroup.
#include "cg_internal.hpp"

namespace cg {

namespace {

constexpr int kThreads = 256;
constexpr int kTileRows = 32;

// part[blockIdx.x] (d x d, FP64) = sum over the block's rows r of A[r]^T A[r].
template <typename T>
__global__ __launch_bounds__(kThreads) void gram_partial_kernel(const T* __restrict__ A,
                                                                int64_t rows, int d, int64_t lda,
                                                                double* __restrict__ part) {
  __shared__ double tile[kTileRows][kLemmaMaxD];
  constexpr int kPer = kLemmaMaxD * kLemmaMaxD / kThreads;
  double acc[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) acc[k] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * kLemmaGramRows;
  const int64_t r1 = min(r0 + (int64_t)kLemmaGramRows, rows);
  const int dd = d * d;
  for (int64_t t0 = r0; t0 < r1; t0 += kTileRows) {
    for (int e = threadIdx.x; e < kTileRows * kLemmaMaxD; e += kThreads) {
      const int rr = e / kLemmaMaxD, c = e % kLemmaMaxD;
      const int64_t r = t0 + rr;
      tile[rr][c] = (r < r1 && c < d) ? (double)A[r * lda + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = threadIdx.x + k * kThreads;
      if (e < dd) {
        const int i = e / d, j = e % d;
        double s = acc[k];
        for (int rr = 0; rr < kTileRows; ++rr) s += tile[rr][i] * tile[rr][j];
        acc[k] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int e = threadIdx.x + k * kThreads;
    if (e < dd) part[(int64_t)blockIdx.x * dd + e] = acc[k];
  }
}

__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

__device__ double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < kThreads / 64; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

// One workgroup.  partY: nY partials of Y^T Y; partM: nM partials of
// (S U)^T (S U), or nM = 0.  stats: see cg_lemma_stats.
__global__ __launch_bounds__(kThreads) void lemma_stats_kernel(const double* __restrict__ partY,
                                                               int64_t nY,
                                                               const double* __restrict__ partM,
                                                               int64_t nM, int d, int64_t m,
                                                               double* __restrict__ stats) {
  extern __shared__ double lds[];
  double* GY = lds;                       // d x d
  double* A = GY + kLemmaMaxD * kLemmaMaxD;   // M, then its Cholesky factor
  double* Xi = A + kLemmaMaxD * kLemmaMaxD;   // columns of L^-1
  __shared__ double red[kThreads / 64];
  __shared__ int notpd;
  const int dd = d * d;
  for (int e = threadIdx.x; e < dd; e += kThreads) {
    double s = 0.0;
    for (int64_t w = 0; w < nY; ++w) s += partY[w * dd + e];
    GY[e] = s;
    double t = 0.0;
    for (int64_t w = 0; w < nM; ++w) t += partM[w * dd + e];
    A[e] = t;
  }
  if (threadIdx.x == 0) notpd = 0;
  __syncthreads();
  // pair statistic over i < j
  double dev = 0.0;
  for (int e = threadIdx.x; e < dd; e += kThreads) {
    const int i = e / d, j = e % d;
    if (i < j) dev = fmax(dev, fabs(GY[i * d + i] + GY[j * d + j] + 2.0 * GY[i * d + j] - 2.0 * (double)m));
  }
  dev = block_max(dev, red);
  if (nM == 0) {
    if (threadIdx.x == 0) {
      stats[0] = dev;
      for (int k = 1; k < kLemmaStats; ++k) stats[k] = __longlong_as_double(0x7ff8000000000000ll);
    }
    return;
  }
  double fro = 0.0, offd = 0.0;
  for (int e = threadIdx.x; e < dd; e += kThreads) {
    const int i = e / d, j = e % d;
    const double g = A[e] - (i == j ? 1.0 : 0.0);
    fro += g * g;
    if (i < j && fabs(A[e]) > 1e-9) offd += 1.0;
  }
  fro = block_sum(fro, red);
  offd = block_sum(offd, red);
  // Cholesky A = L L^T in place (lower triangle), right-looking
  for (int k = 0; k < d; ++k) {
    if (threadIdx.x == 0) {
      const double piv = A[k * d + k];
      if (!(piv > 0.0)) notpd = 1;
      A[k * d + k] = piv > 0.0 ? sqrt(piv) : 1.0;
    }
    __syncthreads();
    const double lkk = A[k * d + k];
    for (int i = k + 1 + threadIdx.x; i < d; i += kThreads) A[i * d + k] /= lkk;
    __syncthreads();
    const int rem = d - k - 1;
    for (int e = threadIdx.x; e < rem * rem; e += kThreads) {
      const int i = k + 1 + e / rem, j = k + 1 + e % rem;
      if (j <= i) A[i * d + j] -= A[i * d + k] * A[j * d + k];
    }
    __syncthreads();
  }
  // tr(M^-1) = ||L^-1||_F^2: thread j solves L x = e_j by forward substitution
  double tr = 0.0, ld = 0.0;
  for (int j = threadIdx.x; j < d; j += kThreads) {
    for (int i = 0; i < d; ++i) {
      double s = i == j ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= A[i * d + k] * Xi[k * kLemmaMaxD + j];
      const double x = i < j ? 0.0 : s / A[i * d + i];
      Xi[i * kLemmaMaxD + j] = x;
      tr += x * x;
    }
    ld += 2.0 * log(A[j * d + j]);
  }
  tr = block_sum(tr, red);
  ld = block_sum(ld, red);
  if (threadIdx.x == 0) {
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    const double kl = notpd ? inf : 0.5 * (tr - (double)d) + 0.5 * ld;
    stats[0] = dev;
    stats[1] = fro;
    stats[2] = kl;
    // (KL >= 0; rounding can leave it a hair below zero when M is I)
    stats[3] = notpd ? 1.0 : fmin(1.0, sqrt(fmax((double)m * kl / 2.0, 0.0)));
    stats[4] = offd;
    stats[5] = notpd ? 0.0 : 1.0;
  }
}

}  // namespace

size_t lemma_workspace_bytes(int64_t m, int64_t B, int64_t d, bool with_su) {
  const int64_t parts = (m + kLemmaGramRows - 1) / kLemmaGramRows +
                        (with_su ? (B + kLemmaGramRows - 1) / kLemmaGramRows : 0);
  return align256((size_t)parts * d * d * 8);
}

template <typename T>
hipError_t launch_lemma_stats(const T* Y, const T* SU, int64_t m, int64_t B, int d, double* ws,
                              double* stats, hipStream_t s) {
  const int64_t nY = (m + kLemmaGramRows - 1) / kLemmaGramRows;
  const int64_t nM = SU ? (B + kLemmaGramRows - 1) / kLemmaGramRows : 0;
  gram_partial_kernel<T><<<(unsigned)nY, kThreads, 0, s>>>(Y, m, d, d, ws);
  if (nM) gram_partial_kernel<T><<<(unsigned)nM, kThreads, 0, s>>>(SU, B, d, d, ws + nY * d * d);
  const size_t lds = (size_t)3 * kLemmaMaxD * kLemmaMaxD * 8;
  hipError_t e = hipFuncSetAttribute((const void*)lemma_stats_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  lemma_stats_kernel<<<1, kThreads, lds, s>>>(ws, nY, ws + nY * d * d, nM, d, m, stats);
  return hipGetLastError();
}

template hipError_t launch_lemma_stats<float>(const float*, const float*, int64_t, int64_t, int,
                                              double*, double*, hipStream_t);
template hipError_t launch_lemma_stats<double>(const double*, const double*, int64_t, int64_t, int,
                                               double*, double*, hipStream_t);

}  // namespace cg
