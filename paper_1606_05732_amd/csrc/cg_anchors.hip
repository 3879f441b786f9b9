// Step 3 of Algorithm 1 (CountGauss NMF, Section 4): for every row of
// Z = T X, the column where it is largest (I_max) and where it is smallest
// (I_min).  The paper leaves ties open; the lowest column index wins here.
// NaN entries never win, and a row without a number gives -1.
//
// One wavefront per row: lane l scans columns l, l + 64, ... in increasing
// order (so its own ties keep the lowest column), then a butterfly over the
// 64 lanes in which a candidate replaces another when it is larger (for
// I_max) or on an equal value with a lower column.
#include "cg_internal.hpp"

namespace cg {

namespace {

constexpr int kRowsPerBlock = 4;

template <typename T>
__device__ __forceinline__ void take_if_better(T v, int j, bool larger, T& best, int& at) {
  if (j >= 0 && (at < 0 || (larger ? v > best : v < best) || (v == best && j < at))) {
    best = v;
    at = j;
  }
}

template <typename T>
__global__ __launch_bounds__(64 * kRowsPerBlock) void row_extrema_kernel(
    const T* __restrict__ Z, int64_t m, int64_t d, int64_t ldz, int32_t* __restrict__ imax,
    int32_t* __restrict__ imin) {
  const int64_t row = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;   // whole wavefronts leave together
  const T* __restrict__ z = Z + row * ldz;
  T hi = T(0), lo = T(0);
  int ih = -1, il = -1;
  for (int64_t j = lane; j < d; j += 64) {
    const T v = z[j];
    if (v != v) continue;
    if (ih < 0 || v > hi) {
      hi = v;
      ih = (int)j;
    }
    if (il < 0 || v < lo) {
      lo = v;
      il = (int)j;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const T ohi = __shfl_xor(hi, off, 64), olo = __shfl_xor(lo, off, 64);
    const int oih = __shfl_xor(ih, off, 64), oil = __shfl_xor(il, off, 64);
    take_if_better(ohi, oih, true, hi, ih);
    take_if_better(olo, oil, false, lo, il);
  }
  if (lane == 0) {
    imax[row] = ih;
    imin[row] = il;
  }
}

}  // namespace

template <typename T>
hipError_t launch_row_extrema(const T* Z, int64_t m, int64_t d, int64_t ldz, int32_t* imax,
                              int32_t* imin, hipStream_t s) {
  const int64_t blocks = (m + kRowsPerBlock - 1) / kRowsPerBlock;
  row_extrema_kernel<T><<<(unsigned)blocks, 64 * kRowsPerBlock, 0, s>>>(Z, m, d, ldz, imax, imin);
  return hipGetLastError();
}

template hipError_t launch_row_extrema<float>(const float*, int64_t, int64_t, int64_t, int32_t*,
                                              int32_t*, hipStream_t);
template hipError_t launch_row_extrema<double>(const double*, int64_t, int64_t, int64_t, int32_t*,
                                               int32_t*, hipStream_t);

}  // namespace cg
