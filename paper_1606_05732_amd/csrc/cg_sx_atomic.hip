// S X by device-scope atomic adds (Section 1.1: S X in O(nnz(X))).
//
// Every stored entry (r, c, v) of X adds sigma(r) v to SX[h(r)][c].  One
// wavefront owns a chunk of 256 consecutive rows: each lane hashes four
// rows with a single Philox call (the four output words of one counter
// serve rows 4q..4q+3) and parks the packed (bucket, sign) words in LDS;
// the chunk's entries are then streamed with fully coalesced loads and
// each lane issues one no-return FP32/FP64 atomic.  Consecutive lanes of
// one row hit the same S X row, so their atomics share a cache line.
#include "cg_internal.hpp"
#include "cg_rng.hpp"

namespace cg {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// Packed hashes of the wave's rows [r0, r0 + nr) into sh[0 .. nr).
__device__ __forceinline__ void hash_rows_to_lds(uint32_t* sh, uint64_t g0, int nr, uint32_t B,
                                                 Key key, int lane) {
  uint32_t hv[4];
  hash4(g0 + 4 * (uint64_t)lane, B, key.k0, key.k1, hv);
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (4 * lane + t < nr) sh[4 * lane + t] = hv[t];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void fill_zero_kernel(T* __restrict__ p, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = T(0);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void sx_csr_atomic_kernel(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const T* __restrict__ vals, int64_t n, int32_t nnz, int d, uint32_t B, Key key,
    uint64_t row_offset, T* __restrict__ SX) {
  __shared__ uint32_t s_hash[kWaves][kRowsPerWave];
  __shared__ int32_t s_ptr[kWaves][kRowsPerWave + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * kWaves + wave) * kRowsPerWave;
  const int nr = r0 < n ? (int)min((int64_t)kRowsPerWave, n - r0) : 0;
  uint32_t* sh = s_hash[wave];
  int32_t* sp = s_ptr[wave];
  if (nr > 0) {
    hash_rows_to_lds(sh, row_offset + (uint64_t)r0, nr, B, key, lane);
    for (int i = lane; i <= nr; i += 64) {
      // clamp so that malformed row_ptr can never index outside [0, nnz)
      sp[i] = min(max(row_ptr[r0 + i], 0), nnz);
    }
  }
  __syncthreads();
  if (nr == 0) return;
  const int32_t kb = sp[0], ke = sp[nr];
  for (int32_t base = kb; base < ke; base += 64) {
    const int32_t k = base + lane;
    if (k < ke) {
      const int32_t c = col_idx[k];
      const T v = vals[k];
      // local row of entry k: the largest i < nr with sp[i] <= k
      int lo = 0;
#pragma unroll
      for (int step = kRowsPerWave / 2; step > 0; step >>= 1)
        if (lo + step < nr && sp[lo + step] <= k) lo += step;
      const uint32_t hp = sh[lo];
      if ((unsigned)c < (unsigned)d)
        atomic_add(&SX[(size_t)hash_bucket(hp) * d + c], hash_negative(hp) ? -v : v);
    }
  }
}

// Dense X, d <= 64: LPR lanes per row (power of two >= d), 64/LPR rows per
// pass, U passes in flight before their atomics are issued.
template <typename T, int LPR>
__global__ __launch_bounds__(kThreads) void sx_dense_atomic_kernel(
    const T* __restrict__ X, int64_t ldx, int64_t n, int d, uint32_t B, Key key,
    uint64_t row_offset, T* __restrict__ SX) {
  constexpr int RPP = 64 / LPR;
  constexpr int U = 8;
  __shared__ uint32_t s_hash[kWaves][kRowsPerWave];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * kWaves + wave) * kRowsPerWave;
  const int nr = r0 < n ? (int)min((int64_t)kRowsPerWave, n - r0) : 0;
  uint32_t* sh = s_hash[wave];
  if (nr > 0) hash_rows_to_lds(sh, row_offset + (uint64_t)r0, nr, B, key, lane);
  __syncthreads();
  if (nr == 0) return;
  const int sub = lane / LPR, c = lane % LPR;
  const bool col_ok = c < d;
  const T* xr = X + r0 * ldx;
  for (int j0 = 0; j0 < nr; j0 += RPP * U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * RPP + sub;
      v[u] = (j < nr && col_ok) ? xr[(int64_t)j * ldx + c] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * RPP + sub;
      if (j < nr && col_ok) {
        const uint32_t hp = sh[j];
        atomic_add(&SX[(size_t)hash_bucket(hp) * d + c], hash_negative(hp) ? -v[u] : v[u]);
      }
    }
  }
}

// Dense X, d > 64: workgroup (bx, by) takes columns [64 by, 64 by + 64), a
// lane per column, and each of its wavefronts a run of rpw rows (at most
// kRowsPerWave, a multiple of 4), U rows in flight before their atomics.
// A row's 64 columns are one coalesced load and 64 atomics on adjacent
// words of its S X row.  rpw shrinks for small X, so that a 1000-row X
// still spreads over some thousand wavefronts.
template <typename T>
__global__ __launch_bounds__(kThreads) void sx_dense_wide_kernel(
    const T* __restrict__ X, int64_t ldx, int64_t n, int d, uint32_t B, Key key,
    uint64_t row_offset, T* __restrict__ SX, int rpw) {
  constexpr int U = 8;
  __shared__ uint32_t s_hash[kWaves][kRowsPerWave];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * kWaves + wave) * rpw;
  const int nr = r0 < n ? (int)min((int64_t)rpw, n - r0) : 0;
  uint32_t* sh = s_hash[wave];
  if (nr > 0) hash_rows_to_lds(sh, row_offset + (uint64_t)r0, nr, B, key, lane);
  __syncthreads();
  const int c = (int)blockIdx.y * 64 + lane;
  if (nr == 0 || c >= d) return;
  const T* xc = X + r0 * ldx + c;
  for (int j0 = 0; j0 < nr; j0 += U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = j0 + u < nr ? xc[(int64_t)(j0 + u) * ldx] : T(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j0 + u < nr) {
        const uint32_t hp = sh[j0 + u];
        atomic_add(&SX[(size_t)hash_bucket(hp) * d + c], hash_negative(hp) ? -v[u] : v[u]);
      }
    }
  }
}

// Rows per wavefront of the wide kernel: about 4096 wavefronts over the
// whole product (rows x 64-column groups), 4 to kRowsPerWave rows each.
inline int wide_rows_per_wave(int64_t n, int d) {
  const int64_t groups = (d + 63) / 64;
  int64_t r = (n * groups + 4095) / 4096;
  r = (r + 3) / 4 * 4;
  return (int)(r < 4 ? 4 : r > kRowsPerWave ? kRowsPerWave : r);
}

inline unsigned blocks_for_rows(int64_t n) {
  const int64_t per = (int64_t)kWaves * kRowsPerWave;
  return (unsigned)((n + per - 1) / per);
}

}  // namespace

template <typename T>
hipError_t launch_fill_zero(T* p, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + kThreads - 1) / kThreads;
  if (blocks > 16384) blocks = 16384;
  fill_zero_kernel<T><<<(unsigned)blocks, kThreads, 0, s>>>(p, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sx_csr_atomic(const int32_t* row_ptr, const int32_t* col_idx, const T* vals,
                                int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                                uint64_t row_offset, T* SX, hipStream_t s) {
  sx_csr_atomic_kernel<T><<<blocks_for_rows(n), kThreads, 0, s>>>(
      row_ptr, col_idx, vals, n, (int32_t)nnz, d, B, key, row_offset, SX);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sx_dense_atomic(const T* X, int64_t ldx, int64_t n, int d, uint32_t B, Key key,
                                  uint64_t row_offset, T* SX, hipStream_t s) {
  const unsigned g = blocks_for_rows(n);
  if (d <= 8)
    sx_dense_atomic_kernel<T, 8><<<g, kThreads, 0, s>>>(X, ldx, n, d, B, key, row_offset, SX);
  else if (d <= 16)
    sx_dense_atomic_kernel<T, 16><<<g, kThreads, 0, s>>>(X, ldx, n, d, B, key, row_offset, SX);
  else if (d <= 32)
    sx_dense_atomic_kernel<T, 32><<<g, kThreads, 0, s>>>(X, ldx, n, d, B, key, row_offset, SX);
  else if (d <= 64)
    sx_dense_atomic_kernel<T, 64><<<g, kThreads, 0, s>>>(X, ldx, n, d, B, key, row_offset, SX);
  else {
    const int rpw = wide_rows_per_wave(n, d);
    const int64_t per = (int64_t)kWaves * rpw;
    const dim3 grid((unsigned)((n + per - 1) / per), (unsigned)((d + 63) / 64));
    sx_dense_wide_kernel<T><<<grid, kThreads, 0, s>>>(X, ldx, n, d, B, key, row_offset, SX, rpw);
  }
  return hipGetLastError();
}

template hipError_t launch_fill_zero<float>(float*, size_t, hipStream_t);
template hipError_t launch_fill_zero<double>(double*, size_t, hipStream_t);
template hipError_t launch_fill_zero<int32_t>(int32_t*, size_t, hipStream_t);
template hipError_t launch_sx_csr_atomic<float>(const int32_t*, const int32_t*, const float*,
                                                int64_t, int64_t, int, uint32_t, Key, uint64_t,
                                                float*, hipStream_t);
template hipError_t launch_sx_csr_atomic<double>(const int32_t*, const int32_t*, const double*,
                                                 int64_t, int64_t, int, uint32_t, Key, uint64_t,
                                                 double*, hipStream_t);
template hipError_t launch_sx_dense_atomic<float>(const float*, int64_t, int64_t, int, uint32_t,
                                                  Key, uint64_t, float*, hipStream_t);
template hipError_t launch_sx_dense_atomic<double>(const double*, int64_t, int64_t, int, uint32_t,
                                                   Key, uint64_t, double*, hipStream_t);

}  // namespace cg
