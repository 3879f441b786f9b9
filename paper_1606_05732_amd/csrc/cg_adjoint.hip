// Adjoint of the transform: T^T dY = S^T (G^T dY).  T = G S is linear
// (Section 1.1), so this is the gradient of <dY, T X> with respect to X.
//
//  gt_dy_kernel   Z = G^T dY (B x d): contraction over the m rows of G,
//                 G regenerated in registers exactly as in the forward
//                 product (same Philox counters), on 16x16x4 MFMA.
//  gather_*       dX[r][:] = sigma(r) Z[h(r)][:]  (dense), or
//                 dvals[k] = sigma(r) Z[h(r)][col_k]  (CSR values).
//
// Also the small kernels behind the cg_debug_* test entry points.
#include "cg_internal.hpp"
#include "cg_rng.hpp"

namespace cg {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  using type = v4f;
};
template <>
struct Vec4<double> {
  using type = v4d;
};

__device__ __forceinline__ v4f mfma_k4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma_k4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Result row held in accumulator register r for kq = lane / 16: FP32
// 16x16x4 keeps rows 4 kq .. 4 kq + 3, FP64 16x16x4 rows kq, kq+4, kq+8,
// kq+12 (measured on gfx950).
template <typename T>
__device__ __forceinline__ int d_row(int kq, int r) {
  return sizeof(T) == 8 ? kq + 4 * r : 4 * kq + r;
}

// One wavefront computes Z for 16 MB consecutive buckets b (MB blocks of
// 16) and up to 16 NB columns.  MFMA roles: M = bucket (lane % 16), K =
// row i of G, N = column of dY.  K slot kq of step s holds G row
// 4 (4 s + kq) + t for sub-step t, so one Philox block (b, 4 s + kq) feeds
// the four sub-steps.  A step's dY values serve all MB bucket blocks.
// (dY is read from memory -- it stays in the caches; staging it in LDS per
// workgroup cost more occupancy than it saved.)
constexpr int kGtMB = 2;

template <typename T, int NB>
__global__ __launch_bounds__(kThreads) void gt_dy_kernel(const T* __restrict__ dY, int m, int d,
                                                         int64_t B, Key key, T* __restrict__ Z) {
  using V = typename Vec4<T>::type;
  constexpr int MB = kGtMB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int bb = lane & 15, kq = lane >> 4;
  const int n0 = blockIdx.y * NB * 16;
  const int64_t b0 = ((int64_t)blockIdx.x * kWaves + wave) * 16 * MB;
  if (b0 >= B) return;
  V acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = V{0, 0, 0, 0};
  int col[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) col[nb] = n0 + nb * 16 + bb;
  const int steps = (m + 15) / 16;
  for (int s = 0; s < steps; ++s) {
    const int qq = 4 * s + kq;
    T g[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int64_t b = b0 + 16 * mb + bb;
#pragma unroll
      for (int t = 0; t < 4; ++t) g[mb][t] = T(0);
      if (b < B && 4 * qq < m) box_muller(gauss_block((uint32_t)b, (uint32_t)qq, key.k0, key.k1), g[mb]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = 4 * qq + t;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const T y = (i < m && col[nb] < d) ? dY[(size_t)i * d + col[nb]] : T(0);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mfma_k4(g[mb][t], y, acc[mb][nb]);
      }
    }
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = b0 + 16 * mb + d_row<T>(kq, r);
        if (row < B && col[nb] < d) Z[row * d + col[nb]] = acc[mb][nb][r];
      }
}

__device__ __forceinline__ void hash_rows_to_lds(uint32_t* sh, uint64_t g0, int nr, uint32_t B,
                                                 Key key, int lane) {
  uint32_t hv[4];
  hash4(g0 + 4 * (uint64_t)lane, B, key.k0, key.k1, hv);
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (4 * lane + t < nr) sh[4 * lane + t] = hv[t];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void gather_dense_kernel(const T* __restrict__ Z, int64_t n,
                                                                int d, uint32_t B, Key key,
                                                                uint64_t row_offset,
                                                                T* __restrict__ dX, int64_t lddx) {
  __shared__ uint32_t s_hash[kWaves][kRowsPerWave];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * kWaves + wave) * kRowsPerWave;
  const int nr = r0 < n ? (int)min((int64_t)kRowsPerWave, n - r0) : 0;
  uint32_t* sh = s_hash[wave];
  if (nr > 0) hash_rows_to_lds(sh, row_offset + (uint64_t)r0, nr, B, key, lane);
  __syncthreads();
  if (nr == 0) return;
  // lanes per row: smallest power of two >= min(d, 64)
  int lpr = 1;
  while (lpr < d && lpr < 64) lpr <<= 1;
  const int rpp = 64 / lpr;
  const int sub = lane / lpr, c0 = lane % lpr;
  for (int j = sub; j < nr; j += rpp) {
    const uint32_t hp = sh[j];
    const T* src = Z + (size_t)hash_bucket(hp) * d;
    T* dst = dX + (r0 + j) * lddx;
    const bool neg = hash_negative(hp);
    for (int c = c0; c < d; c += lpr) {
      const T v = src[c];
      dst[c] = neg ? -v : v;
    }
  }
}

// FP32 rows whose d is a multiple of 4, with Z, dX and the row stride
// 16-byte aligned: 16-byte loads and stores, d / 4 lanes per row (rounded
// up to a power of two, at most 64), and four groups of rows per step, so
// that every lane has four row reads in flight before its first store.
// The dX rows are whole lines written once: non-temporal stores, so that Z
// (read at random rows) keeps the caches.
__global__ __launch_bounds__(kThreads) void gather_dense_vec_kernel(const float* __restrict__ Z,
                                                                    int64_t n, int d, uint32_t B,
                                                                    Key key, uint64_t row_offset,
                                                                    float* __restrict__ dX,
                                                                    int64_t lddx) {
  __shared__ uint32_t s_hash[kWaves][kRowsPerWave];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * kWaves + wave) * kRowsPerWave;
  const int nr = r0 < n ? (int)min((int64_t)kRowsPerWave, n - r0) : 0;
  uint32_t* sh = s_hash[wave];
  if (nr > 0) hash_rows_to_lds(sh, row_offset + (uint64_t)r0, nr, B, key, lane);
  __syncthreads();
  if (nr == 0) return;
  const int d4 = d >> 2;
  int lpr = 1;
  while (lpr < d4 && lpr < 64) lpr <<= 1;
  const int rpp = 64 / lpr;   // rows per wavefront instruction
  const int sub = lane / lpr, c0 = lane % lpr;
  constexpr int U = 4;
  for (int j0 = 0; j0 < nr; j0 += U * rpp) {
    for (int c = c0; c < d4; c += lpr) {
      v4f v[U];
      uint32_t hp[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = min(j0 + u * rpp + sub, nr - 1);   // clamped: a row past nr is reread, not written
        hp[u] = sh[j];
        v[u] = ((const v4f*)(Z + (size_t)hash_bucket(hp[u]) * d))[c];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * rpp + sub;
        if (j < nr) {
          const v4f w = hash_negative(hp[u]) ? -v[u] : v[u];
          __builtin_nontemporal_store(w, (v4f*)(dX + (r0 + j) * lddx) + c);
        }
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void gather_csr_kernel(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const T* __restrict__ Z, int64_t n, int32_t nnz, int d, uint32_t B, Key key,
    uint64_t row_offset, T* __restrict__ dvals) {
  __shared__ uint32_t s_hash[kWaves][kRowsPerWave];
  __shared__ int32_t s_ptr[kWaves][kRowsPerWave + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * kWaves + wave) * kRowsPerWave;
  const int nr = r0 < n ? (int)min((int64_t)kRowsPerWave, n - r0) : 0;
  uint32_t* sh = s_hash[wave];
  int32_t* sp = s_ptr[wave];
  if (nr > 0) {
    hash_rows_to_lds(sh, row_offset + (uint64_t)r0, nr, B, key, lane);
    for (int i = lane; i <= nr; i += 64) sp[i] = min(max(row_ptr[r0 + i], 0), nnz);
  }
  __syncthreads();
  if (nr == 0) return;
  const int32_t kb = sp[0], ke = sp[nr];
  for (int32_t base = kb; base < ke; base += 64) {
    const int32_t k = base + lane;
    if (k < ke) {
      const int32_t c = col_idx[k];
      int lo = 0;
#pragma unroll
      for (int step = kRowsPerWave / 2; step > 0; step >>= 1)
        if (lo + step < nr && sp[lo + step] <= k) lo += step;
      const uint32_t hp = sh[lo];
      T v = T(0);
      if ((unsigned)c < (unsigned)d) v = Z[(size_t)hash_bucket(hp) * d + c];
      dvals[k] = hash_negative(hp) ? -v : v;
    }
  }
}

__global__ void debug_philox_kernel(Key key, const uint32_t* __restrict__ ctr, int64_t count,
                                    uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const Words4 c{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
  const Words4 w = philox10(c, key.k0, key.k1);
  out[4 * i] = w.x;
  out[4 * i + 1] = w.y;
  out[4 * i + 2] = w.z;
  out[4 * i + 3] = w.w;
}

__global__ void debug_hash_kernel(Key key, uint32_t B, uint64_t row0, int64_t count,
                                  uint32_t* __restrict__ h, int8_t* __restrict__ sigma) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t g = row0 + (uint64_t)i;
  const Words4 w = hash_block(g >> 2, key.k0, key.k1);
  const uint32_t hp = pack_hash(word_at(w, (int)(g & 3)), B);
  h[i] = hash_bucket(hp);
  sigma[i] = hash_negative(hp) ? (int8_t)-1 : (int8_t)1;
}

template <typename T>
__global__ void debug_gaussian_kernel(Key key, int64_t m, int64_t b0, int64_t nb,
                                      T* __restrict__ G) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nq = (m + 3) / 4;
  if (i >= nq * nb) return;
  const int64_t q = i / nb, j = i % nb;
  T z[4];
  box_muller(gauss_block((uint32_t)(b0 + j), (uint32_t)q, key.k0, key.k1), z);
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (4 * q + t < m) G[(4 * q + t) * nb + j] = z[t];
}

inline unsigned blocks_for_rows(int64_t n) {
  const int64_t per = (int64_t)kWaves * kRowsPerWave;
  return (unsigned)((n + per - 1) / per);
}

}  // namespace

template <typename T>
hipError_t launch_gt_dy(const T* dY, int m, int d, int64_t B, Key key, T* Z, hipStream_t s) {
  const int need = (d + 15) / 16;
  const int nb = need < 4 ? need : 4;
  const unsigned gx = (unsigned)((B + 16 * kGtMB * kWaves - 1) / (16 * kGtMB * kWaves));
  const unsigned gy = (unsigned)((d + 16 * nb - 1) / (16 * nb));
  dim3 grid(gx, gy);
  switch (nb) {
    case 1: gt_dy_kernel<T, 1><<<grid, kThreads, 0, s>>>(dY, m, d, B, key, Z); break;
    case 2: gt_dy_kernel<T, 2><<<grid, kThreads, 0, s>>>(dY, m, d, B, key, Z); break;
    case 3: gt_dy_kernel<T, 3><<<grid, kThreads, 0, s>>>(dY, m, d, B, key, Z); break;
    default: gt_dy_kernel<T, 4><<<grid, kThreads, 0, s>>>(dY, m, d, B, key, Z); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_dense(const T* Z, int64_t n, int d, uint32_t B, Key key,
                               uint64_t row_offset, T* dX, int64_t lddx, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (d % 4 == 0 && lddx % 4 == 0 && ((uintptr_t)Z & 15) == 0 && ((uintptr_t)dX & 15) == 0) {
      gather_dense_vec_kernel<<<blocks_for_rows(n), kThreads, 0, s>>>(Z, n, d, B, key, row_offset,
                                                                        dX, lddx);
      return hipGetLastError();
    }
  }
  gather_dense_kernel<T><<<blocks_for_rows(n), kThreads, 0, s>>>(Z, n, d, B, key, row_offset, dX,
                                                                 lddx);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_csr(const int32_t* row_ptr, const int32_t* col_idx, const T* Z,
                             int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                             uint64_t row_offset, T* dvals, hipStream_t s) {
  gather_csr_kernel<T><<<blocks_for_rows(n), kThreads, 0, s>>>(row_ptr, col_idx, Z, n,
                                                               (int32_t)nnz, d, B, key,
                                                               row_offset, dvals);
  return hipGetLastError();
}

hipError_t launch_debug_philox(Key key, const uint32_t* ctr, int64_t count, uint32_t* out,
                               hipStream_t s) {
  if (count == 0) return hipSuccess;
  debug_philox_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(key, ctr, count, out);
  return hipGetLastError();
}

hipError_t launch_debug_hash(Key key, uint32_t B, uint64_t row0, int64_t count, uint32_t* h,
                             int8_t* sigma, hipStream_t s) {
  if (count == 0) return hipSuccess;
  debug_hash_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(key, B, row0, count, h, sigma);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_debug_gaussian(Key key, int64_t m, int64_t b0, int64_t nb, T* G, hipStream_t s) {
  const int64_t total = (m + 3) / 4 * nb;
  if (total == 0) return hipSuccess;
  debug_gaussian_kernel<T><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(key, m, b0, nb, G);
  return hipGetLastError();
}

template hipError_t launch_gt_dy<float>(const float*, int, int, int64_t, Key, float*, hipStream_t);
template hipError_t launch_gt_dy<double>(const double*, int, int, int64_t, Key, double*,
                                         hipStream_t);
template hipError_t launch_gather_dense<float>(const float*, int64_t, int, uint32_t, Key, uint64_t,
                                               float*, int64_t, hipStream_t);
template hipError_t launch_gather_dense<double>(const double*, int64_t, int, uint32_t, Key,
                                                uint64_t, double*, int64_t, hipStream_t);
template hipError_t launch_gather_csr<float>(const int32_t*, const int32_t*, const float*, int64_t,
                                             int64_t, int, uint32_t, Key, uint64_t, float*,
                                             hipStream_t);
template hipError_t launch_gather_csr<double>(const int32_t*, const int32_t*, const double*,
                                              int64_t, int64_t, int, uint32_t, Key, uint64_t,
                                              double*, hipStream_t);
template hipError_t launch_debug_gaussian<float>(Key, int64_t, int64_t, int64_t, float*,
                                                 hipStream_t);
template hipError_t launch_debug_gaussian<double>(Key, int64_t, int64_t, int64_t, double*,
                                                  hipStream_t);

}  // namespace cg
