// Streaming probes of the memory system, the ceilings the kernels are
// measured against: a device copy, a read and a write of `bytes` (plain or
// non-temporal accesses), with
// 16-byte accesses, consecutive lanes on consecutive addresses, eight
// accesses in flight per lane, over a grid of 32 workgroups per CU.
#include "cg_internal.hpp"
#include "cg_rng.hpp"

namespace cg {

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kThreads = 256;
constexpr int kUnroll = 8;

// NT: non-temporal accesses (streamed past the caches).
template <bool NT>
__device__ __forceinline__ u32x4 ld(const u32x4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool NT>
__device__ __forceinline__ void st(u32x4* p, u32x4 v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <bool NT>
__global__ __launch_bounds__(kThreads) void stream_copy_kernel(const u32x4* __restrict__ src,
                                                               u32x4* __restrict__ dst,
                                                               int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
    u32x4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = ld<NT>(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) st<NT>(dst + i + u * stride, v[u]);
  }
  for (; i < n; i += stride) st<NT>(dst + i, ld<NT>(src + i));
}

// The xor of everything read, one word per workgroup (so the loads stay).
template <bool NT>
__global__ __launch_bounds__(kThreads) void stream_read_kernel(const u32x4* __restrict__ src,
                                                               uint32_t* __restrict__ out,
                                                               int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  u32x4 acc = {0u, 0u, 0u, 0u};
  for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
    u32x4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = ld<NT>(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc ^= v[u];
  }
  for (; i < n; i += stride) acc ^= ld<NT>(src + i);
  uint32_t x = acc.x ^ acc.y ^ acc.z ^ acc.w;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x ^= (uint32_t)__shfl_xor((int)x, off, 64);
  __shared__ uint32_t s[kThreads / 64];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = 0;
    for (int w = 0; w < kThreads / 64; ++w) r ^= s[w];
    out[blockIdx.x] = r;
  }
}

template <bool NT>
__global__ __launch_bounds__(kThreads) void stream_write_kernel(u32x4* __restrict__ dst, int64_t n,
                                                                uint32_t value) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  const u32x4 v = {value, value, value, value};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) st<NT>(dst + i, v);
}

// The generator's own ceiling: the normals of G for columns [0, B) and
// row quads [0, m / 4) (Philox4x32-10 of counter (b, q, 1, 0), FP32
// Box-Muller, exactly as the contractions draw them), with nothing else:
// each thread adds up its normals and writes one sum.  Thread t takes the
// contiguous run of blocks [t per, (t + 1) per) in (b, q) order, with the
// counters stepped by increments (one division per thread, none per
// block), eight blocks in flight.
__global__ __launch_bounds__(kThreads) void normals_rate_kernel(Key key, uint32_t quads, int64_t B,
                                                                int64_t per,
                                                                float* __restrict__ sink) {
  const int64_t t0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t nblk = B * quads;
  constexpr int U = 8;
  float acc = 0.0f;
  int64_t k = t0 * per;
  const int64_t kend = min(k + per, nblk);
  uint32_t b = 0u, q = 0u;
  if (k < kend) {
    b = (uint32_t)(k / quads);
    q = (uint32_t)(k % quads);
  }
  for (; k + U <= kend; k += U) {
    uint32_t bb[U], qq[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      bb[u] = b;
      qq[u] = q;
      if (++q == quads) {
        q = 0u;
        ++b;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float z[4];
      box_muller(gauss_block(bb[u], qq[u], key.k0, key.k1), z);
      acc += (z[0] + z[1]) + (z[2] + z[3]);
    }
  }
  for (; k < kend; ++k) {
    float z[4];
    box_muller(gauss_block(b, q, key.k0, key.k1), z);
    acc += (z[0] + z[1]) + (z[2] + z[3]);
    if (++q == quads) {
      q = 0u;
      ++b;
    }
  }
  sink[t0] = acc;
}

}  // namespace

int stream_blocks() { return 256 * 32; }

// 2048 workgroups: eight wavefronts per SIMD, each thread drawing a run
// of blocks long enough that the launch's own ramp does not dominate
constexpr int kNormalsBlocks = 2048;
int normals_threads() { return kNormalsBlocks * kThreads; }

hipError_t launch_normals_rate(Key key, int64_t m, int64_t B, float* sink, hipStream_t s) {
  const int64_t T = (int64_t)normals_threads();
  const int64_t per = (B * (m / 4) + T - 1) / T;
  normals_rate_kernel<<<(unsigned)kNormalsBlocks, kThreads, 0, s>>>(key, (uint32_t)(m / 4), B, per,
                                                                    sink);
  return hipGetLastError();
}

hipError_t launch_stream(int kind, const void* src, void* dst, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 16;
  const unsigned blocks = (unsigned)stream_blocks();
  const bool nt = kind >= 3;
  switch (kind % 3) {
    case 0:
      if (nt) stream_copy_kernel<true><<<blocks, kThreads, 0, s>>>((const u32x4*)src, (u32x4*)dst, n);
      else stream_copy_kernel<false><<<blocks, kThreads, 0, s>>>((const u32x4*)src, (u32x4*)dst, n);
      break;
    case 1:
      if (nt) stream_read_kernel<true><<<blocks, kThreads, 0, s>>>((const u32x4*)src, (uint32_t*)dst, n);
      else stream_read_kernel<false><<<blocks, kThreads, 0, s>>>((const u32x4*)src, (uint32_t*)dst, n);
      break;
    default:
      if (nt) stream_write_kernel<true><<<blocks, kThreads, 0, s>>>((u32x4*)dst, n, 0x3f800000u);
      else stream_write_kernel<false><<<blocks, kThreads, 0, s>>>((u32x4*)dst, n, 0x3f800000u);
      break;
  }
  return hipGetLastError();
}

}  // namespace cg
