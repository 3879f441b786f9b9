// S X by bucket-range binning with LDS accumulation (FP32 data).
//
// Device-scope float atomics are resolved far from the CUs on this GPU and
// cost one memory-side read-modify-write each, and float atomics in LDS are
// several times slower than integer ones.  So S X (Section 1.1: every
// stored entry (r, c, v) adds sigma(r) v to SX[h(r)][c]) is computed in
// two passes over the data without any floating-point atomic:
//
//  1. split: the buckets are cut into R ranges of Bp = 2^k consecutive
//     buckets whose S X slice fits in LDS.  A workgroup takes a tile of
//     16384 rows, counts its items per range (bin_count), an exclusive scan
//     over (range, tile) gives every tile a private window in each range's
//     item list, and bin_scatter writes the items there.
//  2. reduce: one workgroup per range accumulates its items into an LDS
//     slice and writes the slice -- every bucket of S X is written exactly
//     once, so no zero fill is needed.
//
// CSR items are (cell = local bucket * d + column, sigma v).  They are
// summed as 64-bit fixed-point integers with ds_add_u64: the range's scale
// 2^f is chosen from the largest |v| in the range and the item count so
// that no partial sum can overflow, and integer addition does not depend
// on order -- the result is bitwise reproducible run to run.  A range that
// holds a NaN or infinity is summed with float atomics instead (same
// propagation as the atomic path).
//
// Dense items are (row | sign << 31, local bucket).  In the reduce the four
// wavefronts of a workgroup own disjoint buckets (lb mod 4), read every
// item of the range, gather the rows they own whole (lanes = columns) and
// add them with plain LDS read-add-write; up to 64 / LPR rows are added at
// once, each into its own copy of the slice, and the copies are added in a
// fixed order at the end.
#include "cg_internal.hpp"
#include "cg_rng.hpp"

namespace cg {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = 4;
constexpr int kTileRows = 16384;
constexpr int kSubRows = kWaves * kRowsPerWave;   // rows staged per pass in the CSR scatter

// One dynamic LDS area per kernel, typed at each use.
extern __shared__ __align__(16) unsigned char dyn_lds[];

// ------------------------------------------------------------------ count
template <bool CSR>
__global__ __launch_bounds__(kThreads) void bin_count_kernel(
    const int32_t* __restrict__ row_ptr, int64_t n, int32_t nnz, uint32_t B, Key key,
    uint64_t row_offset, int bp_shift, int R, int64_t ntiles, uint32_t* __restrict__ hist) {
  uint32_t* s_cnt = (uint32_t*)dyn_lds;
  for (int i = threadIdx.x; i < R; i += kThreads) s_cnt[i] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kTileRows;
  const int64_t t1 = min(t0 + (int64_t)kTileRows, n);
  for (int64_t r = t0 + 4 * (int64_t)threadIdx.x; r < t1; r += 4 * kThreads) {
    uint32_t hv[4];
    hash4(row_offset + (uint64_t)r, B, key.k0, key.k1, hv);
    int32_t ptr[5];
    if (CSR) {
#pragma unroll
      for (int j = 0; j < 5; ++j) ptr[j] = r + j <= t1 ? min(max(row_ptr[r + j], 0), nnz) : 0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (r + j < t1) {
        const uint32_t len = CSR ? (uint32_t)max(ptr[j + 1] - ptr[j], 0) : 1u;
        if (len) atomicAdd(&s_cnt[hash_bucket(hv[j]) >> bp_shift], len);
      }
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < R; p += kThreads) hist[(int64_t)p * ntiles + blockIdx.x] = s_cnt[p];
}

// Per-range base offset of this tile and the number of slots it owns.
__device__ __forceinline__ void load_windows(const uint32_t* __restrict__ offs, int R,
                                             int64_t ntiles, uint32_t total, uint32_t* s_base,
                                             uint32_t* s_lim) {
  const int64_t len = (int64_t)R * ntiles;
  for (int p = threadIdx.x; p < R; p += kThreads) {
    const int64_t idx = (int64_t)p * ntiles + blockIdx.x;
    const uint32_t base = offs[idx];
    // never past the item buffer, even if a malformed CSR made the counts
    // exceed nnz
    const uint32_t next = min(idx + 1 < len ? offs[idx + 1] : total, total);
    s_base[p] = base;
    s_lim[p] = next > base ? next - base : 0u;
  }
}

// ------------------------------------------------------------------ scatter
__global__ __launch_bounds__(kThreads) void bin_scatter_csr_kernel(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ vals, int64_t n, int32_t nnz, int d, uint32_t B, Key key,
    uint64_t row_offset, int bp_shift, int R, int64_t ntiles, const uint32_t* __restrict__ offs,
    uint32_t total, uint2* __restrict__ items, uint32_t* __restrict__ hmax) {
  uint32_t* smem = (uint32_t*)dyn_lds;
  uint32_t* s_base = smem;
  uint32_t* s_lim = smem + R;
  uint32_t* s_cnt = smem + 2 * R;
  uint32_t* s_max = smem + 3 * R;
  uint32_t* s_hash = smem + 4 * R;                                  // kWaves * 256
  int32_t* s_ptr = (int32_t*)(s_hash + kWaves * kRowsPerWave);     // kWaves * 257
  load_windows(offs, R, ntiles, total, s_base, s_lim);
  for (int p = threadIdx.x; p < R; p += kThreads) {
    s_cnt[p] = 0;
    s_max[p] = 0;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* sh = s_hash + wave * kRowsPerWave;
  int32_t* sp = s_ptr + wave * (kRowsPerWave + 1);
  const uint32_t bmask = (1u << bp_shift) - 1u;
  const int64_t t0 = (int64_t)blockIdx.x * kTileRows;
  const int64_t t1 = min(t0 + (int64_t)kTileRows, n);
  for (int64_t sub = t0; sub < t1; sub += kSubRows) {
    __syncthreads();
    const int64_t r0 = sub + (int64_t)wave * kRowsPerWave;
    const int nr = r0 < t1 ? (int)min((int64_t)kRowsPerWave, t1 - r0) : 0;
    if (nr > 0) {
      uint32_t hv[4];
      hash4(row_offset + (uint64_t)r0 + 4 * (uint64_t)lane, B, key.k0, key.k1, hv);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (4 * lane + t < nr) sh[4 * lane + t] = hv[t];
      for (int i = lane; i <= nr; i += 64) sp[i] = min(max(row_ptr[r0 + i], 0), nnz);
    }
    __syncthreads();
    if (nr == 0) continue;
    const int32_t kb = sp[0], ke = sp[nr];
    for (int32_t base = kb; base < ke; base += 64) {
      const int32_t k = base + lane;
      if (k < ke) {
        const int32_t c = col_idx[k];
        const float v = vals[k];
        int lo = 0;
#pragma unroll
        for (int step = kRowsPerWave / 2; step > 0; step >>= 1)
          if (lo + step < nr && sp[lo + step] <= k) lo += step;
        const uint32_t hp = sh[lo];
        const uint32_t bucket = hash_bucket(hp);
        const uint32_t p = bucket >> bp_shift;
        const bool ok = (unsigned)c < (unsigned)d;
        const uint32_t cell = ok ? (bucket & bmask) * (uint32_t)d + (uint32_t)c : 0u;
        const float sv = ok ? (hash_negative(hp) ? -v : v) : 0.0f;
        const uint32_t slot = atomicAdd(&s_cnt[p], 1u);
        if (slot < s_lim[p]) items[s_base[p] + slot] = make_uint2(cell, __float_as_uint(sv));
        atomicMax(&s_max[p], __float_as_uint(fabsf(sv)));
      }
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < R; p += kThreads) hmax[(int64_t)p * ntiles + blockIdx.x] = s_max[p];
}

__global__ __launch_bounds__(kThreads) void bin_scatter_dense_kernel(
    int64_t n, uint32_t B, Key key, uint64_t row_offset, int bp_shift, int R, int64_t ntiles,
    const uint32_t* __restrict__ offs, uint32_t total, uint2* __restrict__ items) {
  uint32_t* smem = (uint32_t*)dyn_lds;
  uint32_t* s_base = smem;
  uint32_t* s_lim = smem + R;
  uint32_t* s_cnt = smem + 2 * R;
  load_windows(offs, R, ntiles, total, s_base, s_lim);
  for (int p = threadIdx.x; p < R; p += kThreads) s_cnt[p] = 0;
  __syncthreads();
  const uint32_t bmask = (1u << bp_shift) - 1u;
  const int64_t t0 = (int64_t)blockIdx.x * kTileRows;
  const int64_t t1 = min(t0 + (int64_t)kTileRows, n);
  for (int64_t r = t0 + 4 * (int64_t)threadIdx.x; r < t1; r += 4 * kThreads) {
    uint32_t hv[4];
    hash4(row_offset + (uint64_t)r, B, key.k0, key.k1, hv);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (r + j < t1) {
        const uint32_t bucket = hash_bucket(hv[j]);
        const uint32_t p = bucket >> bp_shift;
        const uint32_t slot = atomicAdd(&s_cnt[p], 1u);
        if (slot < s_lim[p])
          items[s_base[p] + slot] =
              make_uint2((uint32_t)(r + j) | (hv[j] & 0x80000000u), bucket & bmask);
      }
    }
  }
}

// ------------------------------------------------------------------ reduce
__device__ __forceinline__ uint32_t block_max_u32(uint32_t v, uint32_t* s_red) {
  s_red[threadIdx.x] = v;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s_red[threadIdx.x] = max(s_red[threadIdx.x], s_red[threadIdx.x + off]);
    __syncthreads();
  }
  const uint32_t r = s_red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void range_of(const uint32_t* __restrict__ offs, int p, int R,
                                         int64_t ntiles, uint32_t total, uint32_t* start,
                                         uint32_t* end) {
  const uint32_t s = offs[(int64_t)p * ntiles];
  const uint32_t e = p + 1 < R ? offs[(int64_t)(p + 1) * ntiles] : total;
  *start = min(s, total);
  *end = min(max(e, *start), total);
}

__global__ __launch_bounds__(kThreads) void bin_reduce_csr_kernel(
    const uint2* __restrict__ items, const uint32_t* __restrict__ offs,
    const uint32_t* __restrict__ hmax, int64_t ntiles, int R, uint32_t total, uint32_t B, int d,
    int bp_shift, float* __restrict__ SX) {
  unsigned long long* s_acc = (unsigned long long*)dyn_lds;
  __shared__ uint32_t s_red[kThreads];
  const int p = blockIdx.x;
  const int cells = (1 << bp_shift) * d;
  for (int i = threadIdx.x; i < cells; i += kThreads) s_acc[i] = 0ull;
  uint32_t mx = 0;
  for (int64_t t = threadIdx.x; t < ntiles; t += kThreads) mx = max(mx, hmax[(int64_t)p * ntiles + t]);
  const uint32_t amax_bits = block_max_u32(mx, s_red);   // also orders the zero fill
  uint32_t start, end;
  range_of(offs, p, R, ntiles, total, &start, &end);
  if (amax_bits >= 0x7f800000u) {
    // a NaN or an infinity in this range: float atomics keep IEEE semantics
    float* acc = (float*)s_acc;
    for (int i = threadIdx.x; i < cells; i += kThreads) acc[i] = 0.0f;
    __syncthreads();
    for (uint32_t i = start + threadIdx.x; i < end; i += kThreads) {
      const uint2 it = items[i];
      if (it.x < (uint32_t)cells) atomicAdd(&acc[it.x], __uint_as_float(it.y));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cells; i += kThreads) {
      const int64_t bucket = ((int64_t)p << bp_shift) + i / d;
      if (bucket < B) SX[bucket * d + i % d] = acc[i];
    }
    return;
  }
  // |partial sums| <= count * amax < 2^(E + lg) with amax < 2^E, count <= 2^lg
  int E = 0;
  if (amax_bits) frexpf(__uint_as_float(amax_bits), &E);
  const uint32_t count = end - start;
  int lg = 0;
  while (lg < 32 && (1u << lg) < count) ++lg;
  const int f = 61 - E - lg;
  const double scale = ldexp(1.0, f), inv = ldexp(1.0, -f);
  uint32_t i = start + threadIdx.x;
  for (; i + 3 * kThreads < end; i += 4 * kThreads) {
    uint2 it[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) it[u] = items[i + u * kThreads];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (it[u].x < (uint32_t)cells)
        atomicAdd(&s_acc[it[u].x],
                  (unsigned long long)__double2ll_rn((double)__uint_as_float(it[u].y) * scale));
  }
  for (; i < end; i += kThreads) {
    const uint2 it = items[i];
    if (it.x < (uint32_t)cells)
      atomicAdd(&s_acc[it.x], (unsigned long long)__double2ll_rn((double)__uint_as_float(it.y) * scale));
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cells; c += kThreads) {
    const int64_t bucket = ((int64_t)p << bp_shift) + c / d;
    if (bucket < B) SX[bucket * d + c % d] = (float)((double)(long long)s_acc[c] * inv);
  }
}

template <int LPR>
__global__ __launch_bounds__(kThreads) void bin_reduce_dense_kernel(
    const float* __restrict__ X, int64_t ldx, int64_t n, const uint2* __restrict__ items,
    const uint32_t* __restrict__ offs, int64_t ntiles, int R, uint32_t total, uint32_t B, int d,
    int bp_shift, float* __restrict__ SX) {
  constexpr int RPP = 64 / LPR;   // rows added per instruction, one slice copy each
  constexpr int U = 4;            // instructions' rows gathered before adding
  float* s_acc = (float*)dyn_lds;
  const int p = blockIdx.x;
  const int Bp = 1 << bp_shift;
  const int cells = Bp * d;
  for (int i = threadIdx.x; i < RPP * cells; i += kThreads) s_acc[i] = 0.0f;
  __syncthreads();
  uint32_t start, end;
  range_of(offs, p, R, ntiles, total, &start, &end);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane / LPR, c = lane % LPR;
  const bool cok = c < d;
  float* mycopy = s_acc + j * cells;
  for (uint32_t base = start; base < end; base += 64) {
    const uint32_t i = base + lane;
    uint2 it = make_uint2(0u, 0xffffffffu);
    if (i < end) it = items[i];
    const bool mine = i < end && it.y < (uint32_t)Bp && (int)(it.y % kWaves) == wave &&
                      (int64_t)(it.x & 0x7fffffffu) < n;
    uint64_t mask = __ballot(mine);
    while (mask) {
      float xv[U];
      uint32_t lbv[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        uint64_t mm = mask;
        for (int k = 0; k < u * RPP + j && mm; ++k) mm &= mm - 1;
        const int src = mm ? __ffsll((unsigned long long)mm) - 1 : 0;
        const uint32_t rs = __shfl(it.x, src, 64);
        lbv[u] = __shfl(it.y, src, 64);
        ok[u] = mm != 0 && cok;
        const float x = ok[u] ? X[(int64_t)(rs & 0x7fffffffu) * ldx + c] : 0.0f;
        xv[u] = (rs >> 31) ? -x : x;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) mycopy[lbv[u] * d + c] += xv[u];
      for (int k = 0; k < U * RPP && mask; ++k) mask &= mask - 1;
    }
  }
  __syncthreads();
  for (int cc = threadIdx.x; cc < cells; cc += kThreads) {
    float s = s_acc[cc];
#pragma unroll
    for (int jj = 1; jj < RPP; ++jj) s += s_acc[jj * cells + cc];
    const int64_t bucket = ((int64_t)p << bp_shift) + cc / d;
    if (bucket < B) SX[bucket * d + cc % d] = s;
  }
}

int lanes_per_row(int d) {
  int l = 1;
  while (l < d && l < 64) l <<= 1;
  return l;
}

struct Carve {
  uint32_t *hist, *sums, *hmax;
  uint2* items;
};

Carve carve(void* base, const BinGeom& g, int64_t count) {
  char* p = (char*)base;
  Carve c;
  const int64_t hl = (int64_t)g.R * g.ntiles;
  c.hist = (uint32_t*)p;
  p += align256((size_t)hl * 4);
  c.sums = (uint32_t*)p;
  p += align256((size_t)scan_sums_len(hl) * 4);
  c.hmax = (uint32_t*)p;
  p += align256((size_t)hl * 4);
  c.items = (uint2*)p;
  return c;
}

}  // namespace

BinGeom bin_geometry(bool csr, int64_t n, int d, int64_t B) {
  BinGeom g;
  int shift = 0;
  if (csr) {
    while (shift < 30 && ((int64_t)2 << shift) * d <= 4096) ++shift;   // int64 cells, 32 KB
    g.lds_bytes = (size_t)(1 << shift) * d * 8;
  } else {
    const int rpp = 64 / lanes_per_row(d);
    while (shift < 30 && (int64_t)rpp * ((int64_t)2 << shift) * d <= 8192) ++shift;  // 32 KB
    g.lds_bytes = (size_t)rpp * (1 << shift) * d * 4;
  }
  g.bp_shift = shift;
  g.R = (int)((B + ((int64_t)1 << shift) - 1) >> shift);
  g.ntiles = (n + kTileRows - 1) / kTileRows;
  g.ok = g.R <= (csr ? kBinMaxRangesCsr : kBinMaxRangesDense) && d <= (csr ? kMaxD : 64) &&
         n < ((int64_t)1 << 31) && g.R * g.ntiles < ((int64_t)1 << 30);
  return g;
}

size_t binned_scratch_bytes(const BinGeom& g, int64_t count) {
  const int64_t hl = (int64_t)g.R * g.ntiles;
  return 2 * align256((size_t)hl * 4) + align256((size_t)scan_sums_len(hl) * 4) +
         align256((size_t)count * 8);
}

hipError_t launch_sx_binned_csr(const int32_t* row_ptr, const int32_t* col_idx, const float* vals,
                                int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                                uint64_t row_offset, float* SX, void* scratch, hipStream_t s,
                                void* const* events) {
  const BinGeom g = bin_geometry(true, n, d, B);
  Carve c = carve(scratch, g, nnz);
  const int64_t hl = (int64_t)g.R * g.ntiles;
  bin_count_kernel<true><<<(unsigned)g.ntiles, kThreads, g.R * 4, s>>>(
      row_ptr, n, (int32_t)nnz, B, key, row_offset, g.bp_shift, g.R, g.ntiles, c.hist);
  hipError_t e = launch_exclusive_scan(c.hist, hl, c.sums, s);
  if (e != hipSuccess) return e;
  if (events && (e = hipEventRecord((hipEvent_t)events[1], s)) != hipSuccess) return e;
  const size_t smem = (size_t)g.R * 16 + kWaves * kRowsPerWave * 4 + kWaves * (kRowsPerWave + 1) * 4;
  bin_scatter_csr_kernel<<<(unsigned)g.ntiles, kThreads, smem, s>>>(
      row_ptr, col_idx, vals, n, (int32_t)nnz, d, B, key, row_offset, g.bp_shift, g.R, g.ntiles,
      c.hist, (uint32_t)nnz, c.items, c.hmax);
  bin_reduce_csr_kernel<<<(unsigned)g.R, kThreads, g.lds_bytes, s>>>(
      c.items, c.hist, c.hmax, g.ntiles, g.R, (uint32_t)nnz, B, d, g.bp_shift, SX);
  return hipGetLastError();
}

hipError_t launch_sx_binned_dense(const float* X, int64_t ldx, int64_t n, int d, uint32_t B,
                                  Key key, uint64_t row_offset, float* SX, void* scratch,
                                  hipStream_t s, void* const* events) {
  const BinGeom g = bin_geometry(false, n, d, B);
  Carve c = carve(scratch, g, n);
  const int64_t hl = (int64_t)g.R * g.ntiles;
  bin_count_kernel<false><<<(unsigned)g.ntiles, kThreads, g.R * 4, s>>>(
      nullptr, n, 0, B, key, row_offset, g.bp_shift, g.R, g.ntiles, c.hist);
  hipError_t e = launch_exclusive_scan(c.hist, hl, c.sums, s);
  if (e != hipSuccess) return e;
  if (events && (e = hipEventRecord((hipEvent_t)events[1], s)) != hipSuccess) return e;
  bin_scatter_dense_kernel<<<(unsigned)g.ntiles, kThreads, (size_t)g.R * 12, s>>>(
      n, B, key, row_offset, g.bp_shift, g.R, g.ntiles, c.hist, (uint32_t)n, c.items);
  const unsigned gr = (unsigned)g.R;
  switch (lanes_per_row(d)) {
    case 1: bin_reduce_dense_kernel<1><<<gr, kThreads, g.lds_bytes, s>>>(X, ldx, n, c.items, c.hist, g.ntiles, g.R, (uint32_t)n, B, d, g.bp_shift, SX); break;
    case 2: bin_reduce_dense_kernel<2><<<gr, kThreads, g.lds_bytes, s>>>(X, ldx, n, c.items, c.hist, g.ntiles, g.R, (uint32_t)n, B, d, g.bp_shift, SX); break;
    case 4: bin_reduce_dense_kernel<4><<<gr, kThreads, g.lds_bytes, s>>>(X, ldx, n, c.items, c.hist, g.ntiles, g.R, (uint32_t)n, B, d, g.bp_shift, SX); break;
    case 8: bin_reduce_dense_kernel<8><<<gr, kThreads, g.lds_bytes, s>>>(X, ldx, n, c.items, c.hist, g.ntiles, g.R, (uint32_t)n, B, d, g.bp_shift, SX); break;
    case 16: bin_reduce_dense_kernel<16><<<gr, kThreads, g.lds_bytes, s>>>(X, ldx, n, c.items, c.hist, g.ntiles, g.R, (uint32_t)n, B, d, g.bp_shift, SX); break;
    case 32: bin_reduce_dense_kernel<32><<<gr, kThreads, g.lds_bytes, s>>>(X, ldx, n, c.items, c.hist, g.ntiles, g.R, (uint32_t)n, B, d, g.bp_shift, SX); break;
    default: bin_reduce_dense_kernel<64><<<gr, kThreads, g.lds_bytes, s>>>(X, ldx, n, c.items, c.hist, g.ntiles, g.R, (uint32_t)n, B, d, g.bp_shift, SX); break;
  }
  return hipGetLastError();
}

}  // namespace cg
