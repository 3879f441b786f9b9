// Deterministic S X: group the contributions by bucket with a stable
// counting (LSD radix) sort, then let one wavefront sum each bucket in a
// fixed order.  The same input gives the same bits on every run, unlike the
// atomic path whose FP32 summation order depends on timing.
//
// Dense X: the items are rows (key = h(r), payload = r | sign << 31); the
// reduction walks a bucket's rows in increasing row order, lanes across
// columns.
// CSR X: the items are stored entries (key = h(row), payload = column and
// sigma(row) * value); stability keeps each bucket's entries in row-major
// order; lane l of the bucket's wavefront sums entries l, l + S, l + 2S, ...
// into its own LDS row, and the S rows are then added in slot order.
//
// Radix sort: 8-bit digits, tiles of 2048 items per workgroup.  Per pass:
// per-tile digit histograms, one exclusive scan over (digit, tile), and a
// scatter in which each item's rank among equal digits of its tile comes
// from wavefront ballots -- items are visited in index order, so equal
// keys keep their input order.
#include <algorithm>

#include "cg_internal.hpp"
#include "cg_rng.hpp"

namespace cg {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = 4;
constexpr int kTile = 2048;
constexpr int kScanChunk = 4096;
constexpr int kSlotBytes = 16384;  // LDS accumulator bytes per wavefront (CSR reduce)
constexpr int64_t kBucketsPerLaunch = 1 << 24;   // per-bucket reduce launches: 2^30 work-items

template <typename T>
struct Entry {
  int32_t col;
  T v;
};

// ---------------------------------------------------------------- items
__global__ __launch_bounds__(kThreads) void init_rows_kernel(int64_t n, uint32_t B, Key key,
                                                             uint64_t row_offset,
                                                             uint32_t* __restrict__ keys,
                                                             uint32_t* __restrict__ pay) {
  const int64_t r = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * 4;
  if (r >= n) return;
  uint32_t hv[4];
  hash4(row_offset + (uint64_t)r, B, key.k0, key.k1, hv);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (r + t < n) {
      keys[r + t] = hash_bucket(hv[t]);
      pay[r + t] = (uint32_t)(r + t) | (hv[t] & 0x80000000u);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void init_entries_kernel(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const T* __restrict__ vals, int64_t n, int32_t nnz, uint32_t B, Key key, uint64_t row_offset,
    uint32_t* __restrict__ keys, Entry<T>* __restrict__ pay) {
  __shared__ uint32_t s_hash[kWaves][kRowsPerWave];
  __shared__ int32_t s_ptr[kWaves][kRowsPerWave + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * kWaves + wave) * kRowsPerWave;
  const int nr = r0 < n ? (int)min((int64_t)kRowsPerWave, n - r0) : 0;
  uint32_t* sh = s_hash[wave];
  int32_t* sp = s_ptr[wave];
  if (nr > 0) {
    uint32_t hv[4];
    hash4(row_offset + (uint64_t)r0 + 4 * (uint64_t)lane, B, key.k0, key.k1, hv);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (4 * lane + t < nr) sh[4 * lane + t] = hv[t];
    for (int i = lane; i <= nr; i += 64) sp[i] = min(max(row_ptr[r0 + i], 0), nnz);
  }
  __syncthreads();
  if (nr == 0) return;
  const int32_t kb = sp[0], ke = sp[nr];
  for (int32_t base = kb; base < ke; base += 64) {
    const int32_t k = base + lane;
    if (k < ke) {
      int lo = 0;
#pragma unroll
      for (int step = kRowsPerWave / 2; step > 0; step >>= 1)
        if (lo + step < nr && sp[lo + step] <= k) lo += step;
      const uint32_t hp = sh[lo];
      const T v = vals[k];
      keys[k] = hash_bucket(hp);
      pay[k] = Entry<T>{col_idx[k], hash_negative(hp) ? -v : v};
    }
  }
}

// ---------------------------------------------------------------- scan
// Exclusive scan of 256 per-thread values within the block (Hillis-Steele
// over LDS).  Returns the thread's exclusive prefix; *total gets the sum.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s, uint32_t* total) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    const uint32_t add = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  const uint32_t incl = s[t];
  *total = s[kThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kThreads) void scan_sums_kernel(const uint32_t* __restrict__ a,
                                                             int64_t len,
                                                             uint32_t* __restrict__ sums) {
  __shared__ uint32_t s[kThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t v = 0;
  for (int i = threadIdx.x; i < kScanChunk; i += kThreads) {
    const int64_t k = base + i;
    if (k < len) v += a[k];
  }
  uint32_t total;
  block_exclusive_scan(v, s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void scan_top_kernel(uint32_t* __restrict__ sums,
                                                            int64_t nsums) {
  __shared__ uint32_t s[kThreads];
  uint32_t carry = 0;
  for (int64_t base = 0; base < nsums; base += kThreads) {
    const int64_t k = base + threadIdx.x;
    const uint32_t v = k < nsums ? sums[k] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, s, &total);
    if (k < nsums) sums[k] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(kThreads) void scan_apply_kernel(uint32_t* __restrict__ a, int64_t len,
                                                              const uint32_t* __restrict__ sums) {
  __shared__ uint32_t s[kThreads];
  constexpr int per = kScanChunk / kThreads;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * per;
  uint32_t v[per];
  uint32_t tot = 0;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    v[i] = base + i < len ? a[base + i] : 0u;
    tot += v[i];
  }
  uint32_t total;
  uint32_t run = sums[blockIdx.x] + block_exclusive_scan(tot, s, &total);
#pragma unroll
  for (int i = 0; i < per; ++i) {
    if (base + i < len) a[base + i] = run;
    run += v[i];
  }
}

// ---------------------------------------------------------------- radix
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                              int64_t count, int shift,
                                                              int64_t ntiles,
                                                              uint32_t* __restrict__ ghist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int i = threadIdx.x; i < kTile; i += kThreads) {
    const int64_t k = base + i;
    if (k < count) atomicAdd(&h[(keys[k] >> shift) & 255u], 1u);
  }
  __syncthreads();
  ghist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

template <typename P>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const P* __restrict__ pin, uint32_t* __restrict__ kout,
    P* __restrict__ pout, int64_t count, int shift, int64_t ntiles,
    const uint32_t* __restrict__ gofs) {
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_wcnt[kWaves][256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  s_base[tid] = gofs[(int64_t)tid * ntiles + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s_wcnt[w][tid] = 0;
  __syncthreads();
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t tbase = (int64_t)blockIdx.x * kTile;
  for (int round = 0; round < kTile / kThreads; ++round) {
    const int64_t idx = tbase + round * kThreads + tid;
    const bool valid = idx < count;
    uint32_t key = 0;
    P pay{};
    int dg = 0;
    if (valid) {
      key = kin[idx];
      pay = pin[idx];
      dg = (int)((key >> shift) & 255u);
    }
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool b = (dg >> bit) & 1;
      const uint64_t m1 = __ballot(b);
      same &= b ? m1 : ~m1;
    }
    const int wrank = __popcll(same & below);
    if (valid && wrank == 0) s_wcnt[wave][dg] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = s_base[dg] + (uint32_t)wrank;
      for (int w = 0; w < wave; ++w) pos += s_wcnt[w][dg];
      kout[pos] = key;
      pout[pos] = pay;
    }
    __syncthreads();
    s_base[tid] += s_wcnt[0][tid] + s_wcnt[1][tid] + s_wcnt[2][tid] + s_wcnt[3][tid];
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s_wcnt[w][tid] = 0;
    __syncthreads();
  }
}

// off[b] = first index of bucket b in the sorted keys, off[B] = count: one
// thread per bucket (grid-stride), each a binary search for the first key
// at or above b, so the work per thread is O(log count) however many
// buckets lie between two keys.
__global__ __launch_bounds__(kThreads) void bucket_offsets_kernel(const uint32_t* __restrict__ keys,
                                                                  int64_t count, uint32_t B,
                                                                  int32_t* __restrict__ off) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x; b <= (int64_t)B; b += stride) {
    int64_t lo = 0, hi = count;
    if (b == (int64_t)B) {
      lo = count;
    } else {
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        // keys are < B whenever the input is well formed; clamped anyway
        // (a malformed CSR), which keeps them sorted
        if (min((int64_t)keys[mid], (int64_t)B - 1) < b)
          lo = mid + 1;
        else
          hi = mid;
      }
    }
    off[b] = (int32_t)lo;
  }
}

// ---------------------------------------------------------------- reduce
template <typename T, int LPR>
__global__ __launch_bounds__(kThreads) void reduce_rows_kernel(const T* __restrict__ X, int64_t ldx,
                                                               const int32_t* __restrict__ off,
                                                               const uint32_t* __restrict__ rows,
                                                               int32_t count, uint32_t B, int d,
                                                               T* __restrict__ SX, int64_t b_base) {
  constexpr int RPP = 64 / LPR;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t b = b_base + (int64_t)blockIdx.x * kWaves + wave;
  if (b >= B) return;
  const int32_t s = min(max(off[b], 0), count), e = min(max(off[b + 1], s), count);
  const int sub = lane / LPR, c = lane % LPR;
  const bool cok = c < d;
  T acc = T(0);
  int32_t i = s + sub;
  for (; i + 3 * RPP < e; i += 4 * RPP) {
    uint32_t pv[4];
    T x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) pv[u] = rows[i + u * RPP];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = cok ? X[(int64_t)(pv[u] & 0x7fffffffu) * ldx + c] : T(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += (pv[u] >> 31) ? -x[u] : x[u];
  }
  for (; i < e; i += RPP) {
    const uint32_t pv = rows[i];
    const T x = cok ? X[(int64_t)(pv & 0x7fffffffu) * ldx + c] : T(0);
    acc += (pv >> 31) ? -x : x;
  }
  // add the RPP row phases of each column in a fixed order
#pragma unroll
  for (int k = LPR; k < 64; k <<= 1) acc += __shfl_down(acc, k, 64);
  if (sub == 0 && cok) SX[b * d + c] = acc;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void reduce_rows_wide_kernel(
    const T* __restrict__ X, int64_t ldx, const int32_t* __restrict__ off,
    const uint32_t* __restrict__ rows, int32_t count, uint32_t B, int d, T* __restrict__ SX,
    int64_t b_base) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t b = b_base + (int64_t)blockIdx.x * kWaves + wave;
  if (b >= B) return;
  const int32_t s = min(max(off[b], 0), count), e = min(max(off[b + 1], s), count);
  for (int c = lane; c < d; c += 64) {
    T acc = T(0);
    for (int32_t i = s; i < e; ++i) {
      const uint32_t pv = rows[i];
      const T x = X[(int64_t)(pv & 0x7fffffffu) * ldx + c];
      acc += (pv >> 31) ? -x : x;
    }
    SX[b * d + c] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void reduce_entries_kernel(const int32_t* __restrict__ off,
                                                                  const Entry<T>* __restrict__ pay,
                                                                  int32_t count, uint32_t B, int d,
                                                                  int slots, int stride,
                                                                  T* __restrict__ SX,
                                                                  int64_t b_base) {
  __shared__ T s_acc[kWaves][kSlotBytes / sizeof(T)];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t b = b_base + (int64_t)blockIdx.x * kWaves + wave;
  T* acc = s_acc[wave];
  const bool live = b < B;
  if (live)
    for (int i = lane; i < slots * stride; i += 64) acc[i] = T(0);
  __syncthreads();
  if (live && lane < slots) {
    const int32_t s = min(max(off[b], 0), count), e = min(max(off[b + 1], s), count);
    T* mine = acc + lane * stride;
    for (int32_t i = s + lane; i < e; i += slots) {
      const Entry<T> en = pay[i];
      if ((unsigned)en.col < (unsigned)d) mine[en.col] += en.v;
    }
  }
  __syncthreads();
  if (live) {
    for (int c = lane; c < d; c += 64) {
      T sum = T(0);
      for (int sl = 0; sl < slots; ++sl) sum += acc[sl * stride + c];
      SX[b * d + c] = sum;
    }
  }
}

// ---------------------------------------------------------------- driver
struct Scratch {
  uint32_t *kA, *kB;
  void *pA, *pB;
  uint32_t *hist, *sums;
  int32_t* off;
  int64_t ntiles, hlen, nsums;
};

Scratch carve(void* base, int64_t count, int64_t B, size_t psize) {
  Scratch s;
  char* p = (char*)base;
  s.ntiles = (count + kTile - 1) / kTile;
  if (s.ntiles < 1) s.ntiles = 1;
  s.hlen = 256 * s.ntiles;
  s.nsums = (s.hlen + kScanChunk - 1) / kScanChunk;
  auto take = [&](size_t bytes) {
    void* r = p;
    p += align256(bytes);
    return r;
  };
  s.kA = (uint32_t*)take((size_t)count * 4);
  s.kB = (uint32_t*)take((size_t)count * 4);
  s.pA = take((size_t)count * psize);
  s.pB = take((size_t)count * psize);
  s.hist = (uint32_t*)take((size_t)s.hlen * 4);
  s.sums = (uint32_t*)take((size_t)s.nsums * 4);
  s.off = (int32_t*)take((size_t)(B + 1) * 4);
  return s;
}

size_t scratch_bytes(int64_t count, int64_t B, size_t psize) {
  int64_t ntiles = (count + kTile - 1) / kTile;
  if (ntiles < 1) ntiles = 1;
  const int64_t hlen = 256 * ntiles;
  const int64_t nsums = (hlen + kScanChunk - 1) / kScanChunk;
  return 2 * align256((size_t)count * 4) + 2 * align256((size_t)count * psize) +
         align256((size_t)hlen * 4) + align256((size_t)nsums * 4) + align256((size_t)(B + 1) * 4);
}

int key_bits(uint32_t B) {
  int bits = 1;
  while (bits < 31 && ((uint64_t)1 << bits) < B) ++bits;
  return bits;
}

// Sort (keys, payloads) stably by key; the sorted result ends in (kA, pA).
template <typename P>
hipError_t radix_sort(Scratch& s, int64_t count, uint32_t B, hipStream_t st) {
  const int passes = (key_bits(B) + 7) / 8;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = 8 * ps;
    radix_hist_kernel<<<(unsigned)s.ntiles, kThreads, 0, st>>>(s.kA, count, shift, s.ntiles,
                                                               s.hist);
    scan_sums_kernel<<<(unsigned)s.nsums, kThreads, 0, st>>>(s.hist, s.hlen, s.sums);
    scan_top_kernel<<<1, kThreads, 0, st>>>(s.sums, s.nsums);
    scan_apply_kernel<<<(unsigned)s.nsums, kThreads, 0, st>>>(s.hist, s.hlen, s.sums);
    radix_scatter_kernel<P><<<(unsigned)s.ntiles, kThreads, 0, st>>>(
        s.kA, (const P*)s.pA, s.kB, (P*)s.pB, count, shift, s.ntiles, s.hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* tk = s.kA;
    s.kA = s.kB;
    s.kB = tk;
    void* tp = s.pA;
    s.pA = s.pB;
    s.pB = tp;
  }
  bucket_offsets_kernel<<<(unsigned)std::min<int64_t>(((int64_t)B + kThreads) / kThreads, 8192),
                          kThreads, 0, st>>>(s.kA, count, B, s.off);
  return hipGetLastError();
}

}  // namespace

int64_t scan_sums_len(int64_t len) { return (len + kScanChunk - 1) / kScanChunk; }

hipError_t launch_exclusive_scan(uint32_t* a, int64_t len, uint32_t* sums, hipStream_t st) {
  if (len <= 0) return hipSuccess;
  const int64_t ns = scan_sums_len(len);
  scan_sums_kernel<<<(unsigned)ns, kThreads, 0, st>>>(a, len, sums);
  scan_top_kernel<<<1, kThreads, 0, st>>>(sums, ns);
  scan_apply_kernel<<<(unsigned)ns, kThreads, 0, st>>>(a, len, sums);
  return hipGetLastError();
}

size_t sorted_scratch_bytes(int64_t count, int64_t B, size_t payload) {
  return scratch_bytes(count, B, payload);
}

template <typename T>
hipError_t launch_sx_dense_sorted(const T* X, int64_t ldx, int64_t n, int d, uint32_t B, Key key,
                                  uint64_t row_offset, T* SX, void* scratch, hipStream_t st) {
  Scratch s = carve(scratch, n, B, 4);
  const int64_t threads = (n + 3) / 4;
  init_rows_kernel<<<(unsigned)((threads + kThreads - 1) / kThreads), kThreads, 0, st>>>(
      n, B, key, row_offset, s.kA, (uint32_t*)s.pA);
  hipError_t e = radix_sort<uint32_t>(s, n, B, st);
  if (e != hipSuccess) return e;
  const uint32_t* rows = (const uint32_t*)s.pA;
  // one wavefront per bucket, in launches of at most kBucketsPerLaunch
  // buckets (a grid holds fewer than 2^32 work-items)
  for (int64_t b0 = 0; b0 < (int64_t)B; b0 += kBucketsPerLaunch) {
    const unsigned g = (unsigned)((std::min<int64_t>(kBucketsPerLaunch, (int64_t)B - b0) + kWaves - 1) / kWaves);
    if (d <= 8)
      reduce_rows_kernel<T, 8><<<g, kThreads, 0, st>>>(X, ldx, s.off, rows, (int32_t)n, B, d, SX, b0);
    else if (d <= 16)
      reduce_rows_kernel<T, 16><<<g, kThreads, 0, st>>>(X, ldx, s.off, rows, (int32_t)n, B, d, SX,
                                                            b0);
    else if (d <= 32)
      reduce_rows_kernel<T, 32><<<g, kThreads, 0, st>>>(X, ldx, s.off, rows, (int32_t)n, B, d, SX,
                                                            b0);
    else if (d <= 64)
      reduce_rows_kernel<T, 64><<<g, kThreads, 0, st>>>(X, ldx, s.off, rows, (int32_t)n, B, d, SX,
                                                            b0);
    else
      reduce_rows_wide_kernel<T><<<g, kThreads, 0, st>>>(X, ldx, s.off, rows, (int32_t)n, B, d,
                                                           SX, b0);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sx_csr_sorted(const int32_t* row_ptr, const int32_t* col_idx, const T* vals,
                                int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                                uint64_t row_offset, T* SX, void* scratch, hipStream_t st) {
  Scratch s = carve(scratch, nnz, B, sizeof(Entry<T>));
  const unsigned gr = (unsigned)((n + (int64_t)kWaves * kRowsPerWave - 1) /
                                 ((int64_t)kWaves * kRowsPerWave));
  init_entries_kernel<T><<<gr, kThreads, 0, st>>>(row_ptr, col_idx, vals, n, (int32_t)nnz, B, key,
                                                  row_offset, s.kA, (Entry<T>*)s.pA);
  hipError_t e = radix_sort<Entry<T>>(s, nnz, B, st);
  if (e != hipSuccess) return e;
  const int stride = d | 1;   // odd row stride: lanes' slot rows fall in different banks
  int slots = (int)(kSlotBytes / sizeof(T)) / stride;
  if (slots > 64) slots = 64;
  for (int64_t b0 = 0; b0 < (int64_t)B; b0 += kBucketsPerLaunch) {
    const unsigned g = (unsigned)((std::min<int64_t>(kBucketsPerLaunch, (int64_t)B - b0) + kWaves - 1) / kWaves);
    reduce_entries_kernel<T><<<g, kThreads, 0, st>>>(s.off, (const Entry<T>*)s.pA, (int32_t)nnz, B,
                                                     d, slots, stride, SX, b0);
  }
  return hipGetLastError();
}

template hipError_t launch_sx_dense_sorted<float>(const float*, int64_t, int64_t, int, uint32_t,
                                                  Key, uint64_t, float*, void*, hipStream_t);
template hipError_t launch_sx_dense_sorted<double>(const double*, int64_t, int64_t, int, uint32_t,
                                                   Key, uint64_t, double*, void*, hipStream_t);
template hipError_t launch_sx_csr_sorted<float>(const int32_t*, const int32_t*, const float*,
                                                int64_t, int64_t, int, uint32_t, Key, uint64_t,
                                                float*, void*, hipStream_t);
template hipError_t launch_sx_csr_sorted<double>(const int32_t*, const int32_t*, const double*,
                                                 int64_t, int64_t, int, uint32_t, Key, uint64_t,
                                                 double*, void*, hipStream_t);

}  // namespace cg
