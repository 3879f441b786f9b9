// S X by bucket-range binning with LDS accumulation (FP32 data).
//
// Device-scope float atomics are resolved far from the CUs on this GPU and
// cost one memory-side read-modify-write each, and float atomics in LDS are
// several times slower than integer ones.  So S X (Section 1.1: every
// stored entry (r, c, v) adds sigma(r) v to SX[h(r)][c]) is computed in
// two passes over the data without any floating-point atomic:
//
//  1. split: the buckets are cut into R ranges of Bp = 2^k consecutive
//     buckets whose S X slice fits in LDS.  bin_count counts every row
//     tile's items per range; bin_scan turns each range's per-tile counts
//     into offsets inside the range and the range's total; the range
//     bases are prefix sums of the totals, which each consumer forms
//     itself.  That gives every tile a private window in each range's item
//     list, which bin_scatter_* fills.  A scatter workgroup takes its tile
//     in rounds of 1024 rows: it counts the round's items per range, places
//     them in LDS grouped by range, and writes each range's run with
//     consecutive lanes on consecutive addresses.
//  2. reduce: one workgroup per range accumulates its items in LDS and
//     writes the slice; every bucket of S X is written exactly once, so no
//     zero fill is needed.
//
// Global loads are lane-contiguous everywhere: a wavefront reads the
// row_ptr values of its rows as one coalesced block (each lane loads its own
// row starts with one 8- or 16-byte load), and a scatter round reads its whole
// col_idx/vals segment in 16-byte pieces, consecutive lanes on consecutive
// entries, and finds each entry's row afterwards.  (Lanes reading their own
// rows straight from memory touch dozens of cache lines per load
// instruction and starve the address units.)
//
// CSR items are (cell = local bucket * d + column, sigma v).  They are
// summed as 64-bit fixed-point integers with ds_add_u64: the range's scale
// 2^f is chosen from the largest |v| in the range and the item count so
// that no partial sum can overflow, and integer addition does not depend
// on order -- the result is bitwise reproducible run to run.  Each v 2^f is
// split into its nearest integer q and a remainder r, |r| <= 1/2.  Most
// data has r = 0 everywhere (v 2^f is an integer whenever |v| >= 2^(23-f)),
// and then the q sums are exact; a cell whose q sum is at least 2^24 has
// lost at most 1/2 per remainder, relatively no more than an FP32 sum of
// its values would.  Only a range with a cell that received a nonzero
// remainder and whose |q sum| is below 2^24 (a cell of values far below
// the range's largest: another column, another bucket) is read a second
// time, summing the remainders at the finer scale 2^(f + 62 - lg)
// (lg = ceil(log2 count)) into the same LDS while each thread holds its
// cells' q sums in registers, so every cell keeps FP32 precision for values
// down to about max|v| 2^-(100 - 2 lg).  A range that
// holds a NaN or infinity is summed with float atomics instead (same
// propagation as the atomic path).
//
// Dense items are (row | sign << 31, local bucket).  The reduce sorts a
// range's items by bucket in LDS (counting sort); each lane group (the
// lanes of one row, 16 bytes each where rows are 16-byte aligned) then
// owns a contiguous block of buckets, streams their rows -- eight loads in
// flight -- summing in registers, and adds a bucket's sum into the LDS
// slice when the bucket changes (no other group touches those cells, so no
// atomics).
//
// Malformed CSR input (decreasing row_ptr, row_ptr outside [0, nnz],
// columns >= d) never causes an out-of-bounds access: row starts are
// clamped, windows are bounded, columns out of range contribute nothing.
// The result is then unspecified.
#include <algorithm>

#include "cg_internal.hpp"
#include "cg_rng.hpp"

namespace cg {

namespace {

constexpr int kThreads = 1024;                 // reduce kernels
constexpr int kWaves = kThreads / 64;
constexpr int kSThreads = 256;                 // scan and scatter kernels
constexpr int kSWaves = kSThreads / 64;
constexpr int kRPT = 4;                        // scatter: rows per thread per round
constexpr int kWaveRows = kRPT * 64;           // rows per wavefront per round
constexpr int kRoundRows = kRPT * kSThreads;   // rows per workgroup round
constexpr int kTileRows = 16384;               // rows per split tile
constexpr int kInCap = 2048;                   // CSR entries per chunk
constexpr int kEPT = kInCap / kSThreads;       // entries per thread of a chunk
constexpr int kRpWin = kWaveRows + 4;          // LDS words of one row_ptr window
// LDS target of a scatter workgroup: CSR 40 KiB (4 per CU), dense 26 KiB (6 per CU)
constexpr size_t kScatterLdsCsr = 40 * 1024;
constexpr size_t kScatterLdsDense = 26 * 1024;
constexpr int kMinStage = 1024;                // smallest output stage (items)
constexpr int kSparseRound = 512;              // CSR rounds with at most this many entries skip the stage
constexpr int kWalkLen = 2;                    // sparse rounds: rows up to this long are walked by their lane
constexpr int kDenseCap = 8192;                // items sorted per dense reduce pass
constexpr int kCsrMaxCells = 8192;             // cells of a CSR range's S X slice (64 KB of int64)
constexpr int kDenseMaxBlocks = 128;           // 128-bucket blocks of a dense range (16384 / 128)

static_assert(kTileRows % kRoundRows == 0, "tiles hold whole rounds");
static_assert(kEPT % 4 == 0, "an entry-parallel chunk is whole 16-byte groups per thread");
static_assert(kRPT == 2 || kRPT == 4, "rows per thread: 2 or 4");
static_assert(kMinStage >= kRoundRows, "a sparse round keeps one record per row in the stage");
constexpr int kCRPT = 4;                       // count kernel: rows per thread per round
constexpr int kCntThreads = 512;               // count kernel: threads per workgroup
constexpr int kCntWaves = kCntThreads / 64;
constexpr int kCntRoundRows = kCRPT * kCntThreads;
constexpr int kCRoundRows = kCRPT * kSThreads;
constexpr int kCRpWin = 64 * kCRPT + 4;
static_assert(kTileRows % kCRoundRows == 0, "tiles hold whole count rounds");

extern __shared__ __align__(16) unsigned char dyn_lds[];

// Orders LDS accesses of the lanes of one wavefront (their LDS operations
// execute in program order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------- wavefront scans
// Inclusive scans over the 64 lanes of a wavefront on DPP lane moves (no
// LDS round trip): shifts by 1, 2, 4 and 8 lanes inside each row of 16,
// then rows 1 and 3 take lane 15 of the row before and rows 2 and 3 take
// lane 31.  A lane without a source keeps `old`, the operation's identity.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138, kDppBcast15 = 0x142, kDppBcast31 = 0x143;

__device__ __forceinline__ uint32_t wave_incl_add(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr1, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr2, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr4, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr8, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppBcast15, 0xa, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppBcast31, 0xc, 0xf, false);
  return x;
}

__device__ __forceinline__ int32_t wave_incl_max(int32_t x) {
  constexpr int32_t lo = INT32_MIN;
  x = max(x, __builtin_amdgcn_update_dpp(lo, x, kDppRowShr1, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(lo, x, kDppRowShr2, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(lo, x, kDppRowShr4, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(lo, x, kDppRowShr8, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(lo, x, kDppBcast15, 0xa, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(lo, x, kDppBcast31, 0xc, 0xf, false));
  return x;
}

// The value of lane l - 1 (lane 0 gets `first`) and of lane l + 1 (lane 63
// gets `last`).
__device__ __forceinline__ int32_t from_lane_below(int32_t x, int32_t first) {
  return __builtin_amdgcn_update_dpp(first, x, kDppWaveShr1, 0xf, 0xf, false);
}
__device__ __forceinline__ int32_t from_lane_above(int32_t x, int32_t last) {
  return __builtin_amdgcn_update_dpp(last, x, kDppWaveShl1, 0xf, 0xf, false);
}

// Exclusive scan over the NT threads of the block; *total gets the sum.
// Every wavefront reads all wavefront totals, so two barriers suffice; the
// second frees s_w for the next call, and a caller whose next write of s_w
// comes after another barrier anyway leaves it out (FREE = false).
template <int NT, bool FREE = true>
__device__ uint32_t block_exscan(uint32_t v, uint32_t* s_w, uint32_t* total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t x = wave_incl_add(v);
  if (lane == 63) s_w[wave] = x;
  __syncthreads();
  uint32_t before = 0u, all = 0u;
#pragma unroll
  for (int w2 = 0; w2 < NW; ++w2) {
    const uint32_t t = s_w[w2];
    before += w2 < wave ? t : 0u;
    all += t;
  }
  *total = all;
  if (FREE) __syncthreads();
  return before + x - v;
}

// ------------------------------------------------------------------ row_ptr
// Row starts of the wavefront's 64 RPT rows from r0; lane l gets those of
// its rows r0 + RPT l + j (j = 0 .. RPT) -- rows at or past t1 come out
// empty (their starts are clamped to row_ptr[t1]).
//  direct: row_ptr is aligned and all the wavefront's rows lie before t1:
//       one 4 RPT-byte load per lane (its own starts), the last start from
//       the next lane.
//  otherwise: lane-contiguous 4-byte loads handed over through the
//       wavefront's LDS window (64 RPT + 4 words).
template <int RPT>
struct RpLoad {
  int32_t v[RPT];
  int32_t last;
  bool direct;
};

template <int RPT, bool NT = true>
__device__ __forceinline__ RpLoad<RPT> load_row_ptr(const int32_t* __restrict__ row_ptr, int64_t r0,
                                                    int64_t t1, bool aligned) {
  static_assert(RPT == 2 || RPT == 4, "2 or 4 rows per lane");
  const int lane = threadIdx.x & 63;
  RpLoad<RPT> l;
  // readfirstlane: the choice is uniform, so the compiler keeps two paths
  // instead of merging their loads into 4-byte ones
  l.direct = __builtin_amdgcn_readfirstlane((int)(aligned && r0 + 64 * RPT <= t1)) != 0;
  if (l.direct) {
    typedef int32_t vNi __attribute__((ext_vector_type(RPT)));
    const vNi* src = (const vNi*)(row_ptr + r0 + RPT * lane);
    const vNi q = NT ? __builtin_nontemporal_load(src) : *src;
#pragma unroll
    for (int j = 0; j < RPT; ++j) l.v[j] = q[j];
  } else {
#pragma unroll
    for (int j = 0; j < RPT; ++j) l.v[j] = row_ptr[min(r0 + lane + 64 * j, t1)];
  }
  l.last = row_ptr[min(r0 + 64 * RPT, t1)];
  return l;
}

// Values are clamped to [0, nnz] and made non-decreasing, so row lengths
// are never negative.
template <int RPT>
__device__ __forceinline__ void transpose_row_ptr(const RpLoad<RPT>& l, int32_t* w, int32_t nnz,
                                                  int32_t rp[RPT + 1]) {
  const int lane = threadIdx.x & 63;
  if (l.direct) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) rp[j] = l.v[j];
    rp[RPT] = from_lane_above(l.v[0], l.last);
  } else {
#pragma unroll
    for (int j = 0; j < RPT; ++j) w[lane + 64 * j] = l.v[j];
    if (lane == 0) w[64 * RPT] = l.last;
    wave_sync();
#pragma unroll
    for (int j = 0; j <= RPT; ++j) rp[j] = w[RPT * lane + j];
    wave_sync();
  }
#pragma unroll
  for (int j = 0; j <= RPT; ++j) rp[j] = min(max(rp[j], 0), nnz);
#pragma unroll
  for (int j = 1; j <= RPT; ++j) rp[j] = max(rp[j], rp[j - 1]);
}

// Packed hashes of this lane's RPT rows r .. r + RPT - 1 (zero past t1).
template <int RPT>
__device__ __forceinline__ void lane_hashes(int64_t r, int64_t t1, uint64_t row_offset, uint32_t B,
                                            Key key, uint32_t hv[RPT]) {
  if constexpr (RPT == 2) {
    // the lane pair (2i, 2i + 1) shares the Philox block(s) of its four rows;
    // the odd lane takes the upper two words (rows at or past t1 are empty
    // and their hashes unused)
    const int odd = threadIdx.x & 1;
    const int64_t rq = r - 2 * odd;
    uint32_t h4[4] = {0u, 0u, 0u, 0u};
    if (rq < t1) hash4(row_offset + (uint64_t)rq, B, key.k0, key.k1, h4);
    hv[0] = odd ? h4[2] : h4[0];
    hv[1] = odd ? h4[3] : h4[1];
    return;
  }
#pragma unroll
  for (int g = 0; g < RPT; g += 4) {
    uint32_t h4[4] = {0u, 0u, 0u, 0u};
    if (r + g < t1) hash4(row_offset + (uint64_t)(r + g), B, key.k0, key.k1, h4);
#pragma unroll
    for (int t = 0; t < 4 && g + t < RPT; ++t) hv[g + t] = h4[t];
  }
}

// ------------------------------------------------------------------ count
// hist[p * ntiles + t] = items of tile t that fall in range p.  Two rounds
// per iteration, so each wavefront has both rounds' row_ptr loads in flight
// while it hashes their rows.
template <bool CSR>
__device__ __forceinline__ void count_tile(const BinArgs& a, int64_t tile) {
  const int32_t* __restrict__ row_ptr = a.row_ptr;
  const int64_t n = a.n;
  const int32_t nnz = a.nnz;
  const uint32_t B = a.B;
  const Key key = a.key;
  const uint64_t row_offset = a.row_offset;
  const int bp_shift = a.bp_shift, R = a.R;
  uint32_t* s_cnt = (uint32_t*)dyn_lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int32_t* w = (int32_t*)(s_cnt + R) + wave * 2 * kCRpWin;
  for (int i = threadIdx.x; i < R; i += kCntThreads) s_cnt[i] = 0;
  __syncthreads();
  const int64_t t0 = tile * a.tile_rows;
  const int64_t t1 = min(t0 + a.tile_rows, n);
  const bool vec = ((uintptr_t)row_ptr & 15) == 0;
  for (int64_t round = t0; round < t1; round += 2 * kCntRoundRows) {
    const int64_t ra = round + (int64_t)64 * kCRPT * wave, rb = ra + kCntRoundRows;
    RpLoad<kCRPT> la, lb;
    if (CSR) {
      la = load_row_ptr<kCRPT>(row_ptr, ra, t1, vec);
      lb = load_row_ptr<kCRPT>(row_ptr, rb, t1, vec);
    }
    uint32_t ha[kCRPT], hb[kCRPT];
    lane_hashes<kCRPT>(ra + kCRPT * lane, t1, row_offset, B, key, ha);
    lane_hashes<kCRPT>(rb + kCRPT * lane, t1, row_offset, B, key, hb);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int64_t r = (half ? rb : ra) + kCRPT * lane;
      const uint32_t* hv = half ? hb : ha;
      int32_t rp[kCRPT + 1];
      if (CSR) transpose_row_ptr<kCRPT>(half ? lb : la, w + half * kCRpWin, nnz, rp);
#pragma unroll
      for (int j = 0; j < kCRPT; ++j) {
        const uint32_t len = CSR ? (uint32_t)(rp[j + 1] - rp[j]) : (r + j < t1 ? 1u : 0u);
        if (len) atomicAdd(&s_cnt[hash_bucket(hv[j]) >> bp_shift], len);
      }
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < R; p += kCntThreads) a.hist[(int64_t)p * a.ntiles + tile] = s_cnt[p];
}

// The tile a workgroup takes, so that consecutive tiles run on one XCD:
// workgroups go to the eight XCDs in turn (workgroup b to XCD b % 8), and
// XCD x's j-th workgroup takes tile start(x) + j, the XCDs holding
// contiguous runs of tiles.  Tile t's and tile t + 1's item windows of a
// range are adjacent, so the line they share is then completed in one L2
// instead of being written partly from two (and the per-tile counts and
// maxima of a range, adjacent words, likewise).  A bijection for any count.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t ntiles) {
  const int64_t q = ntiles / 8, r = ntiles % 8, x = b % 8, j = b / 8;
  return x * q + (x < r ? x : r) + j;
}

template <bool CSR>
__global__ __launch_bounds__(kCntThreads) void bin_count_kernel(BinArgs a) {
  count_tile<CSR>(a, xcd_tile(blockIdx.x, a.ntiles));
}

// ------------------------------------------------------------------ scan
// Workgroup p: hist[p][0 .. ntiles) becomes its exclusive prefix sums and
// tot[p] the range's item count.
__device__ __forceinline__ void scan_range(const BinArgs& a, int p) {
  __shared__ uint32_t s_w[kSWaves];
  const int64_t ntiles = a.ntiles;
  uint32_t* h = a.hist + (int64_t)p * ntiles;
  uint32_t carry = 0;
  for (int64_t c0 = 0; c0 < ntiles; c0 += 4 * kSThreads) {
    const int64_t i = c0 + 4 * (int64_t)threadIdx.x;
    uint32_t v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = h[min(i + j, ntiles - 1)];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (i + j >= ntiles) v[j] = 0u;
    uint32_t all;
    uint32_t run = carry + block_exscan<kSThreads>(v[0] + v[1] + v[2] + v[3], s_w, &all);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (i + j < ntiles) h[i + j] = run;
      run += v[j];
    }
    carry += all;
  }
  if (threadIdx.x == 0) a.tot[p] = carry;
}

__global__ __launch_bounds__(kSThreads) void bin_scan_kernel(BinArgs a) { scan_range(a, blockIdx.x); }

// ------------------------------------------------------------------ scatter
// LDS of the scatter kernels:
//   stage (cap items) | input chunk (kInCap items) sharing its space with
//   the row_ptr windows and the entry-parallel row arrays and marks (CSR
//   only) | per-range arrays (8 R words) | block scan | segment bounds
struct ScatterLds {
  uint2* stage;
  uint2* in;
  int32_t* rpw;     // kSWaves windows of kRpWin words, aliasing `in`
  // entry-parallel chunks (CSR, aliasing `in`): per row of the round its
  // packed hash and slot base (one 8-byte record), and the row marks of a
  // chunk's entries
  uint2* row_hs;    // kRoundRows
  int32_t* marks;   // kInCap
  uint32_t *g_base, *g_run, *r_cnt, *r_off, *r_fill, *r_max;   // R each
  uint2* fl;        // R: (window slot of stage index 0, window end)
  uint32_t* s_w;    // kSWaves
  int32_t* s_seg;   // 8 words: [1] the round's end as the last lane finds it (the rest unused)
};

__host__ __device__ inline size_t scatter_shared_bytes(bool csr) {
  const size_t in = (size_t)kInCap * 8, win = (size_t)kSWaves * kRpWin * 4;
  const size_t rows = (size_t)2 * kRoundRows * 4 + (size_t)kInCap * 4;
  return csr ? std::max(std::max(in, win), rows) : 0;
}

static_assert((size_t)kSWaves * kRpWin * 4 <= (size_t)2 * kRoundRows * 4,
              "row_ptr windows stay clear of the marks");

__host__ __device__ inline size_t scatter_fixed_bytes(int R, bool csr) {
  return scatter_shared_bytes(csr) + (size_t)8 * R * 4 + kSWaves * 4 + 32;
}

__host__ __device__ constexpr size_t scatter_lds_target(bool csr) {
  return csr ? kScatterLdsCsr : kScatterLdsDense;
}

// Items a scatter round may stage: what the LDS target leaves after the
// fixed arrays, at least kMinStage.
__host__ __device__ inline int stage_cap(int R, bool csr) {
  const int64_t left = (int64_t)scatter_lds_target(csr) - (int64_t)scatter_fixed_bytes(R, csr);
  const int cap = (int)((left > 0 ? left : 0) / 8) & ~63;
  return cap < kMinStage ? kMinStage : cap;
}

__host__ __device__ inline size_t scatter_lds_bytes(int R, bool csr) {
  return (size_t)stage_cap(R, csr) * 8 + scatter_fixed_bytes(R, csr);
}

__device__ __forceinline__ ScatterLds carve_scatter(int R, bool csr) {
  ScatterLds L;
  unsigned char* p = dyn_lds;
  L.stage = (uint2*)p;
  p += (size_t)stage_cap(R, csr) * 8;
  L.in = (uint2*)p;
  L.rpw = (int32_t*)p;
  L.row_hs = (uint2*)p;
  L.marks = (int32_t*)(L.row_hs + kRoundRows);
  p += scatter_shared_bytes(csr);
  uint32_t* q = (uint32_t*)p;
  L.g_base = q;
  L.g_run = q + R;
  L.r_cnt = q + 2 * R;
  L.r_off = q + 3 * R;
  L.r_fill = q + 4 * R;
  L.r_max = q + 5 * R;
  L.fl = (uint2*)(q + 6 * R);
  L.s_w = q + 8 * R;
  L.s_seg = (int32_t*)(L.s_w + kSWaves);
  return L;
}

// This tile's window [g_base, fl.y) in every range's item list: range
// bases are the prefix sums of the range totals, plus the tile's offset
// inside the range (never past the item buffer, even if a malformed CSR
// made the counts exceed nnz).  Also clears the per-range round state.
// (All of a thread's loads -- its ranges' totals and this tile's offsets in
// them -- are issued before the scan over the totals.)
__device__ __forceinline__ void load_windows(const ScatterLds& L, const uint32_t* __restrict__ offs,
                                             const uint32_t* __restrict__ tot, int R,
                                             int64_t ntiles, uint32_t total, int64_t t) {
  constexpr int kMaxR = kBinMaxRangesCsr > kBinMaxRangesDense ? kBinMaxRangesCsr : kBinMaxRangesDense;
  constexpr int kMaxPer = (kMaxR + kSThreads - 1) / kSThreads;
  const int per = (R + kSThreads - 1) / kSThreads;   // <= kMaxPer: bin_geometry bounds R
  const int b = (int)threadIdx.x * per;
  uint32_t tp[kMaxPer], lo[kMaxPer], hi[kMaxPer];
  uint32_t local = 0;
#pragma unroll
  for (int k = 0; k < kMaxPer; ++k) {
    const int p = b + k;
    tp[k] = lo[k] = hi[k] = 0u;
    if (k < per && p < R) {
      tp[k] = tot[p];
      lo[k] = offs[(int64_t)p * ntiles + t];
      hi[k] = t + 1 < ntiles ? offs[(int64_t)p * ntiles + t + 1] : tp[k];
    }
    local += tp[k];
  }
  uint32_t all;
  uint64_t base = block_exscan<kSThreads>(local, L.s_w, &all);
#pragma unroll
  for (int k = 0; k < kMaxPer; ++k) {
    const int p = b + k;
    if (k < per && p < R) {
      L.g_base[p] = (uint32_t)min(base + lo[k], (uint64_t)total);
      L.fl[p] = make_uint2(0u, (uint32_t)min(base + hi[k], (uint64_t)total));
      L.g_run[p] = 0;
      L.r_cnt[p] = 0;
      L.r_fill[p] = 0;
      L.r_max[p] = 0;
    }
    base += tp[k];
  }
}

// Exclusive offsets of the round's per-range counts (each thread scans
// ceil(R / kSThreads) consecutive ranges); returns the total.  The scan's
// s_w is next written after this function's closing barrier.
__device__ __forceinline__ uint32_t round_offsets(const ScatterLds& L, int R) {
  const int per = (R + kSThreads - 1) / kSThreads;
  const int b = (int)threadIdx.x * per;
  uint32_t local = 0;
  for (int k = 0; k < per; ++k)
    if (b + k < R) local += L.r_cnt[b + k];
  uint32_t E;
  uint32_t run = block_exscan<kSThreads, false>(local, L.s_w, &E);
  for (int k = 0; k < per; ++k) {
    const int p = b + k;
    if (p < R) {
      L.r_off[p] = run;
      L.fl[p].x = L.g_base[p] + L.g_run[p] - run;
      run += L.r_cnt[p];
    }
  }
  __syncthreads();
  return E;
}

// Write the round's staged items (grouped by range in stage[0 .. E)) to
// their windows -- consecutive lanes on consecutive slots of a run -- and
// advance each range's write cursor.  `swap` puts the stage's second word
// first (dense items).  No barrier between the two parts: after the
// staging barrier nothing reads the round's counts or cursors again, the
// stores read only the stage and fl, and the next round's first barrier
// orders both parts before any reuse.
__device__ __forceinline__ void flush_stage(const ScatterLds& L, int R, uint32_t E, bool swap,
                                            uint2* __restrict__ items) {
  for (uint32_t i = threadIdx.x; i < E; i += kSThreads) {
    const uint2 it = L.stage[i];
    const uint32_t p = it.x >> 16;
    if (p >= (uint32_t)R) continue;   // a slot no item filled (malformed CSR)
    const uint2 f = L.fl[p];
    const uint32_t pos = i + f.x;
    if (pos < f.y)
      items[pos] = swap ? make_uint2(it.y, it.x & 0xffffu) : make_uint2(it.x & 0xffffu, it.y);
  }
  for (int p = threadIdx.x; p < R; p += kSThreads) {
    L.g_run[p] += L.r_cnt[p];
    L.r_cnt[p] = 0;
    L.r_fill[p] = 0;
  }
}

// kEPT consecutive entries from k (a multiple of 4, 16-byte aligned
// arrays) with 16-byte loads.  A group of four starting past `lim` (the
// last group the chunk needs; lim + 4 <= nnz) reloads group `lim` instead:
// same cache line as a neighbour's load, so nothing past the chunk is
// fetched, and its entries are never used.  Non-temporal: X is read once
// here, and streaming it past the caches keeps the item list this kernel
// writes in the last-level cache for the reduce that reads it next.
__device__ __forceinline__ void load_entries(const int32_t* __restrict__ col_idx,
                                             const float* __restrict__ vals, int32_t k, int32_t lim,
                                             int32_t cc[kEPT], float vv[kEPT]) {
  typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
  typedef float f32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int u = 0; u < kEPT; u += 4) {
    const int32_t g = min(k + u, lim);
    const i32x4 c = __builtin_nontemporal_load((const i32x4*)(col_idx + g));
    const f32x4 v = __builtin_nontemporal_load((const f32x4*)(vals + g));
    cc[u] = c.x;
    cc[u + 1] = c.y;
    cc[u + 2] = c.z;
    cc[u + 3] = c.w;
    vv[u] = v.x;
    vv[u + 1] = v.y;
    vv[u + 2] = v.z;
    vv[u + 3] = v.w;
  }
}

// CSR.  A round is 1024 rows, four consecutive rows per lane.  The lanes
// count their rows' entries per range and reserve slots per row; the
// round's entries -- one contiguous segment of col_idx/vals -- are then
// taken in chunks of kInCap, kEPT consecutive entries per thread, and
// staged by range.  Without 16-byte alignment (or at the arrays' end) a
// chunk is copied into LDS instead and every lane walks its own rows'
// entries there.
__device__ __forceinline__ void scatter_csr_tile(const BinArgs& a, int64_t tile) {
  const int32_t* __restrict__ row_ptr = a.row_ptr;
  const int32_t* __restrict__ col_idx = a.col_idx;
  const float* __restrict__ vals = a.vals;
  const int64_t n = a.n;
  const int32_t nnz = a.nnz;
  const int d = a.d;
  const uint32_t B = a.B;
  const Key key = a.key;
  const uint64_t row_offset = a.row_offset;
  const int bp_shift = a.bp_shift, R = a.R;
  uint2* __restrict__ items = a.items;
  const ScatterLds L = carve_scatter(R, true);
  const uint32_t cap = (uint32_t)stage_cap(R, true);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int32_t* w = L.rpw + wave * kRpWin;
  load_windows(L, a.hist, a.tot, R, a.ntiles, (uint32_t)nnz, tile);
  // no marks yet (the first round's barrier orders this before any use)
#pragma unroll
  for (int u = 0; u < kEPT; u += 4)
    *(int4*)(L.marks + kEPT * threadIdx.x + u) = make_int4(-1, -1, -1, -1);
  const uint32_t bmask = (1u << bp_shift) - 1u;
  const int64_t t0 = tile * a.tile_rows;
  const int64_t t1 = min(t0 + a.tile_rows, n);
  const bool vec = ((uintptr_t)row_ptr & 15) == 0;
  // 16-byte loads of the entries: chunks then start at multiples of 4
  const bool vecx = (((uintptr_t)col_idx | (uintptr_t)vals) & 15) == 0;
  // Software pipeline: a round's row starts are loaded during the round
  // before, and its first chunk of entries is requested before the count
  // and offset scans, so neither load's latency is waited out on its own.
  RpLoad<kRPT> rl_next = load_row_ptr<kRPT>(row_ptr, t0 + (int64_t)kWaveRows * wave, t1, vec);
  // Every wavefront carries the round's bounds itself -- row_ptr at the
  // round's first row, and at its end, loaded a round ahead (uniform loads)
  // -- so all of them take the same sparse-or-not decision without LDS.
  int32_t start_raw = row_ptr[t0];
  int32_t end_next = row_ptr[min(t0 + kRoundRows, t1)];
  // the first round waits for load_windows' state and the marks
  bool after_dense = true;
  for (int64_t round = t0; round < t1; round += kRoundRows) {
    const int64_t r0 = round + (int64_t)kWaveRows * wave;
    const RpLoad<kRPT> rl = rl_next;
    rl_next = load_row_ptr<kRPT>(row_ptr, r0 + kRoundRows, t1, vec);   // clamped to t1 at the end
    const int32_t end_raw = end_next;
    end_next = row_ptr[min(round + 2 * kRoundRows, t1)];
    uint32_t hv[kRPT];
    lane_hashes<kRPT>(r0 + kRPT * lane, t1, row_offset, B, key, hv);
    // the round's first entry (as transpose_row_ptr clamps the first row
    // start) and its end (as the last lane finds it, for well-formed row_ptr)
    const int32_t S0 = min(max(start_raw, 0), nnz);
    const int32_t S1e = max(min(max(end_raw, 0), nnz), S0);
    start_raw = end_raw;
    const bool sparse = S1e - S0 <= kSparseRound;
    // Sparse rounds share nothing in LDS between wavefronts but the range
    // cursors and maxima (atomics), so a wavefront goes from one to the next
    // without waiting; a dense round, and the round after one, waits until
    // every wavefront is done with the LDS state before it.
    if (!sparse || after_dense) __syncthreads();
    after_dense = !sparse;
    if (sparse) {
      // A sparse round: no counts, scans, stage or flush.  Each lane
      // reserves its rows' slots with one LDS atomic per nonempty row, and
      // every entry is stored straight to its range's window.  The order of
      // items inside a range does not change the fixed-point sums.  Only
      // wavefront-private LDS is written besides the range cursors and
      // maxima (atomics); the barrier after the tile's last round orders
      // those before the maxima are written out.
      int32_t rp[kRPT + 1];
      transpose_row_ptr<kRPT>(rl, w, nnz, rp);
      int32_t lmax = 0;
#pragma unroll
      for (int j = 0; j < kRPT; ++j) lmax = max(lmax, rp[j + 1] - rp[j]);
      if (__builtin_amdgcn_readlane(wave_incl_max(lmax), 63) <= kWalkLen) {
        // Short rows only: each lane takes its own rows' entries (at most
        // kWalkLen per row), all loads issued before the slot reservations.
        int32_t cc[kRPT][kWalkLen];
        float vv[kRPT][kWalkLen];
#pragma unroll
        for (int j = 0; j < kRPT; ++j)
#pragma unroll
          for (int e = 0; e < kWalkLen; ++e) {
            cc[j][e] = 0;
            vv[j][e] = 0.0f;
            if (rp[j] + e < rp[j + 1]) {
              cc[j][e] = col_idx[rp[j] + e];
              vv[j][e] = vals[rp[j] + e];
            }
          }
#pragma unroll
        for (int j = 0; j < kRPT; ++j) {
          const uint32_t len = (uint32_t)(rp[j + 1] - rp[j]);
          if (!len) continue;
          const uint32_t bucket = hash_bucket(hv[j]);
          const uint32_t pr = bucket >> bp_shift;
          const uint32_t s0 = L.g_base[pr] + atomicAdd(&L.g_run[pr], len);
          const uint32_t wend = L.fl[pr].y;
          const bool neg = hash_negative(hv[j]);
          uint32_t mb = 0u;
#pragma unroll
          for (int e = 0; e < kWalkLen; ++e) {
            if ((uint32_t)e < len) {
              const bool ok = (uint32_t)cc[j][e] < (uint32_t)d;
              const uint32_t cell = ok ? (bucket & bmask) * (uint32_t)d + (uint32_t)cc[j][e] : 0u;
              const float sv = ok ? (neg ? -vv[j][e] : vv[j][e]) : 0.0f;
              mb = max(mb, __float_as_uint(fabsf(sv)));
              if (s0 + e < wend) items[s0 + e] = make_uint2(cell, __float_as_uint(sv));
            }
          }
          atomicMax(&L.r_max[pr], mb);
        }
        continue;
      }
      // Longer rows: a record per row (packed hash, slot of entry 0) in the
      // wavefront's part of the stage and the row starts in its row_ptr
      // window; the wavefront's entries -- one contiguous segment -- are
      // taken 64 at a time, each finding its row by binary search over the
      // starts, so a long row is spread over the lanes.
      uint2* rec = L.stage + wave * kWaveRows;
#pragma unroll
      for (int j = 0; j < kRPT; ++j) {
        const uint32_t len = (uint32_t)(rp[j + 1] - rp[j]);
        const uint32_t pr = hash_bucket(hv[j]) >> bp_shift;
        const uint32_t s0 = len ? L.g_base[pr] + atomicAdd(&L.g_run[pr], len) : 0u;
        rec[kRPT * lane + j] = make_uint2(hv[j], s0 - (uint32_t)rp[j]);
        w[kRPT * lane + j] = rp[j];
      }
      const int32_t first = __builtin_amdgcn_readfirstlane(rp[0]);
      const int32_t last = __builtin_amdgcn_readlane(rp[kRPT], 63);
      wave_sync();
      for (int32_t k = first + lane; k < last; k += 64) {
        // the last of the wavefront's rows that starts at or before k
        int lo = 0, hi = kWaveRows - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (w[mid] <= k) lo = mid;
          else hi = mid - 1;
        }
        const uint2 r = rec[lo];
        const uint32_t bucket = hash_bucket(r.x);
        const uint32_t pr = bucket >> bp_shift;
        const uint32_t c = (uint32_t)col_idx[k];
        const float v = vals[k];
        const bool ok = c < (uint32_t)d;
        const uint32_t cell = ok ? (bucket & bmask) * (uint32_t)d + c : 0u;
        const float sv = ok ? (hash_negative(r.x) ? -v : v) : 0.0f;
        const uint32_t slot = r.y + (uint32_t)k;
        atomicMax(&L.r_max[pr], __float_as_uint(fabsf(sv)));
        if (slot < L.fl[pr].y) items[slot] = make_uint2(cell, __float_as_uint(sv));
      }
      wave_sync();
      continue;
    }
    const int32_t A = vecx ? (S0 & ~3) : S0;
    // the first chunk's 16-byte loads (uniform; the chunk loop uses them
    // for its first chunk, which takes the vector path exactly when `pre`)
    const int32_t lim0 = (min(A + kInCap, S1e) - 1) & ~3;
    const bool pre = vecx && S1e > A && lim0 + 4 <= nnz;
    int32_t cc0[kEPT];
    float vv0[kEPT];
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
      cc0[u] = 0;
      vv0[u] = 0.f;
    }
    if (pre) load_entries(col_idx, vals, A + kEPT * (int32_t)threadIdx.x, lim0, cc0, vv0);
    int32_t rp[kRPT + 1];
    transpose_row_ptr<kRPT>(rl, w, nnz, rp);
    uint32_t len[kRPT];
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      len[j] = (uint32_t)(rp[j + 1] - rp[j]);   // zero for rows at or past t1
      if (len[j]) atomicAdd(&L.r_cnt[hash_bucket(hv[j]) >> bp_shift], len[j]);
    }
    if (threadIdx.x == kSThreads - 1) L.s_seg[1] = rp[kRPT];
    // the first chunk's row marks (when it takes the vector path); the
    // barriers of the count and offset scans order them before their reads
    if (pre) {
#pragma unroll
      for (int j = 0; j < kRPT; ++j)
        if (len[j] && rp[j] >= A && rp[j] < A + kInCap) L.marks[rp[j] - A] = kRPT * (int32_t)threadIdx.x + j;
    }
    __syncthreads();
    const uint32_t E = round_offsets(L, R);
    const bool staged = E <= cap;
    // slot of entry k of row j: sadj[j] + k (mod 2^32)
    uint32_t sadj[kRPT], maxb[kRPT];
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const uint32_t p = hash_bucket(hv[j]) >> bp_shift;
      const uint32_t b = len[j] ? atomicAdd(&L.r_fill[p], len[j]) : 0u;
      const uint32_t s0 = staged ? L.r_off[p] + b : L.g_base[p] + L.g_run[p] + b;
      sadj[j] = s0 - (uint32_t)rp[j];
      maxb[j] = 0u;
    }
    const int32_t S1 = max(L.s_seg[1], S0);
    // the round's row hashes and slot bases, for the entry-parallel chunks
    // (the barrier at the first chunk orders them before their readers)
    static_assert(kRPT % 2 == 0, "row records are written two per 16-byte store");
#pragma unroll
    for (int j = 0; j < kRPT; j += 2)
      *(uint4*)&L.row_hs[kRPT * threadIdx.x + j] = make_uint4(hv[j], sadj[j], hv[j + 1], sadj[j + 1]);
    int32_t carry = -1;   // row of the entry just before the chunk
    for (int32_t c0 = A; c0 < S1; c0 = (int32_t)min((int64_t)c0 + kInCap, (int64_t)S1)) {
      const int32_t c1 = (int32_t)min((int64_t)c0 + kInCap, (int64_t)S1);
      if (c0 != A) __syncthreads();   // every lane is done with the previous chunk
      const int32_t lim = (c1 - 1) & ~3;
      if (c0 == A ? pre : vecx && lim + 4 <= nnz) {
        // a chunk whose 16-byte groups lie inside the arrays (uniform over
        // the workgroup): thread t takes entries c0 + kEPT t + (0 .. kEPT - 1),
        // loaded with unguarded (clamped) 16-byte loads.  An entry's row is found without a
        // search: each row owner marks the position of its row's first entry
        // (marks[] is all -1 otherwise), and a max-scan over the marks in
        // entry order gives every entry the last row started at or before it.
        const int32_t g = c0 + kEPT * (int32_t)threadIdx.x;
        int32_t cc[kEPT];
        float vv[kEPT];
#pragma unroll
        for (int u = 0; u < kEPT; ++u) {
          cc[u] = cc0[u];
          vv[u] = vv0[u];
        }
        if (c0 != A) {   // a later chunk: its marks (the first chunk's are written)
          load_entries(col_idx, vals, g, lim, cc, vv);
#pragma unroll
          for (int j = 0; j < kRPT; ++j)
            if (len[j] && rp[j] >= c0 && rp[j] < c0 + kInCap)
              L.marks[rp[j] - c0] = kRPT * (int32_t)threadIdx.x + j;
          __syncthreads();
        }
        int32_t mk[kEPT];
#pragma unroll
        for (int u = 0; u < kEPT; u += 4) {
          const int4 m = *(const int4*)(L.marks + kEPT * threadIdx.x + u);
          *(int4*)(L.marks + kEPT * threadIdx.x + u) = make_int4(-1, -1, -1, -1);   // clean for the next chunk
          mk[u] = m.x;
          mk[u + 1] = m.y;
          mk[u + 2] = m.z;
          mk[u + 3] = m.w;
        }
#pragma unroll
        for (int u = 1; u < kEPT; ++u) mk[u] = max(mk[u], mk[u - 1]);
        // inclusive max-scan of the threads' last marks over the wavefront ...
        const int32_t incl = wave_incl_max(mk[kEPT - 1]);
        int32_t before = from_lane_below(incl, -1);
        // ... and over the wavefronts before this one (and the chunk before)
        if (lane == 63) L.s_w[wave] = (uint32_t)incl;
        __syncthreads();
        int32_t wcarry = carry, bmax = carry;
#pragma unroll
        for (int w2 = 0; w2 < kSWaves; ++w2) {
          const int32_t t = (int32_t)L.s_w[w2];
          if (w2 < wave) wcarry = max(wcarry, t);
          bmax = max(bmax, t);
        }
        carry = bmax;
        before = max(before, wcarry);
#pragma unroll
        for (int i = 0; i < kEPT; ++i) {
          const int32_t k = g + i;
          // (a mark left by a copied chunk -- only with decreasing row_ptr --
          // is not a row index: bounded here)
          const int32_t row = max(mk[i], before);
          if (k < S0 || k >= S1 || (uint32_t)row >= (uint32_t)kRoundRows) continue;
          const uint2 rhs = L.row_hs[row];
          const uint32_t hj = rhs.x, sj = rhs.y;
          const uint32_t bucket = hash_bucket(hj);
          const uint32_t pr = bucket >> bp_shift;
          const bool ok = (uint32_t)cc[i] < (uint32_t)d;
          const uint32_t cell = ok ? (bucket & bmask) * (uint32_t)d + (uint32_t)cc[i] : 0u;
          const float sv = ok ? (hash_negative(hj) ? -vv[i] : vv[i]) : 0.0f;
          const uint32_t slot = sj + (uint32_t)k;
          if (pr < (uint32_t)R) atomicMax(&L.r_max[pr], __float_as_uint(fabsf(sv)));
          if (staged) {
            if (slot < E) L.stage[slot] = make_uint2((pr << 16) | cell, __float_as_uint(sv));
          } else if (pr < (uint32_t)R) {
            if (slot < L.fl[pr].y) items[slot] = make_uint2(cell, __float_as_uint(sv));
          }
        }
        continue;
      }
      {
        int32_t cc[kInCap / kSThreads];
        float vv[kInCap / kSThreads];
#pragma unroll
        for (int u = 0; u < kInCap / kSThreads; ++u) {
          const int32_t k = min(c0 + (int32_t)threadIdx.x + u * kSThreads, c1 - 1);
          cc[u] = col_idx[k];
          vv[u] = vals[k];
        }
#pragma unroll
        for (int u = 0; u < kInCap / kSThreads; ++u) {
          const int32_t i = (int32_t)threadIdx.x + u * kSThreads;
          if (i < c1 - c0) L.in[i] = make_uint2((uint32_t)cc[u], __float_as_uint(vv[u]));
        }
      }
      __syncthreads();
      // entries staged in LDS; every lane walks its own rows' entries
      const int32_t a = max(rp[0], c0), e = min(rp[kRPT], c1);
      for (int32_t k = a; k < e; ++k) {
        int j = 0;
#pragma unroll
        for (int q = 1; q < kRPT; ++q) j += k >= rp[q];
        uint32_t hj = hv[0], sj = sadj[0];
#pragma unroll
        for (int q = 1; q < kRPT; ++q)
          if (j == q) {
            hj = hv[q];
            sj = sadj[q];
          }
        const uint2 in = L.in[k - c0];
        const uint32_t bucket = hash_bucket(hj);
        const uint32_t p = bucket >> bp_shift;
        const bool ok = in.x < (uint32_t)d;
        const float v = __uint_as_float(in.y);
        const uint32_t cell = ok ? (bucket & bmask) * (uint32_t)d + in.x : 0u;
        const float sv = ok ? (hash_negative(hj) ? -v : v) : 0.0f;
        const uint32_t slot = sj + (uint32_t)k;
        const uint32_t mb = __float_as_uint(fabsf(sv));
#pragma unroll
        for (int q = 0; q < kRPT; ++q)
          if (j == q) maxb[q] = max(maxb[q], mb);
        if (staged) {
          if (slot < E) L.stage[slot] = make_uint2((p << 16) | cell, __float_as_uint(sv));
        } else {
          // a round too large for the stage (long rows): direct stores
          if (slot < L.fl[p].y) items[slot] = make_uint2(cell, __float_as_uint(sv));
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kRPT; ++j)
      if (len[j]) atomicMax(&L.r_max[hash_bucket(hv[j]) >> bp_shift], maxb[j]);
    __syncthreads();
    flush_stage(L, R, staged ? E : 0u, false, items);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < R; q += kSThreads) a.hmax[(int64_t)q * a.ntiles + tile] = L.r_max[q];
}

// four workgroups per CU (the LDS target's occupancy): at most 128 VGPRs
__global__ __launch_bounds__(kSThreads, 4) void bin_scatter_csr_kernel(BinArgs a) {
  scatter_csr_tile(a, xcd_tile(blockIdx.x, a.ntiles));
}

// Dense.  A round is 1024 rows, four per lane, one item per row (rounds
// twice the CSR size: the per-round scan over the ranges costs as much as
// the round's rows here).
__device__ __forceinline__ void scatter_dense_tile(const BinArgs& a, int64_t tile) {
  const int64_t n = a.n;
  const uint32_t B = a.B;
  const Key key = a.key;
  const uint64_t row_offset = a.row_offset;
  const int bp_shift = a.bp_shift, R = a.R;
  uint2* __restrict__ items = a.items;
  const ScatterLds L = carve_scatter(R, false);
  load_windows(L, a.hist, a.tot, R, a.ntiles, (uint32_t)n, tile);
  const uint32_t bmask = (1u << bp_shift) - 1u;
  const int64_t t0 = tile * a.tile_rows;
  const int64_t t1 = min(t0 + a.tile_rows, n);
  for (int64_t round = t0; round < t1; round += kCRoundRows) {
    const int64_t r = round + (int64_t)kCRPT * threadIdx.x;
    uint32_t hv[kCRPT];
    lane_hashes<kCRPT>(r, t1, row_offset, B, key, hv);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kCRPT; ++j)
      if (r + j < t1) atomicAdd(&L.r_cnt[hash_bucket(hv[j]) >> bp_shift], 1u);
    __syncthreads();
    const uint32_t E = round_offsets(L, R);   // <= kCRoundRows <= stage capacity
#pragma unroll
    for (int j = 0; j < kCRPT; ++j) {
      if (r + j < t1) {
        const uint32_t bucket = hash_bucket(hv[j]);
        const uint32_t p = bucket >> bp_shift;
        const uint32_t slot = atomicAdd(&L.r_fill[p], 1u);
        if (slot < L.r_cnt[p] && L.r_off[p] + slot < E)
          L.stage[L.r_off[p] + slot] = make_uint2(
              (p << 16) | (bucket & bmask), (uint32_t)(r + j) | (hv[j] & 0x80000000u));
      }
    }
    __syncthreads();
    flush_stage(L, R, E, true, items);
  }
}

__global__ __launch_bounds__(kSThreads) void bin_scatter_dense_kernel(BinArgs a) {
  scatter_dense_tile(a, xcd_tile(blockIdx.x, a.ntiles));
}

// ------------------------------------------------------------------ reduce
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* s_red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t r = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) r += s_red[w];
  __syncthreads();
  return r;
}

// CSR range p: the largest |value| bits over its tiles (hm: hmax row p)
// and its items [sum of tot[0 .. p), + tot[p]), clamped to the buffer.
// All loads are issued first and both values reduced in one barrier round
// (the barrier also orders LDS writes made before the call); s_red and
// s_red64 are not reused after it.
__device__ __forceinline__ void csr_range_prologue(const uint32_t* __restrict__ tot,
                                                   const uint32_t* __restrict__ hm, int64_t ntiles,
                                                   int p, uint32_t total, uint32_t* s_red,
                                                   uint64_t* s_red64, uint32_t* amax,
                                                   uint32_t* start, uint32_t* end) {
  uint32_t mx = 0;
  uint64_t s = 0;
  for (int64_t t = threadIdx.x; t < ntiles; t += kThreads) mx = max(mx, hm[t]);
  for (int q = threadIdx.x; q < p; q += kThreads) s += tot[q];
  const uint32_t tp = tot[p];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = max(mx, (uint32_t)__shfl_xor(mx, off, 64));
    s += __shfl_xor(s, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_red[threadIdx.x >> 6] = mx;
    s_red64[threadIdx.x >> 6] = s;
  }
  __syncthreads();
  uint32_t r = 0;
  uint64_t S = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    r = max(r, s_red[w]);
    S += s_red64[w];
  }
  *amax = r;
  *start = (uint32_t)min(S, (uint64_t)total);
  *end = (uint32_t)min(max(S + tp, (uint64_t)*start), (uint64_t)total);
}

// Items of range p: [sum of tot[0 .. p), + tot[p]), clamped to the buffer.
__device__ __forceinline__ void range_of(const uint32_t* __restrict__ tot, int p, uint32_t total,
                                         uint64_t* s_red, uint32_t* start, uint32_t* end) {
  uint64_t s = 0;
  for (int q = threadIdx.x; q < p; q += kThreads) s += tot[q];
  s = block_sum_u64(s, s_red);
  const uint64_t e = s + tot[p];
  *start = (uint32_t)min(s, (uint64_t)total);
  *end = (uint32_t)min(max(e, (uint64_t)*start), (uint64_t)total);
}

// Most cells of one CSR range per thread (cells taken thread-strided).
constexpr int kCsrCellsPerThread = kCsrMaxCells / kThreads;
static_assert(kCsrMaxCells % kThreads == 0, "whole cells per thread");

// Calls op(item) for every item [start, end) of a range: two at a time
// (16-byte loads from an even index; the item buffer is 256-byte aligned),
// an odd first / last item on its own.
template <typename Op>
__device__ __forceinline__ void for_range_items(const uint2* __restrict__ items, uint32_t start,
                                                uint32_t end, Op&& op) {
  const uint32_t e0 = min((start + 1) & ~1u, end), e1 = max(end & ~1u, e0);
  if (threadIdx.x == 0 && start < e0) op(items[start]);
  if (threadIdx.x == 0 && e1 < end) op(items[e1]);
  const uint4* __restrict__ pairs = (const uint4*)(items + e0);
  const uint32_t np = (e1 - e0) / 2;
  constexpr int UR = 4;
  uint32_t i = threadIdx.x;
  for (; i + (UR - 1) * kThreads < np; i += UR * kThreads) {
    uint4 q[UR];
#pragma unroll
    for (int u = 0; u < UR; ++u) q[u] = pairs[i + u * kThreads];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      op(make_uint2(q[u].x, q[u].y));
      op(make_uint2(q[u].z, q[u].w));
    }
  }
  for (; i < np; i += kThreads) {
    const uint4 q = pairs[i];
    op(make_uint2(q.x, q.y));
    op(make_uint2(q.z, q.w));
  }
}

// FP8 scales of the contraction from a range's finished S X slice: one pair
// (2^-e, 2^(e - 6)) per 128-bucket block, e the smallest integer with
// amax <= 448 2^e (at least -100), the same rule as the contraction's own
// scale kernel.  Ranges hold whole blocks (2^bp_shift >= 128 buckets, which
// bin_geometry gives whenever d <= 64); `value(c)` is cell c's FP32 value.
// A block spans 128 d cells, a multiple of 64, and the cells are taken
// thread-strided by a multiple of 64, so the 64 cells a wavefront holds at
// each step lie in one block: each wavefront keeps its running maximum per
// block and adds it with one LDS atomic when its block changes (one atomic
// per cell, on a handful of words, serialises badly).
template <typename F>
__device__ __forceinline__ void emit_fp8_scales(const BinArgs& a, int p, int cells, F&& value,
                                                uint32_t* s_amax) {
  static_assert(kThreads % 64 == 0, "whole wavefronts");
  const int d = a.d, nblk = (1 << a.bp_shift) / 128;
  for (int i = threadIdx.x; i < nblk; i += kThreads) s_amax[i] = 0u;
  __syncthreads();
  // NaNs are skipped; |v| >= 0, so the unsigned order of the bits is the
  // float order
  uint32_t run = 0u;
  int cur = -1;
  auto flush = [&]() {
    for (int off = 32; off > 0; off >>= 1) run = max(run, (uint32_t)__shfl_xor((int)run, off, 64));
    if ((threadIdx.x & 63) == 0 && cur >= 0 && run) atomicMax(&s_amax[cur], run);
  };
  for (int c = threadIdx.x; c < cells; c += kThreads) {
    const int blk = (c / d) >> 7;   // the same in every lane of the wavefront
    if (blk != cur) {
      flush();
      cur = blk;
      run = 0u;
    }
    const float v = fabsf(value(c));
    if (v == v) run = max(run, __float_as_uint(v));
  }
  flush();
  __syncthreads();
  for (int i = threadIdx.x; i < nblk; i += kThreads) {
    const int64_t blk = (((int64_t)p << a.bp_shift) >> 7) + i;
    if (blk * 128 < (int64_t)a.B) {
      const float amax = __uint_as_float(s_amax[i]);
      int e = 0;
      if (amax > 0.0f) {
        int E;
        const float f = frexpf(amax, &E);
        e = f <= 0.875f ? E - 9 : E - 8;   // 448 = 0.875 * 2^9
      }
      e = max(e, -100);
      a.fp8_scale[blk] = make_float2(ldexpf(1.0f, -e), ldexpf(1.0f, e - 6));
    }
  }
}

// FUSED: the range's S X slice goes to `slice` in LDS (float, cells
// thread-strided as in s_acc, zero past B) instead of to a.SX, for the
// fused contraction that follows.  EMIT: a.fp8_scale is set, and the
// range's FP8 block scales are written too (a separate instance, so that
// the other launches carry none of that code or its registers).
template <bool FUSED = false, bool EMIT = false>
__device__ __forceinline__ void reduce_csr_range(const BinArgs& a, int p, float* slice = nullptr) {
  const uint2* __restrict__ items = a.items;
  const uint32_t* __restrict__ tot = a.tot;
  const uint32_t* __restrict__ hmax = a.hmax;
  const int64_t ntiles = a.ntiles;
  const uint32_t total = (uint32_t)a.nnz, B = a.B;
  const int d = a.d, bp_shift = a.bp_shift;
  float* __restrict__ SX = a.SX;
  unsigned long long* s_acc = (unsigned long long*)dyn_lds;
  __shared__ uint32_t s_red[kWaves];
  __shared__ uint64_t s_red64[kWaves];
  __shared__ int s_resid;
  __shared__ uint32_t s_rbits[kCsrMaxCells / 32];   // cells that received a nonzero remainder
  const int cells = (1 << bp_shift) * d;
  for (int i = threadIdx.x; i < cells; i += kThreads) s_acc[i] = 0ull;
  for (int i = threadIdx.x; i < kCsrMaxCells / 32; i += kThreads) s_rbits[i] = 0u;
  if (threadIdx.x == 0) s_resid = 0;
  uint32_t amax_bits, start, end;   // (the prologue's barrier also orders the zero fill)
  csr_range_prologue(tot, hmax + (int64_t)p * ntiles, ntiles, p, total, s_red, s_red64, &amax_bits,
                     &start, &end);
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
      if constexpr (FUSED)
        slice[i] = bucket < B ? acc[i] : 0.0f;
      else if (bucket < B)
        SX[bucket * d + i % d] = acc[i];
    }
    if constexpr (EMIT && !FUSED) {
      if (a.fp8_scale)
        emit_fp8_scales(a, p, cells, [&](int c) {
          const int64_t bucket = ((int64_t)p << bp_shift) + c / d;
          return bucket < B ? acc[c] : 0.0f;
        }, s_rbits);
    }
    return;
  }
  // |partial q sums| <= count (amax 2^f + 1/2) < 2^62 with amax < 2^E,
  // count <= 2^lg; |partial remainder sums| <= count 2^(g - 1) <= 2^61
  int E = 0;
  if (amax_bits) frexpf(__uint_as_float(amax_bits), &E);
  const uint32_t count = end - start;
  int lg = 0;
  while (lg < 32 && (1u << lg) < count) ++lg;
  const int f = 61 - E - lg, g = 62 - lg;
  const double scale = ldexp(1.0, f), inv = ldexp(1.0, -f);
  // v 2^f is exact (a power-of-two scale of a float), and so is its
  // remainder after rounding to the nearest integer
  bool any_rem = false;
  for_range_items(items, start, end, [&](uint2 it) {
    if (it.x < (uint32_t)cells) {
      const double x = (double)__uint_as_float(it.y) * scale;
      const double q = rint(x);
      atomicAdd(&s_acc[it.x], (unsigned long long)(long long)q);
      if (x != q) {
        atomicOr(&s_rbits[it.x >> 5], 1u << (it.x & 31));
        any_rem = true;
      }
    }
  });
  if (any_rem) s_resid = 2;   // some remainder: look at the cells
  __syncthreads();
  if (s_resid == 2) {
    __syncthreads();   // every thread has read the flag before it is reset
    if (threadIdx.x == 0) s_resid = 0;
    __syncthreads();
    bool small = false;
    for (int c = threadIdx.x; c < cells; c += kThreads) {
      const long long h = (long long)s_acc[c];
      small |= ((s_rbits[c >> 5] >> (c & 31)) & 1u) && h < (1ll << 24) && h > -(1ll << 24);
    }
    if (small) s_resid = 1;
    __syncthreads();
  }
  if (!s_resid) {
    for (int c = threadIdx.x; c < cells; c += kThreads) {
      const int64_t bucket = ((int64_t)p << bp_shift) + c / d;
      const float v = (float)((double)(long long)s_acc[c] * inv);
      if constexpr (FUSED)
        slice[c] = bucket < B ? v : 0.0f;
      else if (bucket < B)
        SX[bucket * d + c % d] = v;
    }
    if constexpr (EMIT && !FUSED) {
      if (a.fp8_scale)
        emit_fp8_scales(a, p, cells, [&](int c) {
          const int64_t bucket = ((int64_t)p << bp_shift) + c / d;
          return bucket < B ? (float)((double)(long long)s_acc[c] * inv) : 0.0f;
        }, s_rbits);
    }
    return;
  }
  // second pass: this thread's cells' q sums to registers, then the
  // remainders summed at scale 2^(f + g) in the same LDS
  long long hold[kCsrCellsPerThread];
#pragma unroll
  for (int k = 0; k < kCsrCellsPerThread; ++k) {
    const int c = threadIdx.x + k * kThreads;
    hold[k] = c < cells ? (long long)s_acc[c] : 0ll;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cells; c += kThreads) s_acc[c] = 0ull;
  __syncthreads();
  const double rscale = ldexp(1.0, g), rinv = ldexp(1.0, -f - g);
  for_range_items(items, start, end, [&](uint2 it) {
    if (it.x < (uint32_t)cells) {
      const double x = (double)__uint_as_float(it.y) * scale;
      const double r = x - rint(x);
      if (r != 0.0) atomicAdd(&s_acc[it.x], (unsigned long long)__double2ll_rn(r * rscale));
    }
  });
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kCsrCellsPerThread; ++k) {
    const int c = threadIdx.x + k * kThreads;
    if (c >= cells) break;
    const int64_t bucket = ((int64_t)p << bp_shift) + c / d;
    const float v = (float)((double)hold[k] * inv + (double)(long long)s_acc[c] * rinv);
    if constexpr (FUSED)
      slice[c] = bucket < B ? v : 0.0f;
    else if (bucket < B)
      SX[bucket * d + c % d] = v;
  }
  if constexpr (EMIT && !FUSED) {
    if (a.fp8_scale) {
      // the range's values were written by this workgroup: read them back
      __syncthreads();
      __threadfence_block();
      emit_fp8_scales(a, p, cells, [&](int c) {
        const int64_t bucket = ((int64_t)p << bp_shift) + c / d;
        return bucket < B ? SX[bucket * d + c % d] : 0.0f;
      }, s_rbits);
    }
  }
}

// ------------------------------------------------------- fused contraction
// The fused single pass: a range's S X slice, summed in LDS as above, is
// multiplied at once by the columns of G of the range's buckets (generated
// in registers), so S X never reaches memory; each range leaves one partial
// m x d product, and the split reduction adds the R partials in range
// order (bitwise reproducible).  All sixteen wavefronts take a sixteenth
// of the range's buckets each, in steps of four on 16x16x4 FP32 MFMA with
// the contraction kernel's register tiling (lane (p, kq): G rows 4 q + t of
// quad q = 16 group + p, K slot kq).  For every 64-row group of G and
// 16 NB-column group of S X in turn, the sixteen accumulators are added in
// a fixed tree through LDS (wave w + h into wave w, h = 8, 4, 2, 1, two
// column blocks at a time), and wave 0 writes the partial.
constexpr int kFusedWaves = kThreads / 64;

template <int NB>
__device__ __forceinline__ void fused_contract(const BinArgs& a, int p, const float* slice,
                                               float* red) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int pl = lane & 15, kq = lane >> 4;
  const int d = a.d, m = a.m;
  const int Bp = 1 << a.bp_shift;
  const int64_t bucket0 = (int64_t)p << a.bp_shift;
  const int kc = ((Bp + kFusedWaves - 1) / kFusedWaves + 3) & ~3;
  const int kbeg = wave * kc, kend = min(kbeg + kc, Bp);
  float* __restrict__ out = a.part + (size_t)p * m * d;
  const int mgroups = (m + 63) / 64, ngroups = (d + 16 * NB - 1) / (16 * NB);
  constexpr int NBC = NB < 2 ? NB : 2;   // column blocks per reduction pass
  constexpr int kV = 16 * NBC;           // values per lane per pass
  for (int g = 0; g < mgroups; ++g) {
    const uint32_t q = (uint32_t)(16 * g + pl);
    for (int ng = 0; ng < ngroups; ++ng) {
      const int n0 = ng * 16 * NB;
      v4f acc[4][NB];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[t][nb] = v4f{0, 0, 0, 0};
      for (int k0 = kbeg; k0 < kend; k0 += 4) {
        const int bl = k0 + kq;
        const int64_t bucket = bucket0 + bl;
        const bool ok = bl < kend && bucket < (int64_t)a.B;
        // a zero S X operand makes the normals of a column past the range
        // or past B add nothing, so they need no mask
        float z[4];
        box_muller(gauss_block((uint32_t)bucket, q, a.key.k0, a.key.k1), z);
        float x[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int c = n0 + nb * 16 + pl;
          x[nb] = ok && c < d ? slice[bl * d + c] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[t][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(z[t], x[nb], acc[t][nb], 0, 0, 0);
      }
      for (int h = kFusedWaves / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int nb0 = 0; nb0 < NB; nb0 += NBC) {
          if (wave >= h && wave < 2 * h) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
              for (int c = 0; c < NBC; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  if (nb0 + c < NB)
                    red[((wave - h) * kV + (t * NBC + c) * 4 + r) * 64 + lane] = acc[t][nb0 + c][r];
          }
          __syncthreads();
          if (wave < h) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
              for (int c = 0; c < NBC; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  if (nb0 + c < NB)
                    acc[t][nb0 + c][r] += red[(wave * kV + (t * NBC + c) * 4 + r) * 64 + lane];
          }
          __syncthreads();   // red is reused by the next pass
        }
      }
      if (wave == 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 4 * (16 * g + 4 * kq + r) + t;
              const int col = n0 + nb * 16 + pl;
              if (row < m && col < d) out[(size_t)row * d + col] = acc[t][nb][r];
            }
      }
    }
  }
}

// Two workgroups per CU when the ranges' LDS allows it (the batched
// launch's small ranges do): eight waves per SIMD, 64 registers per lane.
template <bool EMIT>
__global__ __launch_bounds__(kThreads, 8) void bin_reduce_csr_kernel(BinArgs a) {
  reduce_csr_range<false, EMIT>(a, blockIdx.x);
}

// LDS of the fused kernel: the range's fixed-point sums (64 KB, reused for
// the cross-wave sums of the contraction) | its FP32 slice (32 KB)
constexpr size_t kFusedLds = (size_t)kCsrMaxCells * 8 + (size_t)kCsrMaxCells * 4;
static_assert((size_t)(kFusedWaves / 2) * 16 * 2 * 64 * 4 <= (size_t)kCsrMaxCells * 8,
              "a pass of the cross-wave tree fits in the fixed-point area");

template <int NB>
__global__ __launch_bounds__(kThreads) void bin_reduce_fused_kernel(BinArgs a) {
  float* slice = (float*)(dyn_lds + (size_t)kCsrMaxCells * 8);
  reduce_csr_range<true>(a, blockIdx.x, slice);
  __syncthreads();   // the slice is complete; the fixed-point area is free
  fused_contract<NB>(a, blockIdx.x, slice, (float*)dyn_lds);
}

// Dense LDS: slice Bp*d floats | rows and their buckets (kDenseCap) |
// cnt, off, fill (Bp each) | block scan
__host__ __device__ inline size_t dense_reduce_lds_bytes(int Bp, int d) {
  return (size_t)Bp * d * 4 + (size_t)kDenseCap * 6 + (size_t)3 * Bp * 4 + kWaves * 4;
}

// LPR lanes per row, VEC consecutive floats per lane (VEC = 4: one 16-byte
// load per lane, so a wavefront instruction brings 64 / LPR whole rows;
// needs d and ldx multiples of 4 and X 16-byte aligned).
template <int LPR, int VEC>
__device__ __forceinline__ void reduce_dense_range(const BinArgs& a, int p) {
  const float* __restrict__ X = a.X;
  const int64_t ldx = a.ldx, n = a.n;
  const uint2* __restrict__ items = a.items;
  const uint32_t* __restrict__ tot = a.tot;
  const uint32_t total = (uint32_t)n, B = a.B;
  const int d = a.d, bp_shift = a.bp_shift;
  float* __restrict__ SX = a.SX;
  constexpr int RPP = 64 / LPR;                // lane groups: rows per load instruction
  constexpr int U = 8;                         // row loads in flight per lane group
  constexpr int PER = kDenseCap / kThreads;    // items held per thread
  __shared__ uint64_t s_red64[kWaves];
  const int Bp = 1 << bp_shift;
  const int cells = Bp * d;
  float* slice = (float*)dyn_lds;
  uint32_t* rows = (uint32_t*)(slice + cells);
  uint16_t* rb = (uint16_t*)(rows + kDenseCap);
  uint32_t* cnt = (uint32_t*)(rb + kDenseCap);
  uint32_t* off = cnt + Bp;
  uint32_t* fill = off + Bp;
  uint32_t* s_w = fill + Bp;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane / LPR, c = (lane % LPR) * VEC;
  const bool cok = c < d;
  const int cc = cok ? c : 0;
  // wave w owns the contiguous buckets [lb0, lb1)
  const int lb0 = (int)(((int64_t)Bp * wave) / kWaves), lb1 = (int)(((int64_t)Bp * (wave + 1)) / kWaves);
  for (int i = threadIdx.x; i < cells; i += kThreads) slice[i] = 0.0f;
  uint32_t start, end;
  range_of(tot, p, total, s_red64, &start, &end);
  for (uint32_t c0 = start; c0 < end; c0 += kDenseCap) {
    const uint32_t nit = min(end - c0, (uint32_t)kDenseCap);
    for (int b = threadIdx.x; b < Bp; b += kThreads) {
      cnt[b] = 0;
      fill[b] = 0;
    }
    __syncthreads();
    uint2 it[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) it[u] = items[c0 + min(threadIdx.x + u * kThreads, nit - 1)];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const bool ok = threadIdx.x + u * kThreads < nit && it[u].y < (uint32_t)Bp &&
                      (int64_t)(it[u].x & 0x7fffffffu) < n;
      if (!ok) it[u].y = 0xffffffffu;
      else atomicAdd(&cnt[it[u].y], 1u);
    }
    __syncthreads();
    // exclusive scan of the bucket counts (Bp <= 1024: one per thread)
    uint32_t tt;
    const uint32_t ex =
        block_exscan<kThreads>(threadIdx.x < (unsigned)Bp ? cnt[threadIdx.x] : 0u, s_w, &tt);
    if (threadIdx.x < (unsigned)Bp) off[threadIdx.x] = ex;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      if (it[u].y != 0xffffffffu) {
        const uint32_t pos = off[it[u].y] + atomicAdd(&fill[it[u].y], 1u);
        if (pos < (uint32_t)kDenseCap) {
          rows[pos] = it[u].x;
          rb[pos] = (uint16_t)it[u].y;
        }
      }
    }
    __syncthreads();
    // lane group j of wave w owns a contiguous block of buckets, so its rows
    // are contiguous after the sort and no other group touches its slice
    // cells: it streams its rows (U loads in flight), sums each bucket in
    // registers and adds the sum into the slice with a plain read-add-write
    // when the bucket changes
    const int ng = lb1 - lb0;
    const int gb0 = lb0 + (int)(((int64_t)ng * j) / RPP);
    const int gb1 = lb0 + (int)(((int64_t)ng * (j + 1)) / RPP);
    const uint32_t s = gb0 < Bp ? off[gb0] : min(tt, (uint32_t)kDenseCap);
    const uint32_t e = gb1 < Bp ? off[gb1] : min(tt, (uint32_t)kDenseCap);
    float acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = 0.0f;
    int cur = -1;
    auto flush = [&]() {
      if (cur >= 0 && cok) {
        float* dst = slice + cur * d + c;
        if constexpr (VEC == 4) {
          float4 o = *(float4*)dst;
          o.x += acc[0];
          o.y += acc[1];
          o.z += acc[2];
          o.w += acc[3];
          *(float4*)dst = o;
        } else {
          *dst += acc[0];
        }
      }
    };
    for (uint32_t i = s; i < e; i += U) {
      uint32_t rs[U];
      int bk[U];
      float x[U][VEC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t ii = min(i + u, e - 1);
        rs[u] = rows[ii];
        bk[u] = i + u < e ? (int)rb[ii] : -1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // non-temporal: each row of X is read once, and streaming it past
        // the caches keeps S X (written next, read by the contraction) and
        // the item list in the last-level cache
        const float* src = X + (int64_t)(rs[u] & 0x7fffffffu) * ldx + cc;
        if constexpr (VEC == 4) {
          typedef float f32x4 __attribute__((ext_vector_type(4)));
          const f32x4 q = __builtin_nontemporal_load((const f32x4*)src);
          x[u][0] = q.x;
          x[u][1] = q.y;
          x[u][2] = q.z;
          x[u][3] = q.w;
        } else {
          x[u][0] = __builtin_nontemporal_load(src);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (bk[u] < 0) continue;
        if (bk[u] != cur) {
          flush();
          cur = bk[u];
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[v] = 0.0f;
        }
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] += (rs[u] >> 31) ? -x[u][v] : x[u][v];
      }
    }
    flush();
    __syncthreads();
  }
  __syncthreads();
  for (int q = threadIdx.x; q < cells; q += kThreads) {
    const int64_t bucket = ((int64_t)p << bp_shift) + q / d;
    if (bucket < B) SX[bucket * d + q % d] = slice[q];
  }
  if (a.fp8_scale) {
    __shared__ uint32_t s_amax[kDenseMaxBlocks];
    emit_fp8_scales(a, p, cells, [&](int q) {
      const int64_t bucket = ((int64_t)p << bp_shift) + q / d;
      return bucket < B ? slice[q] : 0.0f;
    }, s_amax);
  }
}

template <int LPR, int VEC>
__global__ __launch_bounds__(kThreads) void bin_reduce_dense_kernel(BinArgs a) {
  reduce_dense_range<LPR, VEC>(a, blockIdx.x);
}

int lanes_per_row(int d) {
  int l = 1;
  while (l < d && l < 64) l <<= 1;
  return l;
}

// Kernels using more than 64 KB of LDS say so before their launch.
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 48 * 1024) return hipSuccess;   // headroom for static LDS
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

size_t count_lds_bytes(int R) { return (size_t)R * 4 + (size_t)kCntWaves * 2 * kCRpWin * 4; }

// ------------------------------------------------------------------ batched
// One workgroup per work item of any instance: item -> instance from the
// item table, local index = item - first item of that instance.
__global__ __launch_bounds__(kCntThreads) void bin_count_batched(const BinArgs* __restrict__ args,
                                                               const int32_t* __restrict__ inst,
                                                               const int32_t* __restrict__ first) {
  const int i = inst[blockIdx.x];
  const BinArgs a = args[i];
  count_tile<true>(a, (int64_t)blockIdx.x - first[i]);
}

__global__ __launch_bounds__(kSThreads) void bin_scan_batched(const BinArgs* __restrict__ args,
                                                              const int32_t* __restrict__ inst,
                                                              const int32_t* __restrict__ first) {
  const int i = inst[blockIdx.x];
  const BinArgs a = args[i];
  scan_range(a, (int)((int64_t)blockIdx.x - first[i]));
}

__global__ __launch_bounds__(kSThreads, 4) void bin_scatter_batched(const BinArgs* __restrict__ args,
                                                                 const int32_t* __restrict__ inst,
                                                                 const int32_t* __restrict__ first) {
  const int i = inst[blockIdx.x];
  const BinArgs a = args[i];
  scatter_csr_tile(a, (int64_t)blockIdx.x - first[i]);
}

__global__ __launch_bounds__(kThreads, 8) void bin_reduce_batched(const BinArgs* __restrict__ args,
                                                               const int32_t* __restrict__ inst,
                                                               const int32_t* __restrict__ first) {
  const int i = inst[blockIdx.x];
  const BinArgs a = args[i];
  reduce_csr_range(a, (int)((int64_t)blockIdx.x - first[i]));
}

}  // namespace

BinGeom bin_geometry(bool csr, int64_t n, int d, int64_t B, int64_t tile_rows) {
  BinGeom g;
  int shift = 0;
  if (csr) {
    while (shift < 30 && ((int64_t)2 << shift) * d <= kCsrMaxCells) ++shift;   // int64 cells, 64 KB
    g.lds_bytes = (size_t)(1 << shift) * d * 8;
  } else {
    while (shift < 10 && ((int64_t)2 << shift) * d <= 16384) ++shift;  // float cells, 64 KB
    g.lds_bytes = dense_reduce_lds_bytes(1 << shift, d);
  }
  g.bp_shift = shift;
  g.R = (int)((B + ((int64_t)1 << shift) - 1) >> shift);
  if (tile_rows > 0) {
    g.tile_rows = tile_rows;
  } else {
    // about 1024 tiles (four workgroups per CU), whole 1024-row rounds, at
    // most kBinTileRows: a small X still fills the GPU (each tile's rounds
    // run one after another in its workgroup)
    const int64_t per = (n + 1023) / 1024;
    g.tile_rows = std::min<int64_t>(std::max<int64_t>((per + kRoundRows - 1) / kRoundRows, 1) * kRoundRows,
                                    kBinTileRows);
  }
  g.ntiles = (n + g.tile_rows - 1) / g.tile_rows;
  g.ok = g.R <= (csr ? kBinMaxRangesCsr : kBinMaxRangesDense) && d <= (csr ? kMaxD : 64) &&
         n < ((int64_t)1 << 31) && (int64_t)g.R * g.ntiles < ((int64_t)1 << 30) &&
         g.tile_rows % kRoundRows == 0 && g.tile_rows <= ((int64_t)1 << 24) &&
         scatter_lds_bytes(g.R, csr) <= 160 * 1024 &&
         stage_cap(g.R, csr) >= (csr ? kRoundRows : kCRoundRows);
  return g;
}

bool binned_emits_fp8_scales(bool csr, int64_t n, int d, int64_t B) {
  const BinGeom g = bin_geometry(csr, n, d, B);
  return g.ok && (1 << g.bp_shift) >= 128;
}

size_t binned_scratch_bytes(const BinGeom& g, int64_t count) {
  return bin_carve(nullptr, g.R, g.ntiles, count, nullptr);
}

static BinArgs make_args(const BinGeom& g, int64_t n, int d, uint32_t B, Key key,
                         uint64_t row_offset, float* SX, void* scratch, int64_t count) {
  BinArgs a{};
  a.n = n;
  a.d = d;
  a.B = B;
  a.key = key;
  a.row_offset = row_offset;
  a.bp_shift = g.bp_shift;
  a.R = g.R;
  a.ntiles = g.ntiles;
  a.tile_rows = g.tile_rows;
  a.SX = SX;
  bin_carve((char*)scratch, g.R, g.ntiles, count, &a);
  return a;
}

hipError_t launch_sx_binned_csr(const int32_t* row_ptr, const int32_t* col_idx, const float* vals,
                                int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                                uint64_t row_offset, float* SX, void* scratch, hipStream_t s,
                                void* const* events, float2* fp8_scale) {
  const BinGeom g = bin_geometry(true, n, d, B);
  BinArgs a = make_args(g, n, d, B, key, row_offset, SX, scratch, nnz);
  a.fp8_scale = (1 << g.bp_shift) >= 128 ? fp8_scale : nullptr;
  a.row_ptr = row_ptr;
  a.col_idx = col_idx;
  a.vals = vals;
  a.nnz = (int32_t)nnz;
  const size_t sl = scatter_lds_bytes(g.R, true), cl = count_lds_bytes(g.R);
  hipError_t e;
  if ((e = allow_lds(bin_count_kernel<true>, cl)) != hipSuccess) return e;
  if ((e = allow_lds(bin_scatter_csr_kernel, sl)) != hipSuccess) return e;
  if ((e = allow_lds(bin_reduce_csr_kernel<false>, g.lds_bytes)) != hipSuccess) return e;
  if ((e = allow_lds(bin_reduce_csr_kernel<true>, g.lds_bytes)) != hipSuccess) return e;
  bin_count_kernel<true><<<(unsigned)g.ntiles, kCntThreads, cl, s>>>(a);
  bin_scan_kernel<<<(unsigned)g.R, kSThreads, 0, s>>>(a);
  if (events && events[1] && (e = hipEventRecord((hipEvent_t)events[1], s)) != hipSuccess) return e;
  bin_scatter_csr_kernel<<<(unsigned)g.ntiles, kSThreads, sl, s>>>(a);
  if (a.fp8_scale)
    bin_reduce_csr_kernel<true><<<(unsigned)g.R, kThreads, g.lds_bytes, s>>>(a);
  else
    bin_reduce_csr_kernel<false><<<(unsigned)g.R, kThreads, g.lds_bytes, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_sx_fused_csr(const int32_t* row_ptr, const int32_t* col_idx, const float* vals,
                               int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                               uint64_t row_offset, int m, float* part, void* scratch,
                               hipStream_t s, void* const* events) {
  const BinGeom g = bin_geometry(true, n, d, B);
  BinArgs a = make_args(g, n, d, B, key, row_offset, nullptr, scratch, nnz);
  a.row_ptr = row_ptr;
  a.col_idx = col_idx;
  a.vals = vals;
  a.nnz = (int32_t)nnz;
  a.m = m;
  a.part = part;
  const size_t sl = scatter_lds_bytes(g.R, true), cl = count_lds_bytes(g.R);
  const int nb = d >= 64 ? 4 : (d + 15) / 16;
  hipError_t e;
  if ((e = allow_lds(bin_count_kernel<true>, cl)) != hipSuccess) return e;
  if ((e = allow_lds(bin_scatter_csr_kernel, sl)) != hipSuccess) return e;
  bin_count_kernel<true><<<(unsigned)g.ntiles, kCntThreads, cl, s>>>(a);
  bin_scan_kernel<<<(unsigned)g.R, kSThreads, 0, s>>>(a);
  if (events && events[1] && (e = hipEventRecord((hipEvent_t)events[1], s)) != hipSuccess) return e;
  bin_scatter_csr_kernel<<<(unsigned)g.ntiles, kSThreads, sl, s>>>(a);
  if (events && events[2] && (e = hipEventRecord((hipEvent_t)events[2], s)) != hipSuccess) return e;
#define CG_FUSED(NBV)                                                                   \
  if ((e = allow_lds(bin_reduce_fused_kernel<NBV>, kFusedLds)) != hipSuccess) return e; \
  bin_reduce_fused_kernel<NBV><<<(unsigned)g.R, kThreads, kFusedLds, s>>>(a);
  switch (nb) {
    case 1: CG_FUSED(1) break;
    case 2: CG_FUSED(2) break;
    case 3: CG_FUSED(3) break;
    default: CG_FUSED(4) break;
  }
#undef CG_FUSED
  return hipGetLastError();
}

hipError_t launch_sx_binned_dense(const float* X, int64_t ldx, int64_t n, int d, uint32_t B,
                                  Key key, uint64_t row_offset, float* SX, void* scratch,
                                  hipStream_t s, void* const* events, float2* fp8_scale) {
  const BinGeom g = bin_geometry(false, n, d, B);
  BinArgs a = make_args(g, n, d, B, key, row_offset, SX, scratch, n);
  a.fp8_scale = (1 << g.bp_shift) >= 128 ? fp8_scale : nullptr;
  a.X = X;
  a.ldx = ldx;
  const size_t sl = scatter_lds_bytes(g.R, false), cl = count_lds_bytes(g.R);
  hipError_t e;
  if ((e = allow_lds(bin_count_kernel<false>, cl)) != hipSuccess) return e;
  if ((e = allow_lds(bin_scatter_dense_kernel, sl)) != hipSuccess) return e;
  bin_count_kernel<false><<<(unsigned)g.ntiles, kCntThreads, cl, s>>>(a);
  bin_scan_kernel<<<(unsigned)g.R, kSThreads, 0, s>>>(a);
  if (events && events[1] && (e = hipEventRecord((hipEvent_t)events[1], s)) != hipSuccess) return e;
  bin_scatter_dense_kernel<<<(unsigned)g.ntiles, kSThreads, sl, s>>>(a);
  const unsigned gr = (unsigned)g.R;
  const size_t rl = g.lds_bytes;
#define CG_DENSE_REDUCE(L, V)                                                     \
  if ((e = allow_lds(bin_reduce_dense_kernel<L, V>, rl)) != hipSuccess) return e; \
  bin_reduce_dense_kernel<L, V><<<gr, kThreads, rl, s>>>(a);
  // 16-byte row loads when every row start is 16-byte aligned (a random
  // 256-byte row gather runs at 5.7 TB/s that way, 3.8 TB/s with 4-byte
  // lanes)
  const bool vec4 = d % 4 == 0 && ldx % 4 == 0 && ((uintptr_t)X & 15) == 0;
  if (vec4) {
    switch (lanes_per_row(d / 4)) {
      case 1: CG_DENSE_REDUCE(1, 4) break;
      case 2: CG_DENSE_REDUCE(2, 4) break;
      case 4: CG_DENSE_REDUCE(4, 4) break;
      case 8: CG_DENSE_REDUCE(8, 4) break;
      default: CG_DENSE_REDUCE(16, 4) break;
    }
  } else {
    switch (lanes_per_row(d)) {
      case 1: CG_DENSE_REDUCE(1, 1) break;
      case 2: CG_DENSE_REDUCE(2, 1) break;
      case 4: CG_DENSE_REDUCE(4, 1) break;
      case 8: CG_DENSE_REDUCE(8, 1) break;
      case 16: CG_DENSE_REDUCE(16, 1) break;
      case 32: CG_DENSE_REDUCE(32, 1) break;
      default: CG_DENSE_REDUCE(64, 1) break;
    }
  }
#undef CG_DENSE_REDUCE
  return hipGetLastError();
}

hipError_t launch_sx_binned_batched(const BinArgs* args, const int32_t* tile_inst,
                                    const int32_t* tile_first, int64_t tiles,
                                    const int32_t* range_inst, const int32_t* range_first,
                                    int64_t ranges, int r_max, size_t reduce_lds, hipStream_t s) {
  // every instance's scatter layout fits: scatter_lds_bytes(R) <= max(kScatterLdsCsr,
  // scatter_lds_bytes(r_max)) for R <= r_max (the stage only shrinks to its floor
  // as R grows); count_lds_bytes grows with R
  const size_t sl = std::max(scatter_lds_bytes(r_max, true), kScatterLdsCsr);
  const size_t cl = count_lds_bytes(r_max);
  hipError_t e;
  if ((e = allow_lds(bin_count_batched, cl)) != hipSuccess) return e;
  if ((e = allow_lds(bin_scatter_batched, sl)) != hipSuccess) return e;
  if ((e = allow_lds(bin_reduce_batched, reduce_lds)) != hipSuccess) return e;
  if (tiles > 0) bin_count_batched<<<(unsigned)tiles, kCntThreads, cl, s>>>(args, tile_inst, tile_first);
  if (ranges > 0) bin_scan_batched<<<(unsigned)ranges, kSThreads, 0, s>>>(args, range_inst, range_first);
  if (tiles > 0) bin_scatter_batched<<<(unsigned)tiles, kSThreads, sl, s>>>(args, tile_inst, tile_first);
  if (ranges > 0)
    bin_reduce_batched<<<(unsigned)ranges, kThreads, reduce_lds, s>>>(args, range_inst, range_first);
  return hipGetLastError();
}

}  // namespace cg
