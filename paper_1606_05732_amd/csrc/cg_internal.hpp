// Host-side launchers shared between the kernel sources and the C ABI.
// Every launcher only queues work on `stream`; sizes are validated by the
// caller (cg_capi.hip) before any launcher runs.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cg {

struct Key {
  uint32_t k0, k1;
};
inline Key key_of(uint64_t seed) { return Key{(uint32_t)seed, (uint32_t)(seed >> 32)}; }

// Message for cg_last_error() of the calling thread.
void set_last_error(const char* msg);

constexpr int kRowsPerWave = 256;   // rows hashed and handled per wavefront
constexpr int kMaxD = 1024;         // widest X the library supports

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---- S X --------------------------------------------------------------
template <typename T>
hipError_t launch_fill_zero(T* p, size_t count, hipStream_t s);

template <typename T>
hipError_t launch_sx_csr_atomic(const int32_t* row_ptr, const int32_t* col_idx, const T* vals,
                                int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                                uint64_t row_offset, T* SX, hipStream_t s);

template <typename T>
hipError_t launch_sx_dense_atomic(const T* X, int64_t ldx, int64_t n, int d, uint32_t B, Key key,
                                  uint64_t row_offset, T* SX, hipStream_t s);

// Deterministic path: stable counting sort by bucket, then a fixed-order
// per-bucket reduction.  `count` items (rows for dense X, stored entries for
// CSR) of `payload` bytes each.
size_t sorted_scratch_bytes(int64_t count, int64_t B, size_t payload);
inline size_t sorted_payload_bytes(bool csr, size_t elem) {
  return csr ? (elem == 8 ? 16 : 8) : 4;
}

template <typename T>
hipError_t launch_sx_csr_sorted(const int32_t* row_ptr, const int32_t* col_idx, const T* vals,
                                int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                                uint64_t row_offset, T* SX, void* scratch, hipStream_t s);

template <typename T>
hipError_t launch_sx_dense_sorted(const T* X, int64_t ldx, int64_t n, int d, uint32_t B, Key key,
                                  uint64_t row_offset, T* SX, void* scratch, hipStream_t s);

// Exclusive scan of a[0 .. len) in place; sums needs scan_sums_len(len)
// entries of scratch.
int64_t scan_sums_len(int64_t len);
hipError_t launch_exclusive_scan(uint32_t* a, int64_t len, uint32_t* sums, hipStream_t s);

// Binned path (FP32): bucket ranges of 2^bp_shift buckets whose S X slice
// fits in LDS, R ranges, ntiles row tiles.
constexpr int kBinMaxRangesCsr = 2048;
constexpr int kBinMaxRangesDense = 2048;
struct BinGeom {
  int bp_shift = 0;        // buckets per range = 2^bp_shift
  int R = 0;               // ranges
  int64_t ntiles = 0;      // row tiles
  int64_t tile_rows = 0;   // rows per tile
  size_t lds_bytes = 0;    // LDS of the reduce kernel
  bool ok = false;         // this path applies
};
constexpr int64_t kBinTileRows = 16384;   // default rows per tile (a multiple of 1024)
// tile_rows = 0 picks about n / 1024 rows (whole 1024-row rounds, at most
// kBinTileRows); otherwise a multiple of 1024.
BinGeom bin_geometry(bool csr, int64_t n, int d, int64_t B, int64_t tile_rows = 0);
size_t binned_scratch_bytes(const BinGeom& g, int64_t count);
// Whether the binned reduce can write the FP8 block scales (ranges of at
// least 128 buckets).
bool binned_emits_fp8_scales(bool csr, int64_t n, int d, int64_t B);

// Everything one binned S X needs (one instance).  The scratch arrays are
// laid out by bin_carve.
struct BinArgs {
  const int32_t* row_ptr;   // CSR X
  const int32_t* col_idx;
  const float* vals;
  const float* X;           // dense X
  int64_t ldx;
  int64_t n;
  int32_t nnz;
  int32_t d;
  uint32_t B;
  Key key;
  uint64_t row_offset;
  int32_t bp_shift;
  int32_t R;
  int64_t ntiles;
  int64_t tile_rows;
  uint32_t* hist;   // R x ntiles: counts, then offsets inside each range
  uint32_t* tot;    // R: items per range
  uint32_t* hmax;   // R x ntiles: largest |value| bits (CSR)
  uint2* items;     // one per stored entry (CSR) or row (dense)
  float* SX;        // B x d
  // fused single pass (launch_sx_fused_csr): rows of G and the per-range
  // partial products (R x m x d)
  int32_t m;
  float* part;
  // if not NULL, the reduce also writes the FP8 contraction's scale pair of
  // every 128-bucket block (needs 2^bp_shift >= 128)
  float2* fp8_scale;
};

// Binned scratch at base: hist | tot | hmax | items (each 256-byte aligned).
__host__ __device__ inline size_t bin_carve(char* base, int R, int64_t ntiles, int64_t count,
                                            BinArgs* a) {
  const size_t hl = align256((size_t)R * (size_t)ntiles * 4);
  if (a) {
    a->hist = (uint32_t*)base;
    a->tot = (uint32_t*)(base + hl);
    a->hmax = (uint32_t*)(base + hl + align256((size_t)R * 4));
    a->items = (uint2*)(base + 2 * hl + align256((size_t)R * 4));
  }
  return 2 * hl + align256((size_t)R * 4) + align256((size_t)count * 8);
}

// `events`, if non-NULL, is the caller's stage-event array; events[1] is
// recorded after the split plan (counts and scan).
// fp8_scale: see BinArgs (NULL: not written).
hipError_t launch_sx_binned_csr(const int32_t* row_ptr, const int32_t* col_idx, const float* vals,
                                int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                                uint64_t row_offset, float* SX, void* scratch, hipStream_t s,
                                void* const* events, float2* fp8_scale = nullptr);
hipError_t launch_sx_binned_dense(const float* X, int64_t ldx, int64_t n, int d, uint32_t B,
                                  Key key, uint64_t row_offset, float* SX, void* scratch,
                                  hipStream_t s, void* const* events, float2* fp8_scale = nullptr);

// The fused single pass for CSR X: the binned split, then one workgroup per
// bucket range that sums the range's S X slice in LDS and multiplies it by
// G's columns of those buckets at once, writing part[p] (m x d) for range p
// of the R = bin_geometry(true, n, d, B).R ranges; S X is never written.
// Y is then the fixed-order sum of the R partials.  events[1] / [2] are
// recorded after the split plan and after the scatter.
hipError_t launch_sx_fused_csr(const int32_t* row_ptr, const int32_t* col_idx, const float* vals,
                               int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                               uint64_t row_offset, int m, float* part, void* scratch,
                               hipStream_t s, void* const* events);

// Binned CSR S X of many instances at once: one launch per phase over every
// instance's work items.  args[i] is instance i (device array); tile_inst /
// range_inst give the instance of each tile / range work item and
// tile_first / range_first[i] the first item of instance i.  r_max and
// reduce_lds are the largest R and reduce LDS over the batch.
hipError_t launch_sx_binned_batched(const BinArgs* args, const int32_t* tile_inst,
                                    const int32_t* tile_first, int64_t tiles,
                                    const int32_t* range_inst, const int32_t* range_first,
                                    int64_t ranges, int r_max, size_t reduce_lds, hipStream_t s);

// ---- G (S X) -----------------------------------------------------------
enum class Prec { Native, BF16, FP8 };

struct GsxPlan {
  int kc;          // columns of G per wavefront
  int waves;       // wavefronts per workgroup
  int64_t parts;   // workgroups along B = number of split partials
  int mgroups;     // 64-row groups of G
  int ngroups;     // column groups of S X
  int nb;          // 16-column blocks per wavefront
};

GsxPlan plan_gsx(int64_t m, int64_t B, int64_t d, Prec prec, int kc_request, size_t elem);

// Partial products part[p] (m x d) of workgroup p along B ...  FP8 needs
// `scales`: fp8_scale_bytes(B) of workspace for the per-128-block scales.
// scales_ready: the S X producer already wrote them (else a scale kernel
// runs first).
size_t fp8_scale_bytes(int64_t B);
template <typename T>
hipError_t launch_gsx_partials(const GsxPlan& plan, Prec prec, const T* SX, int64_t B, int d,
                               int m, Key key, T* part, hipStream_t s, void* scales = nullptr,
                               bool scales_ready = false);
// ... and Y = sum over p of part[p] in increasing p.
template <typename T>
hipError_t launch_splitk_reduce(const T* part, int64_t parts, int64_t md, T* Y, hipStream_t s);

// ---- rows route (no S X) ----------------------------------------------
// Y = sum over the nonempty rows r of CSR X of sigma(r) G[:, h(r)] x_r^T,
// the same product as G (S X) taken row by row.  Workgroup p of the split
// takes 4 rpw consecutive rows (rpw per wavefront: a multiple of 256 from
// 256 to 2048, about n / 4096 so that a small X still gives some thousand
// workgroups) and writes one partial m x d product, reduced as the S X
// route's partials are.
inline int rows_per_wave(int64_t n) {
  const int64_t r = (n + 4095) / 4096;
  const int64_t w = (r + 255) / 256 * 256;
  return (int)(w < 256 ? 256 : w > 2048 ? 2048 : w);
}
inline int64_t rows_parts(int64_t n, int rpw) {
  const int64_t per = 4 * (int64_t)rpw;
  return (n + per - 1) / per;
}
// A batch has parallelism enough across its instances: there each
// wavefront takes the most rows, for the fewest partials.
constexpr int kBatchedRowsPerWave = 2048;

// Whether the rows route costs less than S X plus G (S X).  Work per
// column of G -- a nonempty row on the rows route, a bucket on the S X
// route -- is m normals plus one 16x16x4 MFMA per 16 columns of X and 64
// rows of G (about 13 normals' time each).  The S X route also moves S X
// twice (write and read: about 3 per element) and every stored entry as an
// item (about 6 per entry); the rows route adds each entry into an LDS
// tile (about 4).  The row_ptr reads and hashes, common to both, cancel.
// Nonempty rows are at most min(n, nnz).
inline bool rows_route_pays(int64_t n, int64_t d, int64_t nnz, int64_t m, int64_t B) {
  const double col = (double)m + 13.0 * (double)((d + 15) / 16) * (double)((m + 63) / 64);
  const double rows = (double)(n < nnz ? n : nnz) * col + 4.0 * (double)nnz;
  const double sx = (double)B * (col + 3.0 * (double)d) + 6.0 * (double)nnz;
  return rows < sx;
}

// Contraction of many instances (FP32, native precision).  Instance i:
// Y_i = G_i SX_i with its own key, split over B into `parts` chunks of
// 4 kc columns; its work items are parts x mgroups x ngroups (64 rows of G
// by 64 columns of S X each), then ceil(m d / 64) reduction items.  An
// instance on the rows route (route = 1) has no S X: its parts split the
// rows instead (rows_parts(n, kc) of them, kc = kBatchedRowsPerWave rows
// per wavefront), from row_ptr / col_idx / vals.  The single-instance rows
// route takes the same arguments.
struct GsxArgs {
  const float* SX;
  float* part;   // parts x m x d
  float* Y;      // m x d
  int64_t B;
  int32_t d, m, kc, parts, mgroups, ngroups;
  Key key;
  // rows route
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const float* vals;
  int64_t n;
  uint64_t row_offset;
  int32_t nnz, route;
};

// Partial products of the rows route, one per workgroup of the split
// (grid rows_parts(n, rows_per_wave(n)) x mgroups x ngroups; a.part
// receives them; a.kc is ignored).
// dense_gaussian: the same row-by-row product with the dense Gaussian G~
// (column row_offset + r for row r, no sign) in place of sigma(r) G[:, h(r)]:
// G~ X, the product T X stands in for (a.B and the hash are then unused).
hipError_t launch_rows_partials(const GsxArgs& a, hipStream_t s, bool dense_gaussian = false);

// Partial products of G~ X for dense X (n x d, row stride ldx): the
// contraction of launch_gsx_partials over the n rows of X, with column
// row_offset + r of G~ generated in registers for row r.  pl from
// plan_gsx(m, n, d, Prec::Native, kc, elem).
template <typename T>
hipError_t launch_dense_gaussian_partials(const GsxPlan& pl, const T* X, int64_t ldx, int64_t n,
                                          int d, int m, Key key, uint64_t row_offset, T* part,
                                          hipStream_t s);
// 16-column blocks per contraction wavefront of a batched instance: as few
// as its d needs (one column group below d = 64), else four.  The batch's
// contraction queue holds the items of each width together, in increasing
// width; items_by_nb[k] counts those of width k + 1, and each width is its
// own launch.
inline int batched_nb(int64_t d) { return d < 64 ? (int)((d + 15) / 16) : 4; }
hipError_t launch_gsx_batched(const GsxArgs* args, const int32_t* gsx_inst,
                              const int32_t* gsx_first, const int64_t items_by_nb[4],
                              hipStream_t s);
hipError_t launch_splitk_batched(const GsxArgs* args, const int32_t* red_inst,
                                 const int32_t* red_first, int64_t items, hipStream_t s);

// ---- adjoint ----------------------------------------------------------
template <typename T>
hipError_t launch_gt_dy(const T* dY, int m, int d, int64_t B, Key key, T* Z, hipStream_t s);

template <typename T>
hipError_t launch_gather_dense(const T* Z, int64_t n, int d, uint32_t B, Key key,
                               uint64_t row_offset, T* dX, int64_t lddx, hipStream_t s);

template <typename T>
hipError_t launch_gather_csr(const int32_t* row_ptr, const int32_t* col_idx, const T* Z,
                             int64_t n, int64_t nnz, int d, uint32_t B, Key key,
                             uint64_t row_offset, T* dvals, hipStream_t s);

// ---- Algorithm 1 (anchor extraction) -----------------------------------
// imax[i] / imin[i]: the lowest column of the largest / smallest value of
// row i of Z (m x d, row stride ldz); NaNs never win, -1 for a row of NaNs.
template <typename T>
hipError_t launch_row_extrema(const T* Z, int64_t m, int64_t d, int64_t ldz, int32_t* imax,
                              int32_t* imin, hipStream_t s);

// ---- Section 7 diagnostics ---------------------------------------------
constexpr int kLemmaMaxD = 64;        // widest U
constexpr int kLemmaGramRows = 4096;  // rows per Gram partial
constexpr int kLemmaStats = 6;
size_t lemma_workspace_bytes(int64_t m, int64_t B, int64_t d, bool with_su);
// Y: m x d, SU: B x d (or NULL), both row-major with stride d; ws of
// lemma_workspace_bytes; stats: device double[kLemmaStats].
template <typename T>
hipError_t launch_lemma_stats(const T* Y, const T* SU, int64_t m, int64_t B, int d, double* ws,
                              double* stats, hipStream_t s);

// ---- memory ceilings ----------------------------------------------------
// kind 0: copy src -> dst; 1: read src (dst receives stream_blocks() words);
// 2: write dst.  bytes: a multiple of 16, both pointers 16-byte aligned.
int stream_blocks();
hipError_t launch_stream(int kind, const void* src, void* dst, int64_t bytes, hipStream_t s);
// normals of G's columns [0, B), rows [0, m) (m a multiple of 4); one sum
// per thread into sink[normals_threads()]
int normals_threads();
hipError_t launch_normals_rate(Key key, int64_t m, int64_t B, float* sink, hipStream_t s);

// ---- test access ------------------------------------------------------
hipError_t launch_debug_philox(Key key, const uint32_t* ctr, int64_t count, uint32_t* out,
                               hipStream_t s);
hipError_t launch_debug_hash(Key key, uint32_t B, uint64_t row0, int64_t count, uint32_t* h,
                             int8_t* sigma, hipStream_t s);
template <typename T>
hipError_t launch_debug_gaussian(Key key, int64_t m, int64_t b0, int64_t nb, T* G, hipStream_t s);

}  // namespace cg
