/*
 * countgauss.h -- C ABI of libcountgauss.so, the MI355X (gfx950) CountGauss
 * transform.
 *
 * The transform (Kapralov, Potluru, Woodruff, "How to Fake Multiply by a
 * Gaussian Matrix", Section 1.1 and Section 2): an n x d input X (n >> d,
 * dense or sparse with nnz(X) stored entries) is mapped to the m x d result
 *
 *     Y = T X = G (S X),
 *
 * where S is a B x n CountSketch (column r has its one nonzero, sigma(r) in
 * {+1,-1}, at row h(r)) and G is an m x B matrix of i.i.d. unit-variance
 * Gaussians (Theorem 1; no 1/sqrt(m) scaling).  S X costs O(nnz(X)) and
 * G (S X) is a dense m x B by B x d product (Section 1.1).  T is fixed by
 * (m, B, seed): the seed is the whole state, which is how the paper shares
 * the transform between servers (Section 4, "Distributed Environments").
 *
 * Random source (the paper names none): Philox4x32-10, key = the 64-bit
 * seed; row hash from counter (r>>2 as two words, 0, 0), word r&3:
 * sigma = bit 31 ? -1 : +1, h = ((w & 0x7fffffff) * B) >> 31; G[i][b] is
 * Box-Muller of the words of counter (b, i>>2, 1, 0), entry i&3, with
 * u = ((w >> 9) + 1/2) 2^-23.  cg_debug_* expose these for testing.
 *
 * Conventions for every call:
 *  - Pointers named as device pointers are device memory owned by the
 *    caller; the library never allocates, frees or keeps them.  Host
 *    pointers (opts, the batched table) are read during the call only,
 *    except where stated.
 *  - Matrices are row-major.  Indices are int32 (nnz < 2^31).
 *  - Work is queued on opts->stream (a hipStream_t; NULL = the default
 *    stream) and the call returns without waiting for it; results are
 *    ready when the stream has passed this call.  Outputs are overwritten.
 *  - Arguments are validated before anything is queued; on an error
 *    nothing is queued and cg_last_error() holds a message (per thread).
 *  - Scratch memory comes from opts->workspace (device), at least
 *    cg_workspace_bytes() bytes, 256-byte aligned; its contents on entry
 *    do not matter and are garbage afterwards.  Two calls in flight at the
 *    same time must not share a workspace.
 *  - Values are not checked for finiteness: a NaN in row r reaches bucket
 *    h(r) of S X and then every entry of its column of Y.
 *  - Column indices outside [0, d) and row_ptr entries outside [0, nnz]
 *    are skipped / clamped on the device (no fault), giving an unspecified
 *    result; row_ptr must be nondecreasing for a defined result.
 */
#ifndef COUNTGAUSS_H
#define COUNTGAUSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define CG_OK 0
#define CG_EINVAL 1         /* bad size, null pointer, unknown enum        */
#define CG_ENOSPACE 2       /* workspace missing or smaller than required  */
#define CG_EUNSUPPORTED 3   /* valid, but outside what the library supports (e.g. d > 1024) */
#define CG_EHIP 4           /* a HIP runtime call failed (message kept)    */

/* ---- element type of X / Y / dY / dX / S X ---------------------------- */
#define CG_DTYPE_F32 0
#define CG_DTYPE_F64 1

/* ---- input precision of the G (S X) contraction ----------------------- *
 * S X is always accumulated in the data type (FP32 for F32 data, FP64 for
 * F64 data).  The contraction's inputs G and S X may be rounded to:       */
#define CG_PREC_NATIVE 0    /* the data type itself (FP32 or FP64)          */
#define CG_PREC_BF16 1      /* bfloat16, round to nearest even; F32 data    */
#define CG_PREC_FP8 2       /* OCP FP8 E4M3 (max 448), round to nearest
                               even, one power-of-two scale per 128-wide
                               block of B for S X and the constant 2^-6 for
                               G (|G| < 5.77); F32 data                     */
/* All precisions accumulate the contraction in the data type (FP32 for
 * BF16/FP8) and reduce the split over B in a fixed order.                */

/* ---- algorithm for S X ------------------------------------------------- */
#define CG_SX_AUTO 0        /* library's choice: for FP32 CSR data at native
                               precision without sx_out, ROWS where its cost
                               model puts it below the S X route; else
                               BINNED for FP32 data when its bucket ranges
                               fit (d <= 64 for dense X), ATOMIC otherwise */
#define CG_SX_ATOMIC 1      /* one device-scope atomic add per stored entry;
                               summation order within a bucket varies from
                               run to run                                  */
#define CG_SX_SORTED 2      /* stable radix sort by bucket, each bucket
                               summed in increasing row order by one
                               wavefront: bitwise reproducible             */
#define CG_SX_BINNED 3      /* FP32 only: split by bucket range, each range
                               summed in LDS by one workgroup.  CSR sums are
                               two-word 64-bit fixed point with a per-range
                               scale from the range's max |x| (bitwise
                               reproducible; every cell keeps FP32 precision
                               for entries down to about
                               max|x| * 2^-(100 - 2 log2 count), smaller ones
                               lose precision); dense rows are summed in FP32
                               (order varies from run to run)              */
#define CG_SX_ROWS 4        /* FP32 CSR data, native precision, no sx_out:
                               S X is not formed.  Y is accumulated as the
                               sum over the nonempty rows r of
                               sigma(r) G[:, h(r)] x_r^T -- the same product
                               G (S X) (Section 1.1: S puts row r into
                               column h(r) with sign sigma(r)) -- in FP32
                               MFMA partials per 1024 to 8192 rows (more
                               rows per partial for larger n), reduced in a
                               fixed order (bitwise reproducible).  Draws m
                               normals per nonempty row instead of per
                               bucket: for X with few nonempty rows next to
                               B (d^2 m buckets and sparse X).  kc is
                               ignored                                   */
#define CG_SX_FUSED 5       /* FP32 CSR data, native precision, no sx_out:
                               the binned split, then one workgroup per
                               bucket range sums the range's S X slice in
                               LDS (as BINNED) and multiplies it at once by
                               the columns of G of those buckets, so S X
                               never reaches memory; the per-range partial
                               products are added in range order (bitwise
                               reproducible).  kc is ignored            */

/* ---- workspace kinds --------------------------------------------------- */
#define CG_KIND_CSR 0
#define CG_KIND_DENSE 1
#define CG_KIND_ADJOINT 2
#define CG_KIND_ADJOINT_CSR 3
#define CG_KIND_GAUSSIAN_DENSE 4   /* cg_gaussian_dense (B ignored)    */
#define CG_KIND_GAUSSIAN_CSR 5     /* cg_gaussian_csr (B ignored)      */
#define CG_KIND_ANCHORS_COUNTGAUSS 6   /* cg_anchors_dense, T X        */
#define CG_KIND_ANCHORS_GAUSSIAN 7     /* cg_anchors_dense, G~ X       */
#define CG_KIND_LEMMA 8                /* cg_lemma_stats (n ignored)   */

typedef struct cg_opts {
  uint32_t struct_size;     /* sizeof(cg_opts)                             */
  int32_t precision;        /* CG_PREC_*                                   */
  int32_t sx_algo;          /* CG_SX_*                                     */
  int32_t kc;               /* columns of G per wavefront in the contraction,
                               a multiple of 16; 0 = library's choice      */
  void* stream;             /* hipStream_t, NULL = default stream          */
  void* workspace;          /* device scratch                              */
  size_t workspace_bytes;   /* its size                                    */
  int64_t row_offset;       /* global index of local row 0: hashing uses
                               row_offset + r, so row chunks or shards of
                               one X sketch consistently and their Y add up
                               (Section 4, distributed environments)       */
  void* sx_out;             /* optional device B x d buffer (data type): if
                               non-NULL S X is accumulated there and left
                               for the caller; otherwise in the workspace  */
  void* const* stage_events;/* optional host array of CG_STAGE_EVENTS
                               hipEvent_t created by the caller; forward
                               calls record them on the stream at the stage
                               boundaries (see below); NULL = none, and a
                               NULL entry skips its boundary (each record
                               leaves the GPU idle for a few microseconds
                               between the kernels it separates)           */
} cg_opts;

/* Forward stage boundaries recorded into cg_opts.stage_events:
 *   [0] before any work
 *   [1] after the S X prologue: atomic, S X zeroed; binned, the per-tile
 *       counts and their offsets; sorted and rows, right after [0]
 *   [2] after S X is complete (rows: right after [1]; it forms no S X)
 *   [3] after the split contraction (rows: its row partials)
 *   [4] after the fixed-order reduction (Y complete)                      */
#define CG_STAGE_EVENTS 5

/* Fill *opts with defaults (native precision, automatic S X algorithm,
 * default stream, no workspace, row_offset 0). */
void cg_opts_init(cg_opts* opts);

/* Library version, e.g. 100 for 0.1.0. */
int cg_version(void);

/* Human-readable name of a status code (static string). */
const char* cg_status_string(int status);

/* Copy the calling thread's last error message into buf (NUL-terminated,
 * truncated to len).  Returns the full message length. */
size_t cg_last_error(char* buf, size_t len);

/* Bytes of workspace the matching call needs for these sizes and options
 * (nnz is ignored for dense kinds).  Returns CG_OK or CG_EINVAL. */
int cg_workspace_bytes(int kind, int dtype, int64_t n, int64_t d, int64_t m,
                       int64_t B, int64_t nnz, const cg_opts* opts,
                       size_t* bytes);

/*
 * Y = G S X for CSR X (Section 1.1: S X in O(nnz(X)), then G (S X)).
 *   row_ptr  device int32[n+1], row_ptr[0] = 0, row_ptr[n] = nnz
 *   col_idx  device int32[nnz], column of each stored entry (in [0, d))
 *   vals     device dtype[nnz]
 *   Y        device dtype[m*d], overwritten
 * 1 <= n, d <= 1024, 1 <= m, 1 <= B < 2^31, 0 <= nnz < 2^31.
 * dtype F64 requires precision NATIVE.  Errors: CG_EINVAL, CG_ENOSPACE,
 * CG_EUNSUPPORTED, CG_EHIP.
 */
int cg_sketch_csr(const int32_t* row_ptr, const int32_t* col_idx,
                  const void* vals, int dtype, int64_t n, int64_t d,
                  int64_t nnz, int64_t m, int64_t B, uint64_t seed, void* Y,
                  const cg_opts* opts);

/*
 * Y = G S X for dense X (n x d, row stride ldx >= d elements).
 * Same sizes, precisions and errors as cg_sketch_csr.
 */
int cg_sketch_dense(const void* X, int64_t ldx, int dtype, int64_t n,
                    int64_t d, int64_t m, int64_t B, uint64_t seed, void* Y,
                    const cg_opts* opts);

/*
 * Adjoint: dX = T^T dY = S^T (G^T dY), the gradient of <dY, T X> with
 * respect to dense X (T = G S is linear, Section 1.1).  First
 * Z = G^T dY (B x d, G regenerated), then dX[r][:] = sigma(r) Z[h(r)][:].
 *   dY  device dtype[m*d];  dX device dtype, n rows of stride lddx >= d,
 *   overwritten.  Precision must be NATIVE.
 */
int cg_sketch_adjoint(const void* dY, int dtype, int64_t n, int64_t d,
                      int64_t m, int64_t B, uint64_t seed, void* dX,
                      int64_t lddx, const cg_opts* opts);

/*
 * Adjoint for CSR X: gradient of <dY, T X> with respect to the stored
 * values, dvals[k] = sigma(r) Z[h(r)][col_idx[k]] for the entry k of row r.
 *   dvals device dtype[nnz], overwritten.
 */
int cg_sketch_adjoint_csr(const int32_t* row_ptr, const int32_t* col_idx,
                          int64_t nnz, const void* dY, int dtype, int64_t n,
                          int64_t d, int64_t m, int64_t B, uint64_t seed,
                          void* dvals, const cg_opts* opts);

/* ---- the dense Gaussian product T X stands in for --------------------- *
 * Y~ = G~ X, with G~ an m x n matrix of i.i.d. unit-variance Gaussians:
 * the projection whose distribution T X matches (Theorem 1 compares G S U
 * with G~ U) and whose cost, O(nnz(X) m), T X avoids (Section 1.1, "Our
 * Results"; the paper's comparison projection "RG").  G~ is generated in
 * registers, never stored: G~[i][r] for the global row r = row_offset +
 * local row is Box-Muller of the Philox words of counter
 * (lo32(r), i >> 2, 2, hi32(r)), entry i & 3 (same key and u mapping as G).
 * The contraction runs on MFMA, split over the rows of X with the partial
 * products added in a fixed order (bitwise reproducible).
 *   dense:  X device dtype, n rows of stride ldx >= d; FP32 or FP64.
 *   CSR:    as cg_sketch_csr; FP32 only (only nonempty rows draw normals).
 *   Y       device dtype[m*d], overwritten.
 * n < 2^31; precision must be NATIVE; workspace of at least
 * cg_workspace_bytes(CG_KIND_GAUSSIAN_DENSE / _CSR, ...) bytes (B is
 * ignored there).  Errors as for cg_sketch_csr.                          */
int cg_gaussian_dense(const void* X, int64_t ldx, int dtype, int64_t n,
                      int64_t d, int64_t m, uint64_t seed, void* Y,
                      const cg_opts* opts);
int cg_gaussian_csr(const int32_t* row_ptr, const int32_t* col_idx,
                    const void* vals, int dtype, int64_t n, int64_t d,
                    int64_t nnz, int64_t m, uint64_t seed, void* Y,
                    const cg_opts* opts);

/* ---- Algorithm 1: anchor extraction for separable NMF ------------------ *
 * Section 4 ("CountGauss NMF"): with X features x points (the anchors are
 * columns), form Z = T X and take, for every row of Z, the column where it
 * is largest (I_max) and smallest (I_min).  Every unique extremum names an
 * anchor of separable X (a linear function over a polytope is extremal at
 * a vertex).  The paper is silent on ties: the lowest column index wins;
 * NaN entries never win and a row without a number gives -1.             */

/* Row extrema of Z (device dtype, m rows of stride ldz >= d): imax[i],
 * imin[i] (device int32[m]).  stream: hipStream_t.                       */
int cg_row_extrema(const void* Z, int dtype, int64_t m, int64_t d,
                   int64_t ldz, int32_t* imax, int32_t* imin, void* stream);

#define CG_PROJ_COUNTGAUSS 0   /* Z = T X (Algorithm 1)                    */
#define CG_PROJ_GAUSSIAN 1     /* Z = G~ X (the Gaussian baseline the paper
                                  compares with, "GP" in Section 6; B unused) */

/* Algorithm 1 on dense X (n x d, row stride ldx; n = features, d = points):
 * Z = T X (proj CG_PROJ_COUNTGAUSS, same options as cg_sketch_dense) or
 * Z = G~ X (CG_PROJ_GAUSSIAN), then its row extrema into imax, imin
 * (device int32[m]).  Z lives in the workspace: at least
 * cg_workspace_bytes(CG_KIND_ANCHORS_COUNTGAUSS / _GAUSSIAN, ...) bytes.
 * opts->stage_events is ignored.  Errors as for cg_sketch_dense.         */
int cg_anchors_dense(const void* X, int64_t ldx, int dtype, int64_t n,
                     int64_t d, int64_t m, int64_t B, uint64_t seed, int proj,
                     int32_t* imax, int32_t* imin, const cg_opts* opts);

/* ---- Section 7 diagnostics --------------------------------------------- *
 * For U (n x d, orthonormal columns, d <= 64), from Y = T U or G~ U
 * (device dtype[m*d]) and optionally S U (device dtype[B*d], e.g. the
 * sx_out of the forward call; NULL = not given), into stats (device
 * double[6]):
 *   [0] max over i < j of | ||Y (e_i + e_j)||^2 - 2 m |: the statistic of
 *       the lower-bound lemma, which a unique collision between the blocks
 *       of two columns moves by about 2 m / L;
 *   [1] ||I - M||_F^2 with M = (S U)^T (S U), the covariance of every row
 *       of T U given S (O(d^2 / B) in expectation, proof of Theorem 1);
 *   [2] KL(N(0, I) || N(0, M)) = 1/2 tr(M^-1 - I) + 1/2 ln det M (the claim
 *       on Gaussian KL divergences; +inf if M is singular);
 *   [3] Pinsker's bound min(1, sqrt(m KL / 2)) on the total variation
 *       between the m rows of T U given S and those of G~ U;
 *   [4] the number of pairs i < j with |M_ij| > 1e-9 (1 after a unique
 *       collision between two columns' blocks);
 *   [5] 1 if M is positive definite, else 0.
 * [1] .. [5] are NaN when SU is NULL.  Gram matrices are summed in FP64 in
 * a fixed order.  Workspace: cg_workspace_bytes(CG_KIND_LEMMA, dtype, -,
 * d, m, B, ...).  Errors: CG_EINVAL, CG_EUNSUPPORTED (d > 64),
 * CG_ENOSPACE, CG_EHIP.                                                  */
int cg_lemma_stats(const void* Y, const void* SU, int dtype, int64_t m,
                   int64_t B, int64_t d, double* stats, const cg_opts* opts);

/* ---- allocation-free forward -------------------------------------------- *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, meaning and result as cg_sketch_csr, but the workspace is a
 * static device buffer of CG_NOALLOC_SCRATCH_BYTES that the library holds
 * on every GPU it runs on until the process ends (opts->workspace and
 * opts->workspace_bytes are ignored; opts may be NULL).  Nothing is
 * allocated or freed.  A call whose workspace (cg_workspace_bytes with kind
 * CG_KIND_CSR) exceeds the buffer fails with CG_ENOSPACE before anything is
 * queued.  Every call on one GPU shares that GPU's buffer: calls that can
 * overlap on one GPU (different streams, or threads without ordering) race
 * and give undefined results; calls queued on one stream are ordered.  The
 * buffer's contents on entry do not matter (every kernel writes what it
 * reads first).  The first call on a device looks up that device's buffer
 * address (hipGetSymbolAddress) with that device current.                */
#define CG_NOALLOC_SCRATCH_BYTES (64u << 20)

int cg_sketch_csr_noalloc(const int32_t* row_ptr, const int32_t* col_idx,
                          const void* vals, int dtype, int64_t n, int64_t d,
                          int64_t nnz, int64_t m, int64_t B, uint64_t seed,
                          void* Y, const cg_opts* opts);

/* ---- many independent instances in one batch ----------------------------- *
 * Independent CSR transforms, each with its own n, d, m, B and seed (FP32,
 * native precision), computed together: each phase of the transform (S X
 * count, scan, scatter and reduce; the contraction; the split reduction)
 * is one launch over the work items of every instance, so small instances
 * share the GPU instead of paying their own launches and tails.  Results
 * equal those of cg_sketch_csr on each instance (S X bit for bit; the
 * contraction up to its summation order, which depends on the tuning).   */
typedef struct cg_instance {
  /* set by the caller */
  const int32_t* row_ptr;   /* device int32[n+1]                            */
  const int32_t* col_idx;   /* device int32[nnz] (may be NULL if nnz == 0)  */
  const float* vals;        /* device float[nnz] (may be NULL if nnz == 0)  */
  float* Y;                 /* device float[m*d], overwritten               */
  int64_t n, d, nnz, m, B;  /* as for cg_sketch_csr                         */
  uint64_t seed;            /* this instance's transform                   */
  int64_t row_offset;       /* global index of row 0                        */
  /* set by cg_batched_plan; leave them as planned */
  int64_t ws_off;           /* byte offset of its scratch in the workspace  */
  int64_t tile_rows;        /* rows per S X work item                       */
  int32_t tiles;            /* S X work items (row tiles)                   */
  int32_t ranges;           /* bucket ranges of 2^bp_shift buckets          */
  int32_t bp_shift;
  int32_t kc;               /* columns of G per contraction wavefront
                               (rows route: rows of X per wavefront)     */
  int32_t parts;            /* contraction splits along B (4 kc columns)    */
  int32_t gsx_items;        /* contraction work items                       */
  int32_t red_items;        /* split-reduction work items                   */
  int32_t first_tile;       /* its first item in each phase's queue (the
                               contraction queue holds the instances of each
                               MFMA width, ceil(d/16) up to 4 blocks of 16
                               columns, together, in increasing width)    */
  int32_t first_range;
  int32_t first_gsx;
  int32_t first_red;
  int32_t route;            /* 0: S X then G (S X); 1: rows route (no S X,
                               see CG_SX_ROWS): no tiles or ranges, and its
                               parts split the rows, 4 kc per part       */
} cg_instance;

/*
 * Plan a batch: validate every instance, choose its route (the rows route
 * where the cost model of CG_SX_AUTO puts it below the S X route) and its
 * tile shapes from the tuning table (by the class ceil(log2 d) of its d),
 * and fill the planning fields of inst (host array of count entries,
 * in/out).  *workspace_bytes
 * receives the workspace cg_sketch_batched needs.  Host only; queues
 * nothing.  Errors: CG_EINVAL / CG_EUNSUPPORTED, the message naming the
 * instance (e.g. d too large for the binned S X, a NULL pointer).
 */
int cg_batched_plan(cg_instance* inst, int32_t count, const cg_opts* opts,
                    size_t* workspace_bytes);

/*
 * Compute every instance's Y.  inst is the table cg_batched_plan filled
 * (unchanged since, with the tuning table unchanged; else CG_EINVAL); it is
 * copied to the workspace on opts->stream, so it must stay valid until the
 * stream has passed this call.  opts is required (workspace of at least
 * the planned size, 256-byte aligned; precision must be native; sx_algo,
 * kc and row_offset of opts are ignored: each instance has its own).
 * Instances must not share a Y.  Errors as for cg_sketch_csr.
 */
int cg_sketch_batched(const cg_instance* inst, int32_t count,
                      const cg_opts* opts);

/*
 * Tuning table of the batched planner, one entry per d class c =
 * ceil(log2 d), c = 0 .. 10: rows_per_item[c] (rows per S X work item, a
 * multiple of 1024 in [1024, 2^24]) and kc_per_item[c] (columns of G per
 * contraction wavefront, a multiple of 16 in [16, 2^20]) for the first
 * `classes` classes.  A NULL array leaves that column unchanged; both NULL
 * restore the built-in table (16384 rows, kc 512).  Host only; plans made
 * before a change no longer match (cg_sketch_batched rejects them).
 */
int cg_set_tuning(const int32_t* rows_per_item, const int32_t* kc_per_item,
                  int32_t classes);

/* Read the first `classes` entries of the tuning table (NULL: skipped). */
int cg_get_tuning(int32_t* rows_per_item, int32_t* kc_per_item, int32_t classes);

/* ---- test access to the random source ---------------------------------- */

/* Memory ceilings for the rooflines: a device copy of `bytes` (src to
 * dst), a read of src (dst receives 8192 uint32 checksums), or a write of
 * dst, with 16-byte accesses on consecutive addresses over 8192
 * workgroups.  bytes: a positive multiple of 16; pointers 16-byte aligned
 * device memory.  stream: hipStream_t.                                    */
#define CG_STREAM_COPY 0
#define CG_STREAM_READ 1
#define CG_STREAM_WRITE 2
#define CG_STREAM_COPY_NT 3    /* the same with non-temporal accesses   */
#define CG_STREAM_READ_NT 4
#define CG_STREAM_WRITE_NT 5
int cg_debug_stream(int kind, const void* src, void* dst, int64_t bytes,
                    void* stream);

/* The generator's ceiling for the contraction rooflines: draws the m x B
 * normals of G (columns 0 .. B-1, rows 0 .. m-1, the counters and FP32
 * Box-Muller the contractions use; Section 1.1's G) and nothing else; each
 * of CG_NORMALS_SINK threads writes the sum of its normals to sink[t].
 * m: a positive multiple of 4 up to 2^24; 1 <= B < 2^31.  sink: device
 * float[CG_NORMALS_SINK].  stream: hipStream_t.                           */
#define CG_NORMALS_SINK (1 << 19)
int cg_debug_normals(uint64_t seed, int64_t m, int64_t B, float* sink,
                     void* stream);

/* out[4k..4k+3] = Philox4x32-10(counter ctr[4k..4k+3], key(seed)) for
 * k < count.  ctr, out: device uint32 arrays.  stream: hipStream_t. */
int cg_debug_philox(uint64_t seed, const uint32_t* ctr, int64_t count,
                    uint32_t* out, void* stream);

/* Bucket h and sign sigma (+1/-1) of global rows row0 .. row0+count-1.
 * h: device uint32[count]; sigma: device int8[count]. */
int cg_debug_hash(uint64_t seed, int64_t B, uint64_t row0, int64_t count,
                  uint32_t* h, int8_t* sigma, void* stream);

/* Columns b0 .. b0+nb-1 of G (m x B), written as device dtype[m*nb]
 * row-major; FP32 values are what the FP32 contraction uses. */
int cg_debug_gaussian(uint64_t seed, int64_t m, int64_t b0, int64_t nb,
                      int dtype, void* G, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* COUNTGAUSS_H */
