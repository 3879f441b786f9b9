// C ABI of libcountgauss.so: argument validation, workspace layout and
// dispatch to the kernels.  Nothing here allocates device memory or waits
// for the device; every error is reported before the first launch.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "countgauss.h"
#include "cg_internal.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace

namespace cg {
void set_last_error(const char* msg) { g_last_error = msg; }
}  // namespace cg

namespace {

int hip_fail(hipError_t e, const char* where) {
  return fail(CG_EHIP, "%s: %s", where, hipGetErrorString(e));
}

struct Opts {
  int precision = CG_PREC_NATIVE;
  int sx_algo = CG_SX_AUTO;
  int kc = 0;
  hipStream_t stream = nullptr;
  void* workspace = nullptr;
  size_t workspace_bytes = 0;
  int64_t row_offset = 0;
  void* sx_out = nullptr;
  void* const* events = nullptr;
};

// A NULL entry skips its boundary (each recorded event costs a few
// microseconds of idle GPU between the kernels it separates).
int record(const Opts& o, int i) {
  if (!o.events || !o.events[i]) return CG_OK;
  hipError_t e = hipEventRecord((hipEvent_t)o.events[i], o.stream);
  return e == hipSuccess ? CG_OK : hip_fail(e, "hipEventRecord(stage event)");
}

int read_opts(const cg_opts* o, Opts* out) {
  *out = Opts();
  if (!o) return CG_OK;
  if (o->struct_size < sizeof(cg_opts))
    return fail(CG_EINVAL, "cg_opts.struct_size %u < %zu", o->struct_size, sizeof(cg_opts));
  out->precision = o->precision;
  out->sx_algo = o->sx_algo;
  out->kc = o->kc;
  out->stream = (hipStream_t)o->stream;
  out->workspace = o->workspace;
  out->workspace_bytes = o->workspace_bytes;
  out->row_offset = o->row_offset;
  out->sx_out = o->sx_out;
  out->events = o->stage_events;
  if (out->precision < CG_PREC_NATIVE || out->precision > CG_PREC_FP8)
    return fail(CG_EINVAL, "unknown precision %d", out->precision);
  if (out->sx_algo < CG_SX_AUTO || out->sx_algo > CG_SX_FUSED)
    return fail(CG_EINVAL, "unknown sx_algo %d", out->sx_algo);
  if (out->kc < 0 || out->kc % 16 != 0 || out->kc > (1 << 20))
    return fail(CG_EINVAL, "kc %d must be 0 or a positive multiple of 16 up to 2^20", out->kc);
  if (out->row_offset < 0) return fail(CG_EINVAL, "row_offset %lld < 0", (long long)out->row_offset);
  if (out->workspace && ((uintptr_t)out->workspace & 255))
    return fail(CG_EINVAL, "workspace must be 256-byte aligned");
  return CG_OK;
}

size_t elem_size(int dtype) { return dtype == CG_DTYPE_F64 ? 8 : 4; }

cg::Prec to_prec(int p) {
  return p == CG_PREC_BF16 ? cg::Prec::BF16 : p == CG_PREC_FP8 ? cg::Prec::FP8 : cg::Prec::Native;
}

int check_shape(int dtype, int64_t n, int64_t d, int64_t m, int64_t B, const Opts& o) {
  if (dtype != CG_DTYPE_F32 && dtype != CG_DTYPE_F64) return fail(CG_EINVAL, "unknown dtype %d", dtype);
  if (n < 1) return fail(CG_EINVAL, "n = %lld < 1", (long long)n);
  if (d < 1) return fail(CG_EINVAL, "d = %lld < 1", (long long)d);
  if (m < 1) return fail(CG_EINVAL, "m = %lld < 1", (long long)m);
  if (B < 1 || B > 0x7fffffffLL) return fail(CG_EINVAL, "B = %lld outside [1, 2^31)", (long long)B);
  if (d > cg::kMaxD) return fail(CG_EUNSUPPORTED, "d = %lld > %d", (long long)d, cg::kMaxD);
  if (m > 64LL * 65535) return fail(CG_EUNSUPPORTED, "m = %lld > %d", (long long)m, 64 * 65535);
  // (row-parallel grids stay below 2^32 work-items)
  if (n > (1LL << 33)) return fail(CG_EUNSUPPORTED, "n = %lld > 2^33", (long long)n);
  if (dtype == CG_DTYPE_F64 && o.precision != CG_PREC_NATIVE)
    return fail(CG_EINVAL, "FP64 data supports only native precision");
  if ((double)B * (double)d > 4e12) return fail(CG_EUNSUPPORTED, "B * d too large");
  return CG_OK;
}

// The algorithm a call runs: AUTO resolves to ROWS for FP32 CSR data at
// native precision without sx_out where the cost model favours it, else to
// BINNED for FP32 data whose bucket ranges fit, else ATOMIC.  BINNED asked
// for where it does not apply is -1, ROWS likewise -2 (errors).
constexpr int kNoBinned = -1, kNoRows = -2, kNoFused = -3;

int resolve_algo(int dtype, bool csr, int64_t n, int64_t d, int64_t nnz, int64_t m, int64_t B,
                 const Opts& o) {
  const bool rows_ok = csr && dtype == CG_DTYPE_F32 && o.precision == CG_PREC_NATIVE && !o.sx_out;
  if (o.sx_algo == CG_SX_ROWS) return rows_ok ? CG_SX_ROWS : kNoRows;
  const bool fits = dtype == CG_DTYPE_F32 && cg::bin_geometry(csr, n, (int)d, B).ok;
  if (o.sx_algo == CG_SX_FUSED) return rows_ok && fits ? CG_SX_FUSED : kNoFused;
  if (o.sx_algo == CG_SX_AUTO) {
    if (rows_ok && cg::rows_route_pays(n, d, nnz, m, B)) return CG_SX_ROWS;
    return fits ? CG_SX_BINNED : CG_SX_ATOMIC;
  }
  if (o.sx_algo == CG_SX_BINNED && !fits) return kNoBinned;
  return o.sx_algo;
}

int algo_fail(int algo, bool csr) {
  if (algo == kNoRows)
    return fail(CG_EUNSUPPORTED, "the rows route needs FP32 CSR data, native precision and no sx_out");
  if (algo == kNoFused)
    return fail(CG_EUNSUPPORTED, "the fused pass needs FP32 CSR data, native precision, no sx_out "
                                 "and at most %d bucket ranges", cg::kBinMaxRangesCsr);
  return fail(CG_EUNSUPPORTED, csr ? "binned S X needs FP32 data and at most %d bucket ranges"
                                   : "binned S X needs FP32 data, d <= 64 and at most %d bucket ranges",
              csr ? cg::kBinMaxRangesCsr : cg::kBinMaxRangesDense);
}

// Forward workspace: [S X unless sx_out or ROWS][split partials][FP8 block scales][S X scratch]
struct FwdLayout {
  cg::GsxPlan plan;
  int algo = CG_SX_ATOMIC;
  size_t sx = 0, part = 0, scale = 0, scratch = 0, total = 0;
};

FwdLayout forward_layout(int dtype, bool csr, int64_t n, int64_t d, int64_t nnz, int64_t m,
                         int64_t B, const Opts& o) {
  FwdLayout L;
  const size_t es = elem_size(dtype);
  L.algo = resolve_algo(dtype, csr, n, d, nnz, m, B, o);
  L.plan = cg::plan_gsx(m, B, d, to_prec(o.precision), o.kc, es);
  if (L.algo == CG_SX_ROWS) {
    L.plan.parts = cg::rows_parts(n, cg::rows_per_wave(n));
    L.part = 0;
    L.total = cg::align256((size_t)L.plan.parts * m * d * es);
    return L;
  }
  if (L.algo == CG_SX_FUSED) {
    // [one partial per bucket range][binned scratch]; no S X
    const cg::BinGeom g = cg::bin_geometry(true, n, (int)d, B);
    L.plan.parts = g.R;
    L.part = 0;
    L.scratch = cg::align256((size_t)g.R * m * d * es);
    L.total = L.scratch + cg::align256(cg::binned_scratch_bytes(g, nnz));
    return L;
  }
  const size_t sx_bytes = o.sx_out ? 0 : cg::align256((size_t)B * d * es);
  const size_t part_bytes = cg::align256((size_t)L.plan.parts * m * d * es);
  size_t scratch_bytes = 0;
  if (L.algo == CG_SX_SORTED)
    scratch_bytes = cg::align256(
        cg::sorted_scratch_bytes(csr ? nnz : n, B, cg::sorted_payload_bytes(csr, es)));
  else if (L.algo == CG_SX_BINNED)
    scratch_bytes = cg::align256(
        cg::binned_scratch_bytes(cg::bin_geometry(csr, n, (int)d, B), csr ? nnz : n));
  // FP8: one pair of power-of-two scales per 128-row block of S X
  const size_t scale_bytes = o.precision == CG_PREC_FP8 ? cg::fp8_scale_bytes(B) : 0;
  L.sx = 0;
  L.part = sx_bytes;
  L.scale = sx_bytes + part_bytes;
  L.scratch = L.scale + scale_bytes;
  L.total = L.scratch + scratch_bytes;
  return L;
}

int check_workspace(const Opts& o, size_t need) {
  if (need == 0) return CG_OK;
  if (!o.workspace || o.workspace_bytes < need)
    return fail(CG_ENOSPACE, "workspace of %zu bytes needed, %zu given", need,
                o.workspace ? o.workspace_bytes : (size_t)0);
  return CG_OK;
}

template <typename T>
int forward_typed(const int32_t* row_ptr, const int32_t* col_idx, const T* X, int64_t ldx,
                  bool csr, int64_t n, int64_t d, int64_t nnz, int64_t m, int64_t B,
                  uint64_t seed, T* Y, const Opts& o, const FwdLayout& L) {
  char* ws = (char*)o.workspace;
  T* SX = o.sx_out ? (T*)o.sx_out : (T*)(ws + L.sx);
  T* part = (T*)(ws + L.part);
  const cg::Key key = cg::key_of(seed);
  const uint64_t off = (uint64_t)o.row_offset;
  hipError_t e;
  int st;
  if ((st = record(o, 0))) return st;
  if (L.algo == CG_SX_ROWS) {
    if constexpr (sizeof(T) == 4) {
      if ((st = record(o, 1))) return st;
      if ((st = record(o, 2))) return st;
      cg::GsxArgs a{};
      a.part = part;
      a.B = B;
      a.d = (int32_t)d;
      a.m = (int32_t)m;
      a.key = key;
      a.row_ptr = row_ptr;
      a.col_idx = col_idx;
      a.vals = X;
      a.n = n;
      a.row_offset = off;
      a.nnz = (int32_t)nnz;
      a.route = 1;
      e = cg::launch_rows_partials(a, o.stream);
      if (e != hipSuccess) return hip_fail(e, "rows route");
      if ((st = record(o, 3))) return st;
      e = cg::launch_splitk_reduce<T>(part, L.plan.parts, m * d, Y, o.stream);
      if (e != hipSuccess) return hip_fail(e, "split reduction");
      return record(o, 4);
    }
  }
  if (L.algo == CG_SX_FUSED) {
    if constexpr (sizeof(T) == 4) {
      e = cg::launch_sx_fused_csr(row_ptr, col_idx, X, n, nnz, (int)d, (uint32_t)B, key, off,
                                  (int)m, part, ws + L.scratch, o.stream, o.events);
      if (e != hipSuccess) return hip_fail(e, "fused S X and G (S X)");
      if ((st = record(o, 3))) return st;
      e = cg::launch_splitk_reduce<T>(part, L.plan.parts, m * d, Y, o.stream);
      if (e != hipSuccess) return hip_fail(e, "split reduction");
      return record(o, 4);
    }
  }
  bool scales_ready = false;   // FP8 block scales already written by the S X reduce
  if (L.algo == CG_SX_BINNED) {
    if constexpr (sizeof(T) == 4) {
      void* scratch = ws + L.scratch;
      float2* fs = nullptr;
      if (o.precision == CG_PREC_FP8 && cg::binned_emits_fp8_scales(csr, n, (int)d, B)) {
        fs = (float2*)(ws + L.scale);
        scales_ready = true;
      }
      e = csr ? cg::launch_sx_binned_csr(row_ptr, col_idx, X, n, nnz, (int)d, (uint32_t)B, key, off,
                                         SX, scratch, o.stream, o.events, fs)
              : cg::launch_sx_binned_dense(X, ldx, n, (int)d, (uint32_t)B, key, off, SX, scratch,
                                           o.stream, o.events, fs);
      if (e != hipSuccess) return hip_fail(e, "binned S X");
    }
  } else if (L.algo == CG_SX_SORTED) {
    if ((st = record(o, 1))) return st;
    void* scratch = ws + L.scratch;
    e = csr ? cg::launch_sx_csr_sorted<T>(row_ptr, col_idx, X, n, nnz, (int)d, (uint32_t)B, key,
                                          off, SX, scratch, o.stream)
            : cg::launch_sx_dense_sorted<T>(X, ldx, n, (int)d, (uint32_t)B, key, off, SX, scratch,
                                            o.stream);
    if (e != hipSuccess) return hip_fail(e, "sorted S X");
  } else {
    e = cg::launch_fill_zero<T>(SX, (size_t)B * d, o.stream);
    if (e != hipSuccess) return hip_fail(e, "zero S X");
    if ((st = record(o, 1))) return st;
    e = csr ? cg::launch_sx_csr_atomic<T>(row_ptr, col_idx, X, n, nnz, (int)d, (uint32_t)B, key,
                                          off, SX, o.stream)
            : cg::launch_sx_dense_atomic<T>(X, ldx, n, (int)d, (uint32_t)B, key, off, SX,
                                            o.stream);
    if (e != hipSuccess) return hip_fail(e, "atomic S X");
  }
  if ((st = record(o, 2))) return st;
  e = cg::launch_gsx_partials<T>(L.plan, to_prec(o.precision), SX, B, (int)d, (int)m, key, part,
                                 o.stream, ws + L.scale, scales_ready);
  if (e != hipSuccess) return hip_fail(e, "G (S X)");
  if ((st = record(o, 3))) return st;
  e = cg::launch_splitk_reduce<T>(part, L.plan.parts, m * d, Y, o.stream);
  if (e != hipSuccess) return hip_fail(e, "split reduction");
  return record(o, 4);
}

// Dense Gaussian product G~ X: split partials over the rows of X.
cg::GsxPlan gaussian_dense_plan(int dtype, int64_t n, int64_t d, int64_t m, const Opts& o) {
  return cg::plan_gsx(m, n, d, cg::Prec::Native, o.kc, elem_size(dtype));
}
size_t gaussian_dense_bytes(int dtype, int64_t n, int64_t d, int64_t m, const Opts& o) {
  const cg::GsxPlan pl = gaussian_dense_plan(dtype, n, d, m, o);
  return cg::align256((size_t)pl.parts * m * d * elem_size(dtype));
}
int check_gaussian_dense(const void* X, int64_t ldx, int dtype, int64_t n, int64_t d, int64_t m,
                         const Opts& o) {
  int st = check_shape(dtype, n, d, m, 1, o);
  if (st) return st;
  if (o.precision != CG_PREC_NATIVE) return fail(CG_EINVAL, "the dense Gaussian product supports native precision only");
  if (n > 0x7fffffffLL) return fail(CG_EUNSUPPORTED, "n = %lld >= 2^31", (long long)n);
  if (ldx < d) return fail(CG_EINVAL, "ldx = %lld < d = %lld", (long long)ldx, (long long)d);
  if (!X) return fail(CG_EINVAL, "null pointer argument");
  return CG_OK;
}

// G~ X for validated arguments, workspace of gaussian_dense_bytes.
int run_gaussian_dense(const void* X, int64_t ldx, int dtype, int64_t n, int64_t d, int64_t m,
                       uint64_t seed, void* Y, const Opts& o) {
  const cg::GsxPlan pl = gaussian_dense_plan(dtype, n, d, m, o);
  const cg::Key key = cg::key_of(seed);
  const uint64_t off = (uint64_t)o.row_offset;
  hipError_t e;
  if (dtype == CG_DTYPE_F64) {
    double* part = (double*)o.workspace;
    e = cg::launch_dense_gaussian_partials<double>(pl, (const double*)X, ldx, n, (int)d, (int)m, key,
                                                   off, part, o.stream);
    if (e == hipSuccess) e = cg::launch_splitk_reduce<double>(part, pl.parts, m * d, (double*)Y, o.stream);
  } else {
    float* part = (float*)o.workspace;
    e = cg::launch_dense_gaussian_partials<float>(pl, (const float*)X, ldx, n, (int)d, (int)m, key,
                                                  off, part, o.stream);
    if (e == hipSuccess) e = cg::launch_splitk_reduce<float>(part, pl.parts, m * d, (float*)Y, o.stream);
  }
  return e == hipSuccess ? CG_OK : hip_fail(e, "dense Gaussian product");
}

size_t gaussian_csr_bytes(int64_t n, int64_t d, int64_t m) {
  return cg::align256((size_t)cg::rows_parts(n, cg::rows_per_wave(n)) * m * d * 4);
}

// Workspace of cg_anchors_dense: Z (m x d) then the projection's own.
int anchors_bytes(int proj, int dtype, int64_t n, int64_t d, int64_t m, int64_t B, const Opts& o,
                  size_t* out) {
  const size_t zb = cg::align256((size_t)m * d * elem_size(dtype));
  if (proj == CG_PROJ_COUNTGAUSS) {
    int st = check_shape(dtype, n, d, m, B, o);
    if (st) return st;
    const FwdLayout L = forward_layout(dtype, false, n, d, 0, m, B, o);
    if (L.algo < 0) return algo_fail(L.algo, false);
    *out = zb + L.total;
  } else {
    int st = check_shape(dtype, n, d, m, 1, o);
    if (st) return st;
    *out = zb + gaussian_dense_bytes(dtype, n, d, m, o);
  }
  return CG_OK;
}

}  // namespace

extern "C" {

void cg_opts_init(cg_opts* opts) {
  if (!opts) return;
  memset(opts, 0, sizeof *opts);
  opts->struct_size = sizeof *opts;
}

int cg_version(void) { return 100; }

const char* cg_status_string(int status) {
  switch (status) {
    case CG_OK: return "CG_OK";
    case CG_EINVAL: return "CG_EINVAL (invalid argument)";
    case CG_ENOSPACE: return "CG_ENOSPACE (workspace too small)";
    case CG_EUNSUPPORTED: return "CG_EUNSUPPORTED (outside what the library supports)";
    case CG_EHIP: return "CG_EHIP (HIP runtime error)";
    default: return "unknown status";
  }
}

size_t cg_last_error(char* buf, size_t len) {
  if (buf && len) {
    const size_t k = g_last_error.size() < len - 1 ? g_last_error.size() : len - 1;
    memcpy(buf, g_last_error.data(), k);
    buf[k] = 0;
  }
  return g_last_error.size();
}

int cg_workspace_bytes(int kind, int dtype, int64_t n, int64_t d, int64_t m, int64_t B,
                       int64_t nnz, const cg_opts* opts, size_t* bytes) {
  Opts o;
  int st = read_opts(opts, &o);
  if (st) return st;
  if (!bytes) return fail(CG_EINVAL, "bytes is NULL");
  if ((st = check_shape(dtype, n, d, m, B, o))) return st;
  switch (kind) {
    case CG_KIND_CSR:
      if (nnz < 0) return fail(CG_EINVAL, "nnz = %lld < 0", (long long)nnz);
      {
        const FwdLayout L = forward_layout(dtype, true, n, d, nnz, m, B, o);
        if (L.algo < 0) return algo_fail(L.algo, true);
        *bytes = L.total;
      }
      return CG_OK;
    case CG_KIND_DENSE:
      {
        const FwdLayout L = forward_layout(dtype, false, n, d, 0, m, B, o);
        if (L.algo < 0) return algo_fail(L.algo, false);
        *bytes = L.total;
      }
      return CG_OK;
    case CG_KIND_ADJOINT:
    case CG_KIND_ADJOINT_CSR:
      *bytes = cg::align256((size_t)B * d * elem_size(dtype));
      return CG_OK;
    case CG_KIND_GAUSSIAN_DENSE:
      *bytes = gaussian_dense_bytes(dtype, n, d, m, o);
      return CG_OK;
    case CG_KIND_GAUSSIAN_CSR:
      if (nnz < 0) return fail(CG_EINVAL, "nnz = %lld < 0", (long long)nnz);
      *bytes = gaussian_csr_bytes(n, d, m);
      return CG_OK;
    case CG_KIND_ANCHORS_COUNTGAUSS:
      return anchors_bytes(CG_PROJ_COUNTGAUSS, dtype, n, d, m, B, o, bytes);
    case CG_KIND_ANCHORS_GAUSSIAN:
      return anchors_bytes(CG_PROJ_GAUSSIAN, dtype, n, d, m, B, o, bytes);
    case CG_KIND_LEMMA:
      if (d > cg::kLemmaMaxD) return fail(CG_EUNSUPPORTED, "d = %lld > %d", (long long)d, cg::kLemmaMaxD);
      *bytes = cg::lemma_workspace_bytes(m, B, d, true);
      return CG_OK;
    default:
      return fail(CG_EINVAL, "unknown workspace kind %d", kind);
  }
}

int cg_sketch_csr(const int32_t* row_ptr, const int32_t* col_idx, const void* vals, int dtype,
                  int64_t n, int64_t d, int64_t nnz, int64_t m, int64_t B, uint64_t seed, void* Y,
                  const cg_opts* opts) {
  Opts o;
  int st = read_opts(opts, &o);
  if (st) return st;
  if ((st = check_shape(dtype, n, d, m, B, o))) return st;
  if (nnz < 0) return fail(CG_EINVAL, "nnz = %lld < 0", (long long)nnz);
  if (nnz > 0x7fffffffLL) return fail(CG_EUNSUPPORTED, "nnz = %lld >= 2^31 with int32 indices", (long long)nnz);
  if (!row_ptr || !Y || (nnz > 0 && (!col_idx || !vals)))
    return fail(CG_EINVAL, "null pointer argument");
  if (o.sx_algo == CG_SX_SORTED && n > 0x7fffffffLL)
    return fail(CG_EUNSUPPORTED, "sorted S X needs n < 2^31");
  const FwdLayout L = forward_layout(dtype, true, n, d, nnz, m, B, o);
  if (L.algo < 0) return algo_fail(L.algo, true);
  if ((st = check_workspace(o, L.total))) return st;
  if (dtype == CG_DTYPE_F64)
    return forward_typed<double>(row_ptr, col_idx, (const double*)vals, 0, true, n, d, nnz, m, B,
                                 seed, (double*)Y, o, L);
  return forward_typed<float>(row_ptr, col_idx, (const float*)vals, 0, true, n, d, nnz, m, B, seed,
                              (float*)Y, o, L);
}

int cg_sketch_dense(const void* X, int64_t ldx, int dtype, int64_t n, int64_t d, int64_t m,
                    int64_t B, uint64_t seed, void* Y, const cg_opts* opts) {
  Opts o;
  int st = read_opts(opts, &o);
  if (st) return st;
  if ((st = check_shape(dtype, n, d, m, B, o))) return st;
  if (ldx < d) return fail(CG_EINVAL, "ldx = %lld < d = %lld", (long long)ldx, (long long)d);
  if (!X || !Y) return fail(CG_EINVAL, "null pointer argument");
  if (o.sx_algo == CG_SX_SORTED && n > 0x7fffffffLL)
    return fail(CG_EUNSUPPORTED, "sorted S X needs n < 2^31");
  const FwdLayout L = forward_layout(dtype, false, n, d, 0, m, B, o);
  if (L.algo < 0) return algo_fail(L.algo, false);
  if ((st = check_workspace(o, L.total))) return st;
  if (dtype == CG_DTYPE_F64)
    return forward_typed<double>(nullptr, nullptr, (const double*)X, ldx, false, n, d, 0, m, B,
                                 seed, (double*)Y, o, L);
  return forward_typed<float>(nullptr, nullptr, (const float*)X, ldx, false, n, d, 0, m, B, seed,
                              (float*)Y, o, L);
}

int cg_sketch_adjoint(const void* dY, int dtype, int64_t n, int64_t d, int64_t m, int64_t B,
                      uint64_t seed, void* dX, int64_t lddx, const cg_opts* opts) {
  Opts o;
  int st = read_opts(opts, &o);
  if (st) return st;
  if ((st = check_shape(dtype, n, d, m, B, o))) return st;
  if (o.precision != CG_PREC_NATIVE) return fail(CG_EINVAL, "adjoint supports native precision only");
  if (lddx < d) return fail(CG_EINVAL, "lddx = %lld < d = %lld", (long long)lddx, (long long)d);
  if (!dY || !dX) return fail(CG_EINVAL, "null pointer argument");
  const size_t need = cg::align256((size_t)B * d * elem_size(dtype));
  if ((st = check_workspace(o, need))) return st;
  const cg::Key key = cg::key_of(seed);
  hipError_t e;
  if (dtype == CG_DTYPE_F64) {
    double* Z = (double*)o.workspace;
    e = cg::launch_gt_dy<double>((const double*)dY, (int)m, (int)d, B, key, Z, o.stream);
    if (e == hipSuccess)
      e = cg::launch_gather_dense<double>(Z, n, (int)d, (uint32_t)B, key, (uint64_t)o.row_offset,
                                          (double*)dX, lddx, o.stream);
  } else {
    float* Z = (float*)o.workspace;
    e = cg::launch_gt_dy<float>((const float*)dY, (int)m, (int)d, B, key, Z, o.stream);
    if (e == hipSuccess)
      e = cg::launch_gather_dense<float>(Z, n, (int)d, (uint32_t)B, key, (uint64_t)o.row_offset,
                                         (float*)dX, lddx, o.stream);
  }
  if (e != hipSuccess) return hip_fail(e, "adjoint");
  return CG_OK;
}

int cg_sketch_adjoint_csr(const int32_t* row_ptr, const int32_t* col_idx, int64_t nnz,
                          const void* dY, int dtype, int64_t n, int64_t d, int64_t m, int64_t B,
                          uint64_t seed, void* dvals, const cg_opts* opts) {
  Opts o;
  int st = read_opts(opts, &o);
  if (st) return st;
  if ((st = check_shape(dtype, n, d, m, B, o))) return st;
  if (o.precision != CG_PREC_NATIVE) return fail(CG_EINVAL, "adjoint supports native precision only");
  if (nnz < 0) return fail(CG_EINVAL, "nnz = %lld < 0", (long long)nnz);
  if (nnz > 0x7fffffffLL) return fail(CG_EUNSUPPORTED, "nnz = %lld >= 2^31 with int32 indices", (long long)nnz);
  if (!row_ptr || !dY || (nnz > 0 && (!col_idx || !dvals)))
    return fail(CG_EINVAL, "null pointer argument");
  const size_t need = cg::align256((size_t)B * d * elem_size(dtype));
  if ((st = check_workspace(o, need))) return st;
  const cg::Key key = cg::key_of(seed);
  hipError_t e;
  if (dtype == CG_DTYPE_F64) {
    double* Z = (double*)o.workspace;
    e = cg::launch_gt_dy<double>((const double*)dY, (int)m, (int)d, B, key, Z, o.stream);
    if (e == hipSuccess)
      e = cg::launch_gather_csr<double>(row_ptr, col_idx, Z, n, nnz, (int)d, (uint32_t)B, key,
                                        (uint64_t)o.row_offset, (double*)dvals, o.stream);
  } else {
    float* Z = (float*)o.workspace;
    e = cg::launch_gt_dy<float>((const float*)dY, (int)m, (int)d, B, key, Z, o.stream);
    if (e == hipSuccess)
      e = cg::launch_gather_csr<float>(row_ptr, col_idx, Z, n, nnz, (int)d, (uint32_t)B, key,
                                       (uint64_t)o.row_offset, (float*)dvals, o.stream);
  }
  if (e != hipSuccess) return hip_fail(e, "adjoint (CSR)");
  return CG_OK;
}

}  // extern "C"

// ---- allocation-free forward (CSR) --------------------------------------
// Its workspace is this file-scope device array: every GPU the library runs
// on holds one copy until the process ends.  In host code the name is only
// a stand-in for the symbol; the device address of each GPU's copy comes
// from hipGetSymbolAddress with that GPU current, once, and only that
// address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[CG_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(CG_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(static scratch)");
    if (!p || ((uintptr_t)p & 255)) return fail(CG_EHIP, "static scratch has no 256-byte aligned address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CG_OK;
}

}  // namespace

extern "C" {

int cg_sketch_csr_noalloc(const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                          int dtype, int64_t n, int64_t d, int64_t nnz, int64_t m, int64_t B,
                          uint64_t seed, void* Y, const cg_opts* opts) {
  Opts o;
  int st = read_opts(opts, &o);
  if (st) return st;
  if ((st = check_shape(dtype, n, d, m, B, o))) return st;
  if (nnz < 0) return fail(CG_EINVAL, "nnz = %lld < 0", (long long)nnz);
  if (nnz > 0x7fffffffLL) return fail(CG_EUNSUPPORTED, "nnz = %lld >= 2^31 with int32 indices", (long long)nnz);
  if (!row_ptr || !Y || (nnz > 0 && (!col_idx || !vals)))
    return fail(CG_EINVAL, "null pointer argument");
  if (o.sx_algo == CG_SX_SORTED && n > 0x7fffffffLL)
    return fail(CG_EUNSUPPORTED, "sorted S X needs n < 2^31");
  const FwdLayout L = forward_layout(dtype, true, n, d, nnz, m, B, o);
  if (L.algo < 0) return algo_fail(L.algo, true);
  if (L.total > (size_t)CG_NOALLOC_SCRATCH_BYTES)
    return fail(CG_ENOSPACE, "this call needs %zu bytes of scratch; the static buffer holds %zu",
                L.total, (size_t)CG_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((st = scratch_of_current_device(&ws))) return st;
  o.workspace = ws;
  o.workspace_bytes = (size_t)CG_NOALLOC_SCRATCH_BYTES;
  if (dtype == CG_DTYPE_F64)
    return forward_typed<double>(row_ptr, col_idx, (const double*)vals, 0, true, n, d, nnz, m, B,
                                 seed, (double*)Y, o, L);
  return forward_typed<float>(row_ptr, col_idx, (const float*)vals, 0, true, n, d, nnz, m, B, seed,
                              (float*)Y, o, L);
}

int cg_gaussian_dense(const void* X, int64_t ldx, int dtype, int64_t n, int64_t d, int64_t m,
                      uint64_t seed, void* Y, const cg_opts* opts) {
  Opts o;
  int st = read_opts(opts, &o);
  if (st) return st;
  if ((st = check_gaussian_dense(X, ldx, dtype, n, d, m, o))) return st;
  if (!Y) return fail(CG_EINVAL, "null pointer argument");
  if ((st = check_workspace(o, gaussian_dense_bytes(dtype, n, d, m, o)))) return st;
  return run_gaussian_dense(X, ldx, dtype, n, d, m, seed, Y, o);
}

int cg_row_extrema(const void* Z, int dtype, int64_t m, int64_t d, int64_t ldz, int32_t* imax,
                   int32_t* imin, void* stream) {
  if (dtype != CG_DTYPE_F32 && dtype != CG_DTYPE_F64) return fail(CG_EINVAL, "unknown dtype %d", dtype);
  if (m < 1 || d < 1) return fail(CG_EINVAL, "m = %lld, d = %lld: both must be >= 1", (long long)m, (long long)d);
  if (d > 0x7fffffffLL || m > (1LL << 40)) return fail(CG_EUNSUPPORTED, "Z too large");
  if (ldz < d) return fail(CG_EINVAL, "ldz = %lld < d = %lld", (long long)ldz, (long long)d);
  if (!Z || !imax || !imin) return fail(CG_EINVAL, "null pointer argument");
  const hipError_t e =
      dtype == CG_DTYPE_F64
          ? cg::launch_row_extrema<double>((const double*)Z, m, d, ldz, imax, imin, (hipStream_t)stream)
          : cg::launch_row_extrema<float>((const float*)Z, m, d, ldz, imax, imin, (hipStream_t)stream);
  return e == hipSuccess ? CG_OK : hip_fail(e, "row extrema");
}

int cg_anchors_dense(const void* X, int64_t ldx, int dtype, int64_t n, int64_t d, int64_t m,
                     int64_t B, uint64_t seed, int proj, int32_t* imax, int32_t* imin,
                     const cg_opts* opts) {
  Opts o;
  int st = read_opts(opts, &o);
  if (st) return st;
  if (proj != CG_PROJ_COUNTGAUSS && proj != CG_PROJ_GAUSSIAN)
    return fail(CG_EINVAL, "unknown projection %d", proj);
  if (!imax || !imin) return fail(CG_EINVAL, "null pointer argument");
  size_t need = 0;
  if ((st = anchors_bytes(proj, dtype, n, d, m, B, o, &need))) return st;
  if (proj == CG_PROJ_COUNTGAUSS) {
    if (ldx < d) return fail(CG_EINVAL, "ldx = %lld < d = %lld", (long long)ldx, (long long)d);
    if (!X) return fail(CG_EINVAL, "null pointer argument");
  } else if ((st = check_gaussian_dense(X, ldx, dtype, n, d, m, o))) {
    return st;
  }
  if ((st = check_workspace(o, need))) return st;
  // workspace: [Z = the projection, m x d][the projection's own workspace]
  const size_t zb = cg::align256((size_t)m * d * elem_size(dtype));
  void* Z = o.workspace;
  Opts inner = o;
  inner.workspace = (char*)o.workspace + zb;
  inner.workspace_bytes = o.workspace_bytes - zb;
  inner.events = nullptr;
  if (proj == CG_PROJ_COUNTGAUSS) {
    const FwdLayout L = forward_layout(dtype, false, n, d, 0, m, B, inner);
    st = dtype == CG_DTYPE_F64
             ? forward_typed<double>(nullptr, nullptr, (const double*)X, ldx, false, n, d, 0, m, B,
                                     seed, (double*)Z, inner, L)
             : forward_typed<float>(nullptr, nullptr, (const float*)X, ldx, false, n, d, 0, m, B,
                                    seed, (float*)Z, inner, L);
  } else {
    st = run_gaussian_dense(X, ldx, dtype, n, d, m, seed, Z, inner);
  }
  if (st) return st;
  const hipError_t e =
      dtype == CG_DTYPE_F64
          ? cg::launch_row_extrema<double>((const double*)Z, m, d, d, imax, imin, o.stream)
          : cg::launch_row_extrema<float>((const float*)Z, m, d, d, imax, imin, o.stream);
  return e == hipSuccess ? CG_OK : hip_fail(e, "row extrema");
}

int cg_gaussian_csr(const int32_t* row_ptr, const int32_t* col_idx, const void* vals, int dtype,
                    int64_t n, int64_t d, int64_t nnz, int64_t m, uint64_t seed, void* Y,
                    const cg_opts* opts) {
  Opts o;
  int st = read_opts(opts, &o);
  if (st) return st;
  if ((st = check_shape(dtype, n, d, m, 1, o))) return st;
  if (dtype != CG_DTYPE_F32) return fail(CG_EUNSUPPORTED, "the CSR dense Gaussian product needs FP32 data");
  if (o.precision != CG_PREC_NATIVE) return fail(CG_EINVAL, "the dense Gaussian product supports native precision only");
  if (nnz < 0) return fail(CG_EINVAL, "nnz = %lld < 0", (long long)nnz);
  if (nnz > 0x7fffffffLL) return fail(CG_EUNSUPPORTED, "nnz = %lld >= 2^31 with int32 indices", (long long)nnz);
  if (n > 0x7fffffffLL) return fail(CG_EUNSUPPORTED, "n = %lld >= 2^31", (long long)n);
  if (!row_ptr || !Y || (nnz > 0 && (!col_idx || !vals)))
    return fail(CG_EINVAL, "null pointer argument");
  const size_t need = gaussian_csr_bytes(n, d, m);
  if ((st = check_workspace(o, need))) return st;
  cg::GsxArgs a{};
  a.part = (float*)o.workspace;
  a.B = 1;
  a.d = (int32_t)d;
  a.m = (int32_t)m;
  a.key = cg::key_of(seed);
  a.row_ptr = row_ptr;
  a.col_idx = col_idx;
  a.vals = (const float*)vals;
  a.n = n;
  a.row_offset = (uint64_t)o.row_offset;
  a.nnz = (int32_t)nnz;
  a.route = 1;
  hipError_t e = cg::launch_rows_partials(a, o.stream, true);
  if (e == hipSuccess)
    e = cg::launch_splitk_reduce<float>(a.part, cg::rows_parts(n, cg::rows_per_wave(n)), m * d,
                                        (float*)Y, o.stream);
  if (e != hipSuccess) return hip_fail(e, "dense Gaussian product (CSR)");
  return CG_OK;
}

int cg_lemma_stats(const void* Y, const void* SU, int dtype, int64_t m, int64_t B, int64_t d,
                   double* stats, const cg_opts* opts) {
  Opts o;
  int st = read_opts(opts, &o);
  if (st) return st;
  if (dtype != CG_DTYPE_F32 && dtype != CG_DTYPE_F64) return fail(CG_EINVAL, "unknown dtype %d", dtype);
  if (m < 1 || d < 1 || (SU && B < 1))
    return fail(CG_EINVAL, "m = %lld, B = %lld, d = %lld: each must be >= 1", (long long)m,
                (long long)B, (long long)d);
  if (d > cg::kLemmaMaxD) return fail(CG_EUNSUPPORTED, "d = %lld > %d", (long long)d, cg::kLemmaMaxD);
  if (m > (1LL << 31) || (SU && B > (1LL << 31)))
    return fail(CG_EUNSUPPORTED, "m or B beyond 2^31 rows");
  if (!Y || !stats) return fail(CG_EINVAL, "null pointer argument");
  if ((st = check_workspace(o, cg::lemma_workspace_bytes(m, B, d, SU != nullptr)))) return st;
  const hipError_t e =
      dtype == CG_DTYPE_F64
          ? cg::launch_lemma_stats<double>((const double*)Y, (const double*)SU, m, B, (int)d,
                                           (double*)o.workspace, stats, o.stream)
          : cg::launch_lemma_stats<float>((const float*)Y, (const float*)SU, m, B, (int)d,
                                          (double*)o.workspace, stats, o.stream);
  return e == hipSuccess ? CG_OK : hip_fail(e, "Section 7 statistics");
}

int cg_debug_stream(int kind, const void* src, void* dst, int64_t bytes, void* stream) {
  if (kind < CG_STREAM_COPY || kind > CG_STREAM_WRITE_NT) return fail(CG_EINVAL, "unknown stream kind %d", kind);
  if (bytes < 16 || bytes % 16) return fail(CG_EINVAL, "bytes = %lld: a positive multiple of 16", (long long)bytes);
  if ((kind % 3 != CG_STREAM_WRITE && !src) || !dst) return fail(CG_EINVAL, "null pointer argument");
  if (((uintptr_t)src | (uintptr_t)dst) & 15) return fail(CG_EINVAL, "pointers must be 16-byte aligned");
  const hipError_t e = cg::launch_stream(kind, src, dst, bytes, (hipStream_t)stream);
  return e == hipSuccess ? CG_OK : hip_fail(e, "stream probe");
}

int cg_debug_normals(uint64_t seed, int64_t m, int64_t B, float* sink, void* stream) {
  if (m < 4 || m % 4 || m > (1LL << 24)) return fail(CG_EINVAL, "m = %lld: a positive multiple of 4 up to 2^24", (long long)m);
  if (B < 1 || B > 0x7fffffffLL) return fail(CG_EINVAL, "B = %lld outside [1, 2^31)", (long long)B);
  if (!sink) return fail(CG_EINVAL, "null pointer argument");
  if (cg::normals_threads() != CG_NORMALS_SINK) return fail(CG_EUNSUPPORTED, "sink size mismatch");
  const hipError_t e = cg::launch_normals_rate(cg::key_of(seed), m, B, sink, (hipStream_t)stream);
  return e == hipSuccess ? CG_OK : hip_fail(e, "normals probe");
}

int cg_debug_philox(uint64_t seed, const uint32_t* ctr, int64_t count, uint32_t* out,
                    void* stream) {
  if (count < 0 || count > (1LL << 30)) return fail(CG_EINVAL, "count %lld out of range", (long long)count);
  if (count > 0 && (!ctr || !out)) return fail(CG_EINVAL, "null pointer argument");
  hipError_t e = cg::launch_debug_philox(cg::key_of(seed), ctr, count, out, (hipStream_t)stream);
  return e == hipSuccess ? CG_OK : hip_fail(e, "debug philox");
}

int cg_debug_hash(uint64_t seed, int64_t B, uint64_t row0, int64_t count, uint32_t* h,
                  int8_t* sigma, void* stream) {
  if (B < 1 || B > 0x7fffffffLL) return fail(CG_EINVAL, "B = %lld outside [1, 2^31)", (long long)B);
  if (count < 0 || count > (1LL << 30)) return fail(CG_EINVAL, "count %lld out of range", (long long)count);
  if (count > 0 && (!h || !sigma)) return fail(CG_EINVAL, "null pointer argument");
  hipError_t e = cg::launch_debug_hash(cg::key_of(seed), (uint32_t)B, row0, count, h, sigma,
                                       (hipStream_t)stream);
  return e == hipSuccess ? CG_OK : hip_fail(e, "debug hash");
}

int cg_debug_gaussian(uint64_t seed, int64_t m, int64_t b0, int64_t nb, int dtype, void* G,
                      void* stream) {
  if (m < 1 || m > (1LL << 24)) return fail(CG_EINVAL, "m = %lld out of range", (long long)m);
  if (b0 < 0 || nb < 0 || b0 + nb > 0x7fffffffLL) return fail(CG_EINVAL, "column range out of [0, 2^31)");
  if ((m + 3) / 4 * nb > (1LL << 30)) return fail(CG_EINVAL, "m * nb too large");
  if (dtype != CG_DTYPE_F32 && dtype != CG_DTYPE_F64) return fail(CG_EINVAL, "unknown dtype %d", dtype);
  if (nb > 0 && !G) return fail(CG_EINVAL, "null pointer argument");
  const cg::Key key = cg::key_of(seed);
  hipError_t e = dtype == CG_DTYPE_F64
                     ? cg::launch_debug_gaussian<double>(key, m, b0, nb, (double*)G, (hipStream_t)stream)
                     : cg::launch_debug_gaussian<float>(key, m, b0, nb, (float*)G, (hipStream_t)stream);
  return e == hipSuccess ? CG_OK : hip_fail(e, "debug gaussian");
}

}  // extern "C"
