// Many independent CSR instances (each its own n, d, m, B and seed) in one
// pass of launches: every phase of the transform -- binned S X (count,
// scan, scatter, reduce), the MFMA contraction with in-register G, and the
// fixed-order split reduction -- is one launch over the work items of all
// instances, so small instances share the GPU instead of each paying its
// own launches and its own tail.
//
// Planning (host): each instance gets its tile shapes from the tuning table
// (rows per S X tile and G columns per contraction wavefront, per class of
// d), its item counts, its first item in each phase's queue and its
// scratch offset.  The launch copies the planned table into the workspace;
// a setup kernel turns it into per-instance kernel arguments and item ->
// instance tables; then the phases run.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "countgauss.h"
#include "cg_internal.hpp"

namespace cg {
namespace {

constexpr int kClasses = 11;   // d classes: ceil(log2 d) = 0 .. 10

struct Tuning {
  int32_t rows[kClasses];
  int32_t kc[kClasses];
};

Tuning default_tuning() {
  Tuning t;
  for (int c = 0; c < kClasses; ++c) {
    t.rows[c] = (int32_t)kBinTileRows;
    t.kc[c] = 512;
  }
  return t;
}

std::mutex g_tuning_mu;
Tuning g_tuning = default_tuning();

int failf(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_last_error(buf);
  return code;
}

int d_class(int64_t d) {
  int c = 0;
  while (c < kClasses - 1 && ((int64_t)1 << c) < d) ++c;
  return c;
}

// Workspace layout of a batch: header (table copy, kernel arguments, first
// items, item tables), then each instance's scratch at its ws_off.
struct Header {
  size_t table, bargs, gargs, firsts, tile_inst, range_inst, gsx_inst, red_inst, bytes;
};

Header header_layout(int32_t count, int64_t tiles, int64_t ranges, int64_t gsx, int64_t red) {
  Header h;
  size_t o = 0;
  h.table = o;
  o += align256((size_t)count * sizeof(cg_instance));
  h.bargs = o;
  o += align256((size_t)count * sizeof(BinArgs));
  h.gargs = o;
  o += align256((size_t)count * sizeof(GsxArgs));
  h.firsts = o;
  o += align256((size_t)count * 4 * 4);
  h.tile_inst = o;
  o += align256((size_t)tiles * 4);
  h.range_inst = o;
  o += align256((size_t)ranges * 4);
  h.gsx_inst = o;
  o += align256((size_t)gsx * 4);
  h.red_inst = o;
  o += align256((size_t)red * 4);
  h.bytes = o;
  return h;
}

// Scratch of one instance: binned S X scratch | S X | contraction partials.
size_t instance_bytes(int64_t R, int64_t tiles, int64_t nnz, int64_t B, int64_t d, int64_t parts,
                      int64_t m) {
  return bin_carve(nullptr, (int)R, tiles, nnz, nullptr) + align256((size_t)(B * d * 4)) +
         align256((size_t)(parts * m * d * 4));
}

struct Plan {
  std::vector<cg_instance> inst;
  int64_t tiles = 0, ranges = 0, gsx = 0, red = 0;
  int64_t gsx_by_nb[4] = {0, 0, 0, 0};   // contraction items of each width
  int r_max = 1;
  size_t reduce_lds = 0;
  Header header;
  size_t bytes = 0;
};

// Validate and plan every instance of src into p (src itself unchanged).
int make_plan(const cg_instance* src, int32_t count, Plan* p) {
  if (!src) return failf(CG_EINVAL, "instance table is NULL");
  if (count < 1) return failf(CG_EINVAL, "count = %d < 1", count);
  Tuning t;
  {
    std::lock_guard<std::mutex> lock(g_tuning_mu);
    t = g_tuning;
  }
  p->inst.assign(src, src + count);
  std::vector<size_t> sizes(count);
  for (int32_t i = 0; i < count; ++i) {
    cg_instance& c = p->inst[i];
    if (!c.row_ptr || !c.Y) return failf(CG_EINVAL, "instance %d: row_ptr or Y is NULL", i);
    if (c.nnz < 0 || c.nnz >= (1LL << 31))
      return failf(CG_EINVAL, "instance %d: nnz = %lld outside [0, 2^31)", i, (long long)c.nnz);
    if (c.nnz > 0 && (!c.col_idx || !c.vals))
      return failf(CG_EINVAL, "instance %d: col_idx or vals is NULL", i);
    if (c.n < 1 || c.n >= (1LL << 31))
      return failf(CG_EINVAL, "instance %d: n = %lld outside [1, 2^31)", i, (long long)c.n);
    if (c.d < 1 || c.d > kMaxD)
      return failf(c.d < 1 ? CG_EINVAL : CG_EUNSUPPORTED, "instance %d: d = %lld outside [1, %d]",
                   i, (long long)c.d, kMaxD);
    if (c.m < 1 || c.m > 64LL * 65535)
      return failf(c.m < 1 ? CG_EINVAL : CG_EUNSUPPORTED, "instance %d: m = %lld outside [1, %d]",
                   i, (long long)c.m, 64 * 65535);
    if (c.B < 1 || c.B > 0x7fffffffLL)
      return failf(CG_EINVAL, "instance %d: B = %lld outside [1, 2^31)", i, (long long)c.B);
    if (c.row_offset < 0)
      return failf(CG_EINVAL, "instance %d: row_offset %lld < 0", i, (long long)c.row_offset);
    const int64_t mgroups = (c.m + 63) / 64, ngroups = (c.d + 63) / 64;
    const int64_t red = (c.m * c.d + 63) / 64;
    const bool rows = rows_route_pays(c.n, c.d, c.nnz, c.m, c.B);
    const int cls = d_class(c.d);
    const BinGeom g = rows ? BinGeom{} : bin_geometry(true, c.n, (int)c.d, c.B, t.rows[cls]);
    if (!rows && !g.ok)
      return failf(CG_EUNSUPPORTED, "instance %d: binned S X does not apply (d = %lld, B = %lld)",
                   i, (long long)c.d, (long long)c.B);
    const int64_t kc = rows ? kBatchedRowsPerWave : t.kc[cls];   // rows route: rows per wavefront
    const int64_t parts = rows ? rows_parts(c.n, (int)kc) : (c.B + 4 * kc - 1) / (4 * kc);
    if (parts * mgroups * ngroups >= (1LL << 31) - 1)
      return failf(CG_EUNSUPPORTED, "instance %d: too many contraction work items", i);
    c.route = rows ? 1 : 0;
    c.tile_rows = rows ? 0 : g.tile_rows;
    c.tiles = rows ? 0 : (int32_t)g.ntiles;
    c.ranges = rows ? 0 : g.R;
    c.bp_shift = rows ? 0 : g.bp_shift;
    c.kc = (int32_t)kc;
    c.parts = (int32_t)parts;
    c.gsx_items = (int32_t)(parts * mgroups * ngroups);
    c.red_items = (int32_t)red;
    c.first_tile = (int32_t)p->tiles;
    c.first_range = (int32_t)p->ranges;
    c.first_gsx = (int32_t)p->gsx_by_nb[batched_nb(c.d) - 1];   // within its width; based below
    c.first_red = (int32_t)p->red;
    p->gsx_by_nb[batched_nb(c.d) - 1] += c.gsx_items;
    p->tiles += c.tiles;
    p->ranges += c.ranges;
    p->gsx += c.gsx_items;
    p->red += c.red_items;
    if (p->tiles >= (1LL << 31) - 1 || p->ranges >= (1LL << 31) - 1 || p->gsx >= (1LL << 31) - 1 ||
        p->red >= (1LL << 31) - 1)
      return failf(CG_EUNSUPPORTED, "batch has more than 2^31 work items in one phase");
    if (!rows && g.R > p->r_max) p->r_max = g.R;
    if (!rows && g.lds_bytes > p->reduce_lds) p->reduce_lds = g.lds_bytes;
    sizes[i] = rows ? align256((size_t)(parts * c.m * c.d * 4))
                    : instance_bytes(g.R, g.ntiles, c.nnz, c.B, c.d, parts, c.m);
  }
  // the contraction queue: the items of each width together, in increasing width
  int64_t base[4] = {0, 0, 0, 0};
  for (int k = 1; k < 4; ++k) base[k] = base[k - 1] + p->gsx_by_nb[k - 1];
  for (int32_t i = 0; i < count; ++i)
    p->inst[i].first_gsx += (int32_t)base[batched_nb(p->inst[i].d) - 1];
  p->header = header_layout(count, p->tiles, p->ranges, p->gsx, p->red);
  size_t off = p->header.bytes;
  for (int32_t i = 0; i < count; ++i) {
    p->inst[i].ws_off = (int64_t)off;
    off += sizes[i];
  }
  p->bytes = off;
  return CG_OK;
}

bool same_plan(const cg_instance& a, const cg_instance& b) {
  return a.ws_off == b.ws_off && a.tile_rows == b.tile_rows && a.tiles == b.tiles &&
         a.ranges == b.ranges && a.bp_shift == b.bp_shift && a.kc == b.kc && a.parts == b.parts &&
         a.gsx_items == b.gsx_items && a.red_items == b.red_items &&
         a.first_tile == b.first_tile && a.first_range == b.first_range &&
         a.first_gsx == b.first_gsx && a.first_red == b.first_red && a.route == b.route;
}

// One workgroup per instance: kernel arguments, first items and the
// instance's entries of the four item tables.
__global__ __launch_bounds__(256) void batched_setup_kernel(
    const cg_instance* __restrict__ tab, char* __restrict__ ws, BinArgs* __restrict__ bargs,
    GsxArgs* __restrict__ gargs, int32_t* __restrict__ firsts, int32_t count,
    int32_t* __restrict__ tile_inst, int32_t* __restrict__ range_inst,
    int32_t* __restrict__ gsx_inst, int32_t* __restrict__ red_inst) {
  const int32_t i = blockIdx.x;
  const cg_instance c = tab[i];
  if (threadIdx.x == 0) {
    char* base = ws + c.ws_off;
    BinArgs a{};
    a.row_ptr = c.row_ptr;
    a.col_idx = c.col_idx;
    a.vals = c.vals;
    a.n = c.n;
    a.nnz = (int32_t)c.nnz;
    a.d = (int32_t)c.d;
    a.B = (uint32_t)c.B;
    a.key = Key{(uint32_t)c.seed, (uint32_t)(c.seed >> 32)};
    a.row_offset = (uint64_t)c.row_offset;
    a.bp_shift = c.bp_shift;
    a.R = c.ranges;
    a.ntiles = c.tiles;
    a.tile_rows = c.tile_rows;
    // the rows route keeps only its partials (at base); no S X scratch
    const size_t bin = c.route ? 0 : bin_carve(base, c.ranges, c.tiles, c.nnz, &a);
    a.SX = c.route ? nullptr : (float*)(base + bin);
    bargs[i] = a;
    GsxArgs g{};
    g.SX = a.SX;
    g.part = c.route ? (float*)base : (float*)(base + bin + align256((size_t)(c.B * c.d * 4)));
    g.Y = c.Y;
    g.B = c.B;
    g.d = (int32_t)c.d;
    g.m = (int32_t)c.m;
    g.kc = c.kc;
    g.parts = c.parts;
    g.mgroups = (int32_t)((c.m + 63) / 64);
    g.ngroups = (int32_t)((c.d + 63) / 64);
    g.key = a.key;
    g.row_ptr = c.row_ptr;
    g.col_idx = c.col_idx;
    g.vals = c.vals;
    g.n = c.n;
    g.row_offset = (uint64_t)c.row_offset;
    g.nnz = (int32_t)c.nnz;
    g.route = c.route;
    gargs[i] = g;
    firsts[i] = c.first_tile;
    firsts[count + i] = c.first_range;
    firsts[2 * count + i] = c.first_gsx;
    firsts[3 * count + i] = c.first_red;
  }
  for (int32_t j = threadIdx.x; j < c.tiles; j += blockDim.x) tile_inst[c.first_tile + j] = i;
  for (int32_t j = threadIdx.x; j < c.ranges; j += blockDim.x) range_inst[c.first_range + j] = i;
  for (int32_t j = threadIdx.x; j < c.gsx_items; j += blockDim.x) gsx_inst[c.first_gsx + j] = i;
  for (int32_t j = threadIdx.x; j < c.red_items; j += blockDim.x) red_inst[c.first_red + j] = i;
}

}  // namespace
}  // namespace cg

extern "C" {

int cg_batched_plan(cg_instance* inst, int32_t count, const cg_opts* opts,
                    size_t* workspace_bytes) {
  if (opts && opts->struct_size < sizeof(cg_opts))
    return cg::failf(CG_EINVAL, "cg_opts.struct_size %u < %zu", opts->struct_size, sizeof(cg_opts));
  if (!workspace_bytes) return cg::failf(CG_EINVAL, "workspace_bytes is NULL");
  cg::Plan p;
  const int rc = cg::make_plan(inst, count, &p);
  if (rc != CG_OK) return rc;
  memcpy(inst, p.inst.data(), (size_t)count * sizeof(cg_instance));
  *workspace_bytes = p.bytes;
  return CG_OK;
}

int cg_sketch_batched(const cg_instance* inst, int32_t count, const cg_opts* opts) {
  if (!opts) return cg::failf(CG_EINVAL, "opts is NULL (the batch needs a workspace)");
  if (opts->struct_size < sizeof(cg_opts))
    return cg::failf(CG_EINVAL, "cg_opts.struct_size %u < %zu", opts->struct_size, sizeof(cg_opts));
  if (opts->precision != CG_PREC_NATIVE)
    return cg::failf(CG_EUNSUPPORTED, "batched instances run in native FP32 only");
  cg::Plan p;
  int rc = cg::make_plan(inst, count, &p);
  if (rc != CG_OK) return rc;
  for (int32_t i = 0; i < count; ++i)
    if (!cg::same_plan(p.inst[i], inst[i]))
      return cg::failf(CG_EINVAL, "instance %d: planned fields differ from cg_batched_plan's "
                       "(plan again after changing an instance or the tuning table)", i);
  char* ws = (char*)opts->workspace;
  if (!ws || ((uintptr_t)ws & 255))
    return cg::failf(CG_ENOSPACE, "workspace missing or not 256-byte aligned");
  if (opts->workspace_bytes < p.bytes)
    return cg::failf(CG_ENOSPACE, "workspace %zu bytes < %zu needed", opts->workspace_bytes, p.bytes);
  hipStream_t s = (hipStream_t)opts->stream;
  const cg::Header& h = p.header;
  cg_instance* tab = (cg_instance*)(ws + h.table);
  cg::BinArgs* bargs = (cg::BinArgs*)(ws + h.bargs);
  cg::GsxArgs* gargs = (cg::GsxArgs*)(ws + h.gargs);
  int32_t* firsts = (int32_t*)(ws + h.firsts);
  int32_t* tile_inst = (int32_t*)(ws + h.tile_inst);
  int32_t* range_inst = (int32_t*)(ws + h.range_inst);
  int32_t* gsx_inst = (int32_t*)(ws + h.gsx_inst);
  int32_t* red_inst = (int32_t*)(ws + h.red_inst);
  hipError_t e = hipMemcpyAsync(tab, inst, (size_t)count * sizeof(cg_instance),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess)
    return cg::failf(CG_EHIP, "hipMemcpyAsync(instance table): %s", hipGetErrorString(e));
  cg::batched_setup_kernel<<<(unsigned)count, 256, 0, s>>>(tab, ws, bargs, gargs, firsts, count,
                                                           tile_inst, range_inst, gsx_inst,
                                                           red_inst);
  if ((e = hipGetLastError()) != hipSuccess)
    return cg::failf(CG_EHIP, "batched setup: %s", hipGetErrorString(e));
  e = cg::launch_sx_binned_batched(bargs, tile_inst, firsts, p.tiles, range_inst, firsts + count,
                                   p.ranges, p.r_max, p.reduce_lds, s);
  if (e != hipSuccess) return cg::failf(CG_EHIP, "batched S X: %s", hipGetErrorString(e));
  e = cg::launch_gsx_batched(gargs, gsx_inst, firsts + 2 * count, p.gsx_by_nb, s);
  if (e != hipSuccess) return cg::failf(CG_EHIP, "batched contraction: %s", hipGetErrorString(e));
  e = cg::launch_splitk_batched(gargs, red_inst, firsts + 3 * count, p.red, s);
  if (e != hipSuccess) return cg::failf(CG_EHIP, "batched reduction: %s", hipGetErrorString(e));
  return CG_OK;
}

int cg_set_tuning(const int32_t* rows_per_item, const int32_t* kc_per_item, int32_t classes) {
  if (!rows_per_item && !kc_per_item) {
    std::lock_guard<std::mutex> lock(cg::g_tuning_mu);
    cg::g_tuning = cg::default_tuning();
    return CG_OK;
  }
  if (classes < 1 || classes > cg::kClasses)
    return cg::failf(CG_EINVAL, "classes = %d outside [1, %d]", classes, cg::kClasses);
  for (int32_t c = 0; c < classes; ++c) {
    if (rows_per_item && (rows_per_item[c] < 1024 || rows_per_item[c] % 1024 != 0 ||
                          rows_per_item[c] > (1 << 24)))
      return cg::failf(CG_EINVAL, "rows_per_item[%d] = %d: a multiple of 1024 in [1024, 2^24]", c,
                       rows_per_item[c]);
    if (kc_per_item && (kc_per_item[c] < 16 || kc_per_item[c] % 16 != 0 ||
                        kc_per_item[c] > (1 << 20)))
      return cg::failf(CG_EINVAL, "kc_per_item[%d] = %d: a multiple of 16 in [16, 2^20]", c,
                       kc_per_item[c]);
  }
  std::lock_guard<std::mutex> lock(cg::g_tuning_mu);
  for (int32_t c = 0; c < classes; ++c) {
    if (rows_per_item) cg::g_tuning.rows[c] = rows_per_item[c];
    if (kc_per_item) cg::g_tuning.kc[c] = kc_per_item[c];
  }
  return CG_OK;
}

int cg_get_tuning(int32_t* rows_per_item, int32_t* kc_per_item, int32_t classes) {
  if (classes < 1 || classes > cg::kClasses)
    return cg::failf(CG_EINVAL, "classes = %d outside [1, %d]", classes, cg::kClasses);
  std::lock_guard<std::mutex> lock(cg::g_tuning_mu);
  for (int32_t c = 0; c < classes; ++c) {
    if (rows_per_item) rows_per_item[c] = cg::g_tuning.rows[c];
    if (kc_per_item) kc_per_item[c] = cg::g_tuning.kc[c];
  }
  return CG_OK;
}

}  // extern "C"
