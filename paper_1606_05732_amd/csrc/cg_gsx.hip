// Y = G (S X): the m x B by B x d product of Section 1.1, on MFMA, with G
// generated in registers and never written to memory.
//
// Work split: the B axis (the contraction) is cut into chunks of kc
// columns of G; one wavefront owns one chunk, one 64-row group of G and up
// to 64 columns of S X.  Four wavefronts of a workgroup add their
// accumulators in a fixed order and write one partial m x d product per
// workgroup; splitk_reduce_kernel then adds the partials in a fixed order.
// The result is therefore reproducible bit for bit, and FP32 sums never
// run over more than kc terms before being combined pairwise-ish.
//
// Register tiling (v_mfma_*_16x16xK): lane l has p = l % 16 and
// kq = l / 16.  In the A operand lane l supplies row p and K slot(s) kq;
// one Philox4x32 block of counter (b, q) yields the four normals
// G[4q + t][b], t = 0..3, so the lane owns row quad q = 16 * group + p and
// feeds four MFMA instructions, one per t: M block t holds the G rows
// 4 (16 group + p) + t.  The B operand (S X) uses the same K slots, so
// every generated normal is used exactly once.  D element (4 kq + r, p)
// of M block t is Y row 4 (16 group + 4 kq + r) + t, column p (FP64: the
// D rows of a lane are kq + 4 r instead, see d_row).
//
// Half groups: when a 64-row group holds at most 32 rows of G (m <= 32,
// or the last group), its row quads are q = 16 group + (p & 7).  Lanes
// p < 8 draw a step's normals and lanes p >= 8 the next step's, for the
// same quads, so every lane draws one Philox block per two steps.  Rows
// are paired in two M blocks: block 0 holds rows 4q (lanes p < 8) and
// 4q + 1 (lanes p >= 8), block 1 rows 4q + 2 and 4q + 3, with lane moves
// (p - 8 -> p, p + 8 -> p) bringing each normal to its lane.  That is half
// the MFMAs of four blocks with the upper half idle, and every existing
// row still sees the same operands in the same order as in a full group,
// so the result is bit for bit the same.
#include "cg_internal.hpp"
#include "cg_rng.hpp"

namespace cg {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

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

// Row of the 16x16 result block held in accumulator register r of a lane
// with kq = lane / 16 (the column is lane % 16).  The FP32 16x16x4 and the
// K=32 variants keep four consecutive rows per lane; the FP64 16x16x4
// interleaves them (measured on gfx950).
template <typename T>
__device__ __forceinline__ int d_row(int kq, int r) {
  return sizeof(T) == 8 ? kq + 4 * r : 4 * kq + r;
}

// Sum the four wavefronts' accumulators (wave 0 + 1 + 2 + 3, in that
// order) and write the workgroup's partial product rows/cols that exist.
// VEC: lane p's NB column blocks hold the consecutive columns
// n0 + NB p + nb (so that one vector load fetches them) instead of
// n0 + 16 nb + p.  PAIRS: the half-group layout, two M blocks (acc[0],
// acc[1]) whose row i holds G row 4 (16 group + i) + 2 t for i < 8 and
// 4 (16 group + i - 8) + 2 t + 1 for i >= 8.
template <typename T, int NB, typename V, bool VEC = false, bool PAIRS = false>
__device__ __forceinline__ void block_reduce_store(V (&acc)[4][NB], T* red, int wave, int lane,
                                                   int group, int n0, int m, int d,
                                                   T* __restrict__ out) {
  constexpr int R = 16 * NB;   // accumulator values per lane
  constexpr int MB = PAIRS ? 2 : 4;
  // wavefronts 0 .. 3 hold the accumulators (any others take part in the
  // barrier only)
  if (wave > 0 && wave < kWaves) {
#pragma unroll
    for (int t = 0; t < MB; ++t)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          red[((wave - 1) * R + (t * NB + nb) * 4 + r) * 64 + lane] = acc[t][nb][r];
  }
  __syncthreads();
  if (wave != 0) return;
  const int p = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int t = 0; t < MB; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int idx = (t * NB + nb) * 4 + r;
        T s = acc[t][nb][r];
        s += red[(0 * R + idx) * 64 + lane];
        s += red[(1 * R + idx) * 64 + lane];
        s += red[(2 * R + idx) * 64 + lane];
        const int i = d_row<T>(kq, r);
        const int row = PAIRS ? (i < 8 ? 4 * (16 * group + i) + 2 * t : 4 * (16 * group + i - 8) + 2 * t + 1)
                              : 4 * (16 * group + i) + t;
        const int col = VEC ? n0 + NB * p + nb : n0 + nb * 16 + p;
        if (row < m && col < d) out[(size_t)row * d + col] = s;
      }
}

// Native precision (FP32 or FP64 inputs, same-type accumulation).  One
// workgroup: split `bx` along B, 64-row group `group` of G, column group
// `ng` of S X.
// Lane p + 8's value in lane p of each 16-lane row (0 in lanes 8 .. 15):
// DPP row_shl:8, no LDS round trip.
__device__ __forceinline__ float from_lane_p8(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x108, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_lane_p8(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x108, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x108, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
// Lane p - 8's value in lane p of each 16-lane row (0 in lanes 0 .. 7):
// DPP row_shr:8.
__device__ __forceinline__ float from_lane_m8(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_lane_m8(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x118, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x118, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Whether this 64-row group of G holds at most 32 existing rows.
__device__ __forceinline__ bool half_group(int m, int group) { return m - 64 * group <= 32; }

template <typename T, int NB>
constexpr int red_elems() {
  return 3 * 16 * NB * 64;
}

// `red`: red_elems<T, NB>() elements of LDS for the cross-wavefront sum.
// HALF: the group holds at most 32 rows of G (see the file comment).
// Normals of K column k (of B for G, TAG 1; a row of X, offset by col0, for
// the dense Gaussian G~, TAG 2), row quad q.
template <int TAG>
__device__ __forceinline__ Words4 k_block(int64_t k, uint64_t col0, uint32_t q, Key key) {
  if constexpr (TAG == 1) return gauss_block((uint32_t)k, q, key.k0, key.k1);
  return dense_gauss_block(col0 + (uint64_t)k, q, key.k0, key.k1);
}

// TAG 1: Y = G (S X) with SX the B x d matrix S X (ld = d).  TAG 2: the
// dense Gaussian product G~ X, the same contraction with X (n x d, row
// stride ld) in place of S X and G~'s columns col0 + k in place of G's.
template <typename T, int NB, bool HALF, int TAG = 1>
__device__ __forceinline__ void gsx_native_block(const T* __restrict__ SX, int64_t ld, uint64_t col0,
                                                 int64_t B, int d, int m, int kc, Key key,
                                                 T* __restrict__ part, int64_t bx, int group,
                                                 int ng, T* red) {
  using V = typename Vec4<T>::type;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = lane & 15, kq = lane >> 4;
  // half groups: lanes p and p + 8 share a row quad, one step apart
  const uint32_t q = (uint32_t)(16 * group + (HALF ? (p & 7) : p));
  const int n0 = ng * NB * 16;
  V acc[4][NB];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[t][nb] = V{0, 0, 0, 0};
  int col[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) col[nb] = n0 + nb * 16 + p;

  const int64_t kbeg = (bx * kWaves + wave) * kc;
  const int64_t kend = min(kbeg + (int64_t)kc, B);
  int ccol[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) ccol[nb] = min(col[nb], d - 1);
  // Groups of KU steps of 4 columns (kc is a multiple of 4 KU).  A group's
  // S X values are loaded two groups ahead, so their latency hides behind
  // the two previous groups' normals and MFMAs.  Loads and normals are taken
  // unguarded at a clamped index and the values past the chunk or the
  // columns zeroed afterwards (a guarded load would be waited for at the
  // end of its branch).
  constexpr int KU = 4;
  auto load_group = [&](int64_t kg, T (&x)[KU][NB]) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int64_t b = kg + 4 * u + kq;
      const int64_t cb = b < kend ? b : kend - 1;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) x[u][nb] = SX[cb * ld + ccol[nb]];
    }
  };
  // (unconditional: indices clamp to kend - 1 >= 0, and the group after
  // the last is a harmless reload)
  T xn[KU][NB], xn2[KU][NB];
  load_group(kbeg, xn);
  load_group(kbeg + 4 * KU, xn2);
  // full groups: the normals of the first step (later ones are drawn a
  // step ahead, below).  Normals of columns past the chunk need no mask:
  // their S X operand is zeroed, and a finite normal times zero adds
  // nothing; their counters are just numbers, so they need no clamp.
  T gn[4];
  if constexpr (!HALF) box_muller(k_block<TAG>(kbeg + kq, col0, q, key), gn);
  for (int64_t kg = kbeg; kg < kend; kg += 4 * KU) {
    T x[KU][NB];
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        x[u][nb] = xn[u][nb];
        xn[u][nb] = xn2[u][nb];
      }
    load_group(kg + 8 * KU, xn2);
    if constexpr (HALF) {
#pragma unroll
      for (int u = 0; u < KU; u += 2) {
        // this lane's normals: step u (p < 8) or step u + 1 (p >= 8), both
        // for row quad q = 16 group + (p & 7)
        const int64_t bg = kg + 4 * (u + (p >> 3)) + kq;
        T g[4];
        box_muller(k_block<TAG>(bg, col0, q, key), g);
        // two M blocks of paired rows: block 0 holds rows 4q (lanes p < 8)
        // and 4q + 1 (lanes p >= 8), block 1 rows 4q + 2 and 4q + 3.  Step
        // u's normals come from lanes p < 8, step u + 1's from lanes p >= 8,
        // each moved to the other half of the row where needed
        const T m1 = from_lane_m8(g[1]), m3 = from_lane_m8(g[3]);
        const T p0 = from_lane_p8(g[0]), p2 = from_lane_p8(g[2]);
        const bool lo = p < 8;
        const T a[2][2] = {{lo ? g[0] : m1, lo ? g[2] : m3}, {lo ? p0 : g[1], lo ? p2 : g[3]}};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          // S X rows of step u + h (this lane's K slot kq, as in a full group)
          const bool bok = kg + 4 * (u + h) + kq < kend;
          T xv[NB];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) xv[nb] = bok && col[nb] < d ? x[u + h][nb] : T(0);
#pragma unroll
          for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[t][nb] = mfma_k4(a[h][t], xv[nb], acc[t][nb]);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int64_t b = kg + 4 * u + kq;
        const bool bok = b < kend;
        // this step's normals were drawn during the step before; the next
        // step's are drawn now, so that their VALU work can overlap this
        // step's MFMAs
        T g[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) g[t] = gn[t];
        box_muller(k_block<TAG>(b + 4, col0, q, key), gn);
        T xv[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) xv[nb] = bok && col[nb] < d ? x[u][nb] : T(0);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[t][nb] = mfma_k4(g[t], xv[nb], acc[t][nb]);
      }
    }
  }
  block_reduce_store<T, NB, V, false, HALF>(acc, red, wave, lane, group, n0, m, d,
                                            part + (size_t)bx * m * d);
}

template <typename T, int NB, int TAG>
__global__ __launch_bounds__(kThreads, 4) void gsx_native_kernel(const T* __restrict__ SX, int64_t ld,
                                                              uint64_t col0, int64_t B, int d, int m,
                                                              int kc, Key key,
                                                              T* __restrict__ part) {
  __shared__ T red[red_elems<T, NB>()];
  if (half_group(m, (int)blockIdx.y))
    gsx_native_block<T, NB, true, TAG>(SX, ld, col0, B, d, m, kc, key, part, blockIdx.x, blockIdx.y,
                                       blockIdx.z, red);
  else
    gsx_native_block<T, NB, false, TAG>(SX, ld, col0, B, d, m, kc, key, part, blockIdx.x,
                                        blockIdx.y, blockIdx.z, red);
}

// Producer/consumer form of the FP32 contraction, for full row groups
// (more than 32 rows of G): eight wavefronts per workgroup.  Wavefronts
// 0-3 are consumers: each owns a chunk of kc columns of G as a wavefront of
// gsx_native_block does, and only multiplies.  Wavefronts 4-7 are
// producers: they draw the normals of all four chunks into LDS, kPcStage
// columns per chunk at a time, double buffered one stage ahead.
// Wavefronts w and w + 4 share a SIMD, so every SIMD has one wavefront on
// the generator's vector work and one on FP32 MFMAs.  A SIMD issues only
// one of the two kinds in any cycle, but each kind can now issue while the
// other waits on its own dependencies.  A consumer lane (p, kq) reads, for its
// K slot kq, the four normals of row quad 16 group + p as one 16-byte LDS
// word, exactly the values a lane of gsx_native_block draws itself, and
// multiplies them in the same order; the cross-wavefront sum is the same
// too, so the partials are bit for bit those of gsx_native_block.
constexpr int kPcStage = 16;                          // columns per chunk per stage
constexpr int kPcStageFloats = kWaves * kPcStage * 64;   // chunks x columns x 16 quads x 4 rows

template <int NB, int TAG>
__global__ __launch_bounds__(2 * kThreads, 2) void gsx_pc_kernel(const float* __restrict__ SX,
                                                               int64_t ld, uint64_t col0, int64_t B,
                                                               int d, int m, int kc, Key key,
                                                               float* __restrict__ part) {
  constexpr int kLds = red_elems<float, NB>() > 2 * kPcStageFloats ? red_elems<float, NB>()
                                                                   : 2 * kPcStageFloats;
  __shared__ __align__(16) float lds[kLds];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int group = (int)blockIdx.y;
  const int n0 = (int)blockIdx.z * NB * 16;
  const int64_t bx = blockIdx.x;
  const int nst = kc / kPcStage;   // kc is a multiple of 16 for FP32
  v4f acc[4][NB];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[t][nb] = v4f{0, 0, 0, 0};
  if (wave >= kWaves) {
    // producer lane L: column j = L / 16 of the stage and quad 16 group +
    // L % 16, for each of the four chunks
    const int L = (wave - kWaves) * 64 + lane;
    const int j = L >> 4, pq = L & 15;
    const uint32_t q = (uint32_t)(16 * group + pq);
    auto produce = [&](int st, int buf) {
#pragma unroll
      for (int c = 0; c < kWaves; ++c) {
        const int64_t b = (bx * kWaves + c) * kc + (int64_t)st * kPcStage + j;
        float g[4];
        box_muller(k_block<TAG>(b, col0, q, key), g);
        *(v4f*)&lds[(((buf * kWaves + c) * kPcStage + j) * 16 + pq) * 4] = v4f{g[0], g[1], g[2], g[3]};
      }
    };
    produce(0, 0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
      if (st + 1 < nst) produce(st + 1, (st + 1) & 1);
      __syncthreads();   // this stage consumed, the next one written
    }
  } else {
    const int p = lane & 15, kq = lane >> 4;
    const int64_t kbeg = (bx * kWaves + wave) * (int64_t)kc;
    const int64_t kend = min(kbeg + (int64_t)kc, B);
    int col[NB], ccol[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      col[nb] = n0 + nb * 16 + p;
      ccol[nb] = min(col[nb], d - 1);
    }
    // S X of a stage (its four K steps), loaded a stage ahead at indices
    // clamped onto the chunk's last row; rows past the chunk (or past B,
    // for a chunk that starts there) are zeroed when used
    const int64_t clast = (kend > kbeg ? kend : B) - 1;
    auto load_stage = [&](int st, float (&x)[4][NB]) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t b = kbeg + (int64_t)st * kPcStage + 4 * k + kq;
        const int64_t cb = b < clast ? b : clast;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) x[k][nb] = SX[cb * ld + ccol[nb]];
      }
    };
    float xn[4][NB];
    load_stage(0, xn);
    __syncthreads();   // stage 0 written
    for (int st = 0; st < nst; ++st) {
      float x[4][NB];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) x[k][nb] = xn[k][nb];
      if (st + 1 < nst) load_stage(st + 1, xn);
      const float* stage = lds + ((st & 1) * kWaves + wave) * kPcStage * 64;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const v4f g = *(const v4f*)&stage[((4 * k + kq) * 16 + p) * 4];
        const bool bok = kbeg + (int64_t)st * kPcStage + 4 * k + kq < kend;
        float xv[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) xv[nb] = bok && col[nb] < d ? x[k][nb] : 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[t][nb] = mfma_k4(g[t], xv[nb], acc[t][nb]);
      }
      __syncthreads();   // this stage consumed, the next one written
    }
  }
  // every stage read before the cross-wavefront sum reuses the LDS (the
  // loop's last barrier)
  block_reduce_store<float, NB, v4f, false, false>(acc, lds, wave, lane, group, n0, m, d,
                                                   part + (size_t)bx * m * d);
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// Largest |x| over x[0 .. cnt) (NaNs ignored), this lane's share: 16-byte
// loads with eight in flight when x is 16-byte aligned, else 4-byte loads.
__device__ __forceinline__ float block_amax(const float* __restrict__ x, int64_t cnt, int lane) {
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  float am[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int64_t tail = 0;
  if (((uintptr_t)x & 15) == 0) {
    const f32x4* x4 = (const f32x4*)x;
    const int64_t n4 = cnt >> 2;
    int64_t i = lane;
    for (; i + 7 * 64 < n4; i += 8 * 64) {
      f32x4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = x4[i + u * 64];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        am[u] = fmaxf(am[u], fmaxf(fmaxf(fabsf(v[u].x), fabsf(v[u].y)),
                                   fmaxf(fabsf(v[u].z), fabsf(v[u].w))));
    }
    for (; i < n4; i += 64) {
      const f32x4 v = x4[i];
      am[0] = fmaxf(am[0], fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
    tail = n4 << 2;
  }
  for (int64_t i = tail + lane; i < cnt; i += 64) am[1] = fmaxf(am[1], fabsf(x[i]));
  return fmaxf(fmaxf(fmaxf(am[0], am[1]), fmaxf(am[2], am[3])),
               fmaxf(fmaxf(am[4], am[5]), fmaxf(am[6], am[7])));
}

// Smallest e with amax <= 448 * 2^e, from amax's binary exponent
// (448 = 0.875 * 2^9); 0 for amax == 0.
__device__ __forceinline__ int fp8_block_exponent(float amax) {
  if (!(amax > 0.0f)) return 0;
  int E;
  const float f = frexpf(amax, &E);
  return f <= 0.875f ? E - 9 : E - 8;
}

// Two FP32 values to OCP FP8 E4M3 (round to nearest even, saturating) in
// the low (HI = false) or high byte pair of `old`.
template <bool HI>
__device__ __forceinline__ int cvt_fp8(float a, float b, int old) {
  return __builtin_amdgcn_cvt_pk_fp8_f32(a, b, old, HI);
}

// Power-of-two scales of the FP8 contraction, one pair per 128-row block of
// S X (all d columns): (2^-e, 2^(e - 6)) with e the smallest integer such
// that the block's largest |value| is at most 448 2^e (NaNs ignored), at
// least -100 so that 2^-e stays finite.  One wavefront per block, 16-byte
// loads with eight in flight; the contraction then reads one pair per
// block instead of the block itself.
__global__ __launch_bounds__(kThreads) void fp8_block_scale_kernel(const float* __restrict__ SX,
                                                                   int64_t B, int d,
                                                                   float2* __restrict__ scale) {
  const int64_t blk = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t nblk = (B + 127) / 128;
  if (blk >= nblk) return;
  const int64_t r0 = blk * 128;
  const int64_t rows = min((int64_t)128, B - r0);
  const float amax = wave_max(block_amax(SX + r0 * d, rows * d, lane));
  const int e = max(fp8_block_exponent(amax), -100);
  if (lane == 0) scale[blk] = make_float2(ldexpf(1.0f, -e), ldexpf(1.0f, e - 6));
}

// Reduced-precision inputs: BF16 (round to nearest even) or FP8 E4M3 with
// one power-of-two scale per 128-wide block of B for S X (from the binned
// S X reduce or fp8_block_scale_kernel) and 2^-6 for G; FP32
// accumulation.  K = 32 per MFMA: lane (p, kq) supplies the eight columns
// b = base + 8 kq + e, e = 0..7, i.e. eight Philox blocks per step.  A
// step's S X values are loaded one step ahead and packed into the MFMA
// operand format as soon as the step begins, so only one step of FP32
// values is ever held (registers decide the occupancy here).
//
// The contraction is bound by the vector ALUs (Philox's 64-bit products
// and Box-Muller's transcendentals), so the rest is kept lean:
//  * VEC (NB = 2 or 4, d a multiple of 16 NB): lane p takes the NB
//    consecutive columns n0 + NB p + nb, one 8- or 16-byte load per row;
//  * rows are addressed by 32-bit element offsets from S X (the host
//    checks B d < 2^31), advanced by a wavefront-uniform step and clamped
//    to the chunk's last row with one min;
//  * a 128-column block wholly inside the chunk (all but at most one per
//    wavefront) takes no per-column masks;
//  * normals and S X values are converted two at a time.
// Eight rows from byte offset `off` (row b's first element), `dstep`
// bytes apart, clamped to `last` (the chunk's last row); the elements at
// byte offsets `col[nb]` of each (with VEC, from col[0] on).  32-bit byte
// offsets from a wavefront-uniform base let the loads use the
// scalar-base addressing form.
template <int NB, bool VEC>
__device__ __forceinline__ void lowp_load_rows(const float* __restrict__ SX, uint32_t off,
                                               uint32_t dstep, uint32_t last,
                                               const uint32_t (&col)[NB], float (&x)[8][NB]) {
  const char* base = (const char*)SX;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t o = min(off + (uint32_t)e * dstep, last);
    if constexpr (VEC && NB == 4) {
      typedef float f4 __attribute__((ext_vector_type(4)));
      const f4 v = *(const f4*)(base + (o + col[0]));
      x[e][0] = v.x;
      x[e][1] = v.y;
      x[e][2] = v.z;
      x[e][3] = v.w;
    } else if constexpr (VEC && NB == 2) {
      typedef float f2 __attribute__((ext_vector_type(2)));
      const f2 v = *(const f2*)(base + (o + col[0]));
      x[e][0] = v.x;
      x[e][1] = v.y;
    } else {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) x[e][nb] = *(const float*)(base + (o + col[nb]));
    }
  }
}

// Two FP32 values to a BF16 pair (round to nearest even), a in the low half.
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  const bf2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}

// The reduced-precision contraction, in producer/consumer form: eight
// wavefronts per workgroup.  Wavefront c < 4 is a consumer: it owns chunk
// c of the workgroup's 4 kc columns of G, loads and packs S X (as above)
// and multiplies.  Wavefront c + 4 is its producer: its lane l draws and
// packs, a 32-column step ahead, the G operand of consumer lane l (eight
// Philox blocks, Box-Muller, BF16 pairs or FP8 bytes) into a double-
// buffered LDS slot of that lane.  The producers never wait on memory, so
// the consumers' S X loads wait behind their work (one wavefront doing both
// was slower at the planner's chunk size, 1024 consumer wavefronts).  Every
// consumer runs all kc / 32 steps of its chunk (steps past its end, which
// only the last chunk has, multiply zeroed S X), so that the eight
// wavefronts meet at the same barriers.  One launch covers the parts
// bx0 + blockIdx.x; SX points at row row0 of S X (the host splits the parts
// so that every row a launch reads lies below row0 + 2^30 / d).
template <int NB, bool FP8, bool VEC>
__global__ __launch_bounds__(2 * kThreads) void gsx_lowp_pc_kernel(
    const float* __restrict__ SX, int64_t row0, int64_t bx0, int64_t B, int d, int m, int kc,
    Key key, const float2* __restrict__ bscale, float* __restrict__ part) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  constexpr int KBLK = FP8 ? 128 : 32;
  constexpr int GW = FP8 ? 2 : 4;                        // G words per M block per step
  constexpr int kSlot = 4 * GW;                          // words per lane per step
  constexpr int kBuf = kWaves * 64 * kSlot;              // words per buffer
  constexpr int kRed = 3 * 16 * NB * 64;
  constexpr int kLds = kRed > 2 * kBuf ? kRed : 2 * kBuf;
  __shared__ __align__(16) float lds[kLds];
  uint32_t* gbuf = (uint32_t*)lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = lane & 15, kq = lane >> 4;
  const int group = blockIdx.y;
  const uint32_t q = (uint32_t)(16 * group + p);
  const int n0 = blockIdx.z * NB * 16;
  const int c = wave & (kWaves - 1);                      // the chunk this wavefront serves
  const int64_t bx = bx0 + blockIdx.x;
  const int64_t kbeg = (bx * kWaves + c) * kc;
  const int64_t kend = min(kbeg + (int64_t)kc, B);
  const int nsteps = kc / 32;                             // kc: a multiple of KBLK
  v4f acc[4][NB];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[t][nb] = v4f{0, 0, 0, 0};
  if (wave >= kWaves) {
    uint32_t* slot = gbuf + (c * 64 + lane) * kSlot;
    auto produce = [&](int st, int buf) {
      const int64_t base = kbeg + 32 * (int64_t)st + kq * 8;
      uint32_t gw[4][GW];
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        float z0[4], z1[4];
        box_muller(gauss_block((uint32_t)(base + e), q, key.k0, key.k1), z0, FP8 ? 64.0f : 1.0f);
        box_muller(gauss_block((uint32_t)(base + e + 1), q, key.k0, key.k1), z1, FP8 ? 64.0f : 1.0f);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if constexpr (FP8) {
            uint32_t& w = gw[t][e >> 2];
            w = (e & 2) ? (uint32_t)cvt_fp8<true>(z0[t], z1[t], (int)w)
                        : (uint32_t)cvt_fp8<false>(z0[t], z1[t], 0);
          } else {
            gw[t][e >> 1] = bf16_pair(z0[t], z1[t]);
          }
        }
      }
      uint32_t* dst = slot + buf * kBuf;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if constexpr (FP8) {
          *(uint2*)(dst + t * GW) = make_uint2(gw[t][0], gw[t][1]);
        } else {
          *(u32x4*)(dst + t * GW) = u32x4{gw[t][0], gw[t][1], gw[t][2], gw[t][3]};
        }
      }
    };
    produce(0, 0);
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
      if (st + 1 < nsteps) produce(st + 1, (st + 1) & 1);
      __syncthreads();   // this step consumed, the next one written
    }
  } else {
    bool cok[NB];
    uint32_t ccol[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int col = VEC ? n0 + NB * p + nb : n0 + 16 * nb + p;
      cok[nb] = col < d;
      ccol[nb] = 4u * (uint32_t)min(col, d - 1);   // bytes
    }
    const uint32_t ud = 4u * (uint32_t)d;
    const uint32_t last = (uint32_t)((kend > kbeg ? kend : B) - 1 - row0) * ud;
    uint32_t off = (uint32_t)(kbeg + kq * 8 - row0) * ud;
    float xn[8][NB];
    lowp_load_rows<NB, VEC>(SX, off, ud, last, ccol, xn);
    const uint32_t* slot = gbuf + (c * 64 + lane) * kSlot;
    const int64_t nblk = (B + 127) / 128;
    float yscale = 1.0f, xscale = 1.0f;
    v4f tmp[4][NB];
    __syncthreads();   // step 0 written
    for (int st = 0; st < nsteps; ++st) {
      const int sub = st % (KBLK / 32);
      const int64_t kb = kbeg + (int64_t)(st - sub) * 32;
      if constexpr (FP8) {
        if (sub == 0) {
          const float2 sc = bscale[min(kb >> 7, nblk - 1)];
          xscale = sc.x;
          yscale = sc.y;
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) tmp[t][nb] = v4f{0, 0, 0, 0};
        }
      }
      const int64_t base = kb + sub * 32 + kq * 8;
      if (kb + sub * 32 + 32 > kend) {   // the same in the whole wavefront
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) xn[e][nb] = base + e < kend ? xn[e][nb] : 0.0f;
      }
      uint32_t xw[NB][4];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          float x0 = xn[e][nb], x1 = xn[e + 1][nb];
          if constexpr (!VEC) {
            x0 = cok[nb] ? x0 : 0.0f;
            x1 = cok[nb] ? x1 : 0.0f;
          }
          if constexpr (FP8) {
            uint32_t& w = xw[nb][e >> 2];
            w = (e & 2) ? (uint32_t)cvt_fp8<true>(x0 * xscale, x1 * xscale, (int)w)
                        : (uint32_t)cvt_fp8<false>(x0 * xscale, x1 * xscale, 0);
          } else {
            xw[nb][e >> 1] = bf16_pair(x0, x1);
          }
        }
      }
      off += 32 * ud;
      lowp_load_rows<NB, VEC>(SX, off, ud, last, ccol, xn);
      const uint32_t* src = slot + (st & 1) * kBuf;
      if constexpr (FP8) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const uint2 g = *(const uint2*)(src + t * GW);
          const long ga = (long)g.x | ((long)g.y << 32);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const long xa = (long)xw[nb][0] | ((long)xw[nb][1] << 32);
            tmp[t][nb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ga, xa, tmp[t][nb], 0, 0, 0);
          }
        }
        if (sub == KBLK / 32 - 1) {
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[t][nb] += tmp[t][nb] * yscale;
        }
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const v8bf gb = __builtin_bit_cast(v8bf, *(const u32x4*)(src + t * GW));
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const v8bf xb = __builtin_bit_cast(v8bf, u32x4{xw[nb][0], xw[nb][1], xw[nb][2], xw[nb][3]});
            acc[t][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gb, xb, acc[t][nb], 0, 0, 0);
          }
        }
      }
      __syncthreads();   // this step consumed, the next one written
    }
  }
  block_reduce_store<float, NB, v4f, VEC>(acc, lds, wave, lane, group, n0, m, d,
                                          part + (size_t)bx * m * d);
}

// Y[o] = sum over partials p of part[p][o]: 16 wavefronts each add a
// contiguous sixteenth of the partials (eight loads in flight), then the
// sixteen sums are added in order.  Fixed order, so the result does not
// depend on timing.
constexpr int kRedWaves = 16;
template <typename T>
__device__ __forceinline__ void splitk_reduce_block(const T* __restrict__ part, int64_t P,
                                                    int64_t md, T* __restrict__ Y, int64_t blk) {
  __shared__ T s[kRedWaves][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t o = blk * 64 + lane;
  const int64_t p0 = P * wave / kRedWaves, p1 = P * (wave + 1) / kRedWaves;
  T acc = T(0);
  if (o < md) {
    int64_t pp = p0;
    for (; pp + 8 <= p1; pp += 8) {
      T a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = part[(pp + u) * md + o];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += a[u];
    }
    for (; pp < p1; ++pp) acc += part[pp * md + o];
  }
  s[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && o < md) {
    T y = s[0][lane];
#pragma unroll
    for (int w = 1; w < kRedWaves; ++w) y += s[w][lane];
    Y[o] = y;
  }
}

template <typename T>
__global__ __launch_bounds__(64 * kRedWaves) void splitk_reduce_kernel(const T* __restrict__ part,
                                                                      int64_t P, int64_t md,
                                                                      T* __restrict__ Y) {
  splitk_reduce_block<T>(part, P, md, Y, blockIdx.x);
}

// ------------------------------------------------------------ rows route
// Y = sum over the nonempty rows r of X of sigma(r) G[:, h(r)] x_r^T: S
// sends row r to column h(r) of S X with sign sigma(r), so this is G (S X)
// taken row by row, and S X is never formed.
//
// Wavefront w of workgroup `bx` takes rows [(4 bx + w) R, (4 bx + w + 1) R)
// with R = a.kc (rows_per_wave), 256 at a time (four per lane).  It
// compacts the nonempty ones -- packed hash, first entry, end -- into its
// LDS in row order (ballots and bit counts, no LDS scan).  The window's
// entries, one contiguous segment of col_idx / vals, are copied into its
// LDS with independent loads when they fit (kRowsWinEntries), so that the
// steps below do not each wait for memory.  It then takes the rows four at
// a time as the K slots of the 16x16x4 MFMAs: lane (p, kq) draws the
// Philox block of G column h(row kq), row quad p, with the row's sign
// applied, and the four rows' entries are added into a dense
// wavefront-private LDS tile, from which the B operand is read.
// In half groups lanes p >= 8 draw the blocks of the next four rows (as in
// the S X contraction), so a step covers eight rows.  Every LDS array is
// private to its wavefront until the closing block reduction.
constexpr int kRowsWin = 256;          // rows per wavefront window
constexpr int kRowsWinEntries = 1024;  // a window's entries copied to LDS (at most)
constexpr int kRowsPhase = 16;         // rows whose tile is built at once
// per wavefront: hash, start, end (kRowsWin each) | kRowsPhase x 64 tile | entries' columns, values
constexpr int kRowsWaveWords = 3 * kRowsWin + kRowsPhase * 64 + 2 * kRowsWinEntries;

template <int NB>
constexpr int rows_lds_elems() {
  return red_elems<float, NB>() > kWaves * kRowsWaveWords ? red_elems<float, NB>()
                                                          : kWaves * kRowsWaveWords;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// TAG 1: the rows of G (S X) as above.  TAG 2: the dense Gaussian product
// G~ X, summed the same way over the nonempty rows r with column r of G~
// (global row row_offset + r, no sign) in place of sigma(r) G[:, h(r)]; the
// compacted row records then hold the local row index instead of the hash.
template <int NB, bool HALF, int TAG = 1>
__device__ __forceinline__ void gx_rows_block(const GsxArgs& a, int64_t bx, int group, int ng,
                                              float* lds) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = lane & 15, kq = lane >> 4;
  uint32_t* rh = (uint32_t*)lds + wave * kRowsWaveWords;
  int32_t* rs = (int32_t*)(rh + kRowsWin);
  int32_t* re = rs + kRowsWin;
  float* tile = (float*)(re + kRowsWin);
  int32_t* ecol = (int32_t*)(tile + kRowsPhase * 64);
  float* eval = (float*)(ecol + kRowsWinEntries);
  constexpr int STEP = HALF ? 8 : 4;   // compacted rows per MFMA step
  const uint32_t q = (uint32_t)(16 * group + (HALF ? (p & 7) : p));
  const int n0 = ng * NB * 16, d = a.d, m = a.m;
  const int32_t nnz = a.nnz;
  const int32_t* __restrict__ row_ptr = a.row_ptr;
  const int32_t* __restrict__ col_idx = a.col_idx;
  const float* __restrict__ vals = a.vals;
  v4f acc[4][NB];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[t][nb] = v4f{0, 0, 0, 0};
  const int64_t w0 = (bx * kWaves + wave) * (int64_t)a.kc;
  const int64_t w1 = min(w0 + (int64_t)a.kc, a.n);
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int64_t r0 = w0; r0 < w1; r0 += kRowsWin) {
    // this lane's rows r0 + 4 lane + j: bounds (clamped, non-decreasing)
    // and packed hashes
    const int64_t rl = r0 + 4 * lane;
    int32_t rp[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) rp[j] = min(max(row_ptr[min(rl + j, w1)], 0), nnz);
#pragma unroll
    for (int j = 1; j < 5; ++j) rp[j] = max(rp[j], rp[j - 1]);
    uint32_t hv[4] = {0u, 0u, 0u, 0u};
    if constexpr (TAG == 1) {
      if (rl < w1) hash4(a.row_offset + (uint64_t)rl, (uint32_t)a.B, a.key.k0, a.key.k1, hv);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) hv[j] = (uint32_t)(rl + j);
    }
    // compaction in row order: the rank of row (lane, j) is the number of
    // nonempty rows of lower lanes plus this lane's before j
    uint64_t mk[4];
    int ne = 0;
    uint32_t rank = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      mk[j] = __ballot(rp[j + 1] > rp[j]);
      ne += __popcll(mk[j]);
      rank += __popcll(mk[j] & lt);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (rp[j + 1] > rp[j]) {
        rh[rank] = hv[j];
        rs[rank] = rp[j];
        re[rank] = rp[j + 1];
        ++rank;
      }
    wave_sync();
    // the window's entries [es, ee): into LDS when they fit, four
    // independent loads per lane at a time
    const int32_t es = ne ? rs[0] : 0, ee = ne ? re[ne - 1] : 0;
    const int32_t cnt = ee > es ? ee - es : 0;
    const bool bulk = cnt <= kRowsWinEntries;
    if (bulk) {
      for (int32_t i0 = 0; i0 < cnt; i0 += 256) {
        int32_t cc[4];
        float vv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t k = es + min(i0 + lane + 64 * u, cnt - 1);
          cc[u] = col_idx[k];
          vv[u] = vals[k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + lane + 64 * u < cnt) {
            ecol[i0 + lane + 64 * u] = cc[u];
            eval[i0 + lane + 64 * u] = vv[u];
          }
      }
      wave_sync();
    }
    for (int e0 = 0; e0 < ne; e0 += kRowsPhase) {
      const int eN = min(e0 + kRowsPhase, ne);
      // the phase's rows laid out dense: tile[i][c - n0] for row e0 + i
#pragma unroll
      for (int i = lane; i < kRowsPhase * 16; i += 64) ((v4f*)tile)[i] = v4f{0, 0, 0, 0};
      // the starts of rows e0 + 1 .. e0 + kRowsPhase - 1 as wavefront-uniform
      // values (rows past eN never match)
      const int32_t my_start = lane < kRowsPhase && e0 + lane < eN ? rs[e0 + lane] : INT32_MAX;
      int32_t st[kRowsPhase];
#pragma unroll
      for (int i = 1; i < kRowsPhase; ++i) st[i] = __builtin_amdgcn_readlane(my_start, i);
      wave_sync();
      const int32_t k0 = rs[e0], k1 = re[eN - 1];
      for (int32_t k = k0 + lane; k < k1; k += 64) {
        int t = 0;
#pragma unroll
        for (int i = 1; i < kRowsPhase; ++i) t += k >= st[i] ? 1 : 0;
        // (k - es is inside the copied segment for well-formed row_ptr;
        // clamped all the same, like every index taken from row_ptr)
        const int32_t kl = min(max(k - es, 0), kRowsWinEntries - 1);
        const int32_t c = bulk ? ecol[kl] : col_idx[k];
        const float v = bulk ? eval[kl] : vals[k];
        if (c >= n0 && c < n0 + 16 * NB && c < d) atomicAdd(&tile[t * 64 + (c - n0)], v);
      }
      wave_sync();
      // the phase's MFMA steps, STEP rows each, with no LDS fence between them
#pragma unroll
      for (int s0 = 0; s0 < kRowsPhase; s0 += STEP) {
        if (e0 + s0 >= eN) break;
        // A: the normals of this lane's row (lanes p >= 8 of a half group:
        // the row four further on), sign applied, zero past the last row
        const int e = e0 + s0 + (HALF ? 4 * (p >> 3) : 0) + kq;
        const bool ok = e < eN;
        const uint32_t hp = ok ? rh[e] : 0u;
        float g[4];
        float sg;
        if constexpr (TAG == 1) {
          box_muller(gauss_block(hash_bucket(hp), q, a.key.k0, a.key.k1), g);
          sg = ok ? (hash_negative(hp) ? -1.0f : 1.0f) : 0.0f;
        } else {
          box_muller(dense_gauss_block(a.row_offset + (uint64_t)hp, q, a.key.k0, a.key.k1), g);
          sg = ok ? 1.0f : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) g[t] *= sg;
        if constexpr (HALF) {
          // paired M blocks as in the contraction kernel's half groups: rows
          // 4q, 4q + 1 and 4q + 2, 4q + 3, lanes p < 8 holding step h = 0's
          // rows and p >= 8 step h = 1's
          const float m1 = from_lane_m8(g[1]), m3 = from_lane_m8(g[3]);
          const float p0 = from_lane_p8(g[0]), p2 = from_lane_p8(g[2]);
          const bool lo = p < 8;
          const float av[2][2] = {{lo ? g[0] : m1, lo ? g[2] : m3}, {lo ? p0 : g[1], lo ? p2 : g[3]}};
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            float xv[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) xv[nb] = tile[(s0 + 4 * h + kq) * 64 + nb * 16 + p];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
              for (int nb = 0; nb < NB; ++nb) acc[t][nb] = mfma_k4(av[h][t], xv[nb], acc[t][nb]);
          }
        } else {
          float xv[NB];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) xv[nb] = tile[(s0 + kq) * 64 + nb * 16 + p];
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[t][nb] = mfma_k4(g[t], xv[nb], acc[t][nb]);
        }
      }
      wave_sync();   // the tile's reads come before the next phase's zeroing
    }
  }
  __syncthreads();   // every wavefront is done with its LDS before the block reduction reuses it
  block_reduce_store<float, NB, v4f, false, HALF>(acc, lds, wave, lane, group, n0, m, d,
                                                  a.part + (size_t)bx * m * d);
}

template <int NB, int TAG>
__global__ __launch_bounds__(kThreads) void gx_rows_kernel(GsxArgs a) {
  __shared__ __align__(16) float lds[rows_lds_elems<NB>()];
  if (half_group(a.m, (int)blockIdx.y))
    gx_rows_block<NB, true, TAG>(a, blockIdx.x, blockIdx.y, blockIdx.z, lds);
  else
    gx_rows_block<NB, false, TAG>(a, blockIdx.x, blockIdx.y, blockIdx.z, lds);
}

// Batched forms: item -> instance from the item table; the local index is
// split into (part, row group, column group) with the part fastest.  One
// kernel per width NB (16-column blocks per wavefront), launched over the
// items of the instances of that width: `base` is the first of them in the
// queue.
template <int NB>
__global__ __launch_bounds__(kThreads) void gsx_batched_kernel(const GsxArgs* __restrict__ args,
                                                               const int32_t* __restrict__ inst,
                                                               const int32_t* __restrict__ first,
                                                               int64_t base) {
  const int64_t item = base + blockIdx.x;
  const int i = inst[item];
  const GsxArgs a = args[i];
  int64_t j = item - first[i];
  const int64_t bx = j % a.parts;
  j /= a.parts;
  const int group = (int)(j % a.mgroups);
  const int ng = (int)(j / a.mgroups);
  __shared__ __align__(16) float red[rows_lds_elems<NB>()];
  const bool half = half_group(a.m, group);
  if (a.route == 1) {
    if (half)
      gx_rows_block<NB, true>(a, bx, group, ng, red);
    else
      gx_rows_block<NB, false>(a, bx, group, ng, red);
  } else if (half) {
    gsx_native_block<float, NB, true>(a.SX, a.d, 0, a.B, a.d, a.m, a.kc, a.key, a.part, bx, group, ng,
                                      red);
  } else {
    gsx_native_block<float, NB, false>(a.SX, a.d, 0, a.B, a.d, a.m, a.kc, a.key, a.part, bx, group,
                                       ng, red);
  }
}

__global__ __launch_bounds__(64 * kRedWaves) void splitk_batched_kernel(
    const GsxArgs* __restrict__ args, const int32_t* __restrict__ inst,
    const int32_t* __restrict__ first) {
  const int i = inst[blockIdx.x];
  const GsxArgs a = args[i];
  splitk_reduce_block<float>(a.part, a.parts, (int64_t)a.m * a.d, a.Y,
                             (int64_t)blockIdx.x - first[i]);
}

template <typename T, int NB, int TAG = 1>
void launch_native(const GsxPlan& pl, const T* SX, int64_t B, int d, int m, Key key, T* part,
                   hipStream_t s, int64_t ld = -1, uint64_t col0 = 0) {
  dim3 grid((unsigned)pl.parts, (unsigned)pl.mgroups, (unsigned)pl.ngroups);
  // FP32 with every row group full (no group of 32 rows or fewer): the
  // producer/consumer form; same partials
  if constexpr (sizeof(T) == 4) {
    if (m % 64 == 0 || m % 64 > 32) {
      gsx_pc_kernel<NB, TAG><<<grid, 2 * kThreads, 0, s>>>(SX, ld < 0 ? (int64_t)d : ld, col0, B, d,
                                                            m, pl.kc, key, part);
      return;
    }
  }
  gsx_native_kernel<T, NB, TAG><<<grid, kThreads, 0, s>>>(SX, ld < 0 ? (int64_t)d : ld, col0, B, d,
                                                           m, pl.kc, key, part);
}

template <int NB, bool FP8>
void launch_lowp(const GsxPlan& pl, const float* SX, int64_t B, int d, int m, Key key,
                 float2* bscale, float* part, hipStream_t s, bool scales_ready = false) {
  if constexpr (FP8) {
    if (!scales_ready) {
    const int64_t nblk = (B + 127) / 128;
    fp8_block_scale_kernel<<<(unsigned)((nblk + kWaves - 1) / kWaves), kThreads, 0, s>>>(SX, B, d,
                                                                                      bscale);
    }
  }
  // parts per launch: every row a launch reads (its chunks plus the
  // prefetch one step past them) lies within 2^30 / d rows of its first,
  // so byte offsets from that row fit in 32 bits
  const int64_t rows_per_part = (int64_t)kWaves * pl.kc;
  const int64_t max_rows = ((int64_t)1 << 30) / d;
  const int64_t per = max((int64_t)1, max_rows / rows_per_part - 1);
  const bool vec = (NB == 2 || NB == 4) && d % (16 * NB) == 0;
  for (int64_t bx0 = 0; bx0 < pl.parts; bx0 += per) {
    const int64_t np = min(per, pl.parts - bx0);
    const int64_t row0 = bx0 * rows_per_part;
    dim3 grid((unsigned)np, (unsigned)pl.mgroups, (unsigned)pl.ngroups);
    if (vec)
      gsx_lowp_pc_kernel<NB, FP8, (NB == 2 || NB == 4)><<<grid, 2 * kThreads, 0, s>>>(
          SX + row0 * d, row0, bx0, B, d, m, pl.kc, key, bscale, part);
    else
      gsx_lowp_pc_kernel<NB, FP8, false><<<grid, 2 * kThreads, 0, s>>>(SX + row0 * d, row0, bx0, B,
                                                                      d, m, pl.kc, key, bscale, part);
  }
}

}  // namespace

GsxPlan plan_gsx(int64_t m, int64_t B, int64_t d, Prec prec, int kc_request, size_t elem) {
  GsxPlan pl;
  pl.waves = kWaves;
  const int max_nb = elem == 8 ? 2 : 4;
  const int need = (int)((d + 15) / 16);
  pl.nb = need < max_nb ? need : max_nb;
  pl.ngroups = (int)((d + 16 * pl.nb - 1) / (16 * pl.nb));
  pl.mgroups = (int)((m + 63) / 64);
  const int gran = prec == Prec::FP8 ? 128 : prec == Prec::BF16 ? 32 : 16;
  int64_t kc = kc_request;
  if (kc <= 0) {
    // about 2048 wavefronts (8 per CU) over the whole product, and at least
    // 64 columns each: fewer, longer chunks than that cost more in split
    // partials (written and reduced) than they gain in parallelism, and
    // longer ones leave CUs idle (measured at m = 64, d = 32 and 64)
    // (the reduced-precision contraction: about 1024 consumer wavefronts,
    // each with a producer wavefront beside it)
    const int64_t target = prec == Prec::Native ? 2048 : 1024;
    const int64_t units = (int64_t)pl.mgroups * pl.ngroups;
    kc = (B * units + target - 1) / target;
    // ... unless 64-column chunks leave fewer than 1024 wavefronts (a
    // small B): then chunks down to the granule, for about 1024 of them, so
    // that the wavefronts' chains of steps stay short
    if (kc < 64) kc = (B * units + 63) / 64 >= 1024 ? 64 : (B * units + 1023) / 1024;
    if (kc > 8192) kc = 8192;
  }
  // at most 2^23 workgroups along B (a grid holds fewer than 2^32 work-items)
  const int64_t kc_min = (B + (int64_t)kWaves * (1 << 23) - 1) / ((int64_t)kWaves * (1 << 23));
  if (kc < kc_min) kc = kc_min;
  kc = (kc + gran - 1) / gran * gran;
  if (kc < gran) kc = gran;
  pl.kc = (int)kc;
  pl.parts = (B + (int64_t)kWaves * kc - 1) / ((int64_t)kWaves * kc);
  return pl;
}

size_t fp8_scale_bytes(int64_t B) { return align256((size_t)((B + 127) / 128) * sizeof(float2)); }

template <typename T>
hipError_t launch_gsx_partials(const GsxPlan& pl, Prec prec, const T* SX, int64_t B, int d, int m,
                               Key key, T* part, hipStream_t s, void* scales, bool scales_ready) {
  if constexpr (sizeof(T) == 8) {
    if (pl.nb == 1)
      launch_native<T, 1>(pl, SX, B, d, m, key, part, s);
    else
      launch_native<T, 2>(pl, SX, B, d, m, key, part, s);
  } else {
    if (prec == Prec::Native) {
      switch (pl.nb) {
        case 1: launch_native<T, 1>(pl, SX, B, d, m, key, part, s); break;
        case 2: launch_native<T, 2>(pl, SX, B, d, m, key, part, s); break;
        case 3: launch_native<T, 3>(pl, SX, B, d, m, key, part, s); break;
        default: launch_native<T, 4>(pl, SX, B, d, m, key, part, s); break;
      }
    } else if (prec == Prec::BF16) {
      switch (pl.nb) {
        case 1: launch_lowp<1, false>(pl, SX, B, d, m, key, nullptr, part, s); break;
        case 2: launch_lowp<2, false>(pl, SX, B, d, m, key, nullptr, part, s); break;
        case 3: launch_lowp<3, false>(pl, SX, B, d, m, key, nullptr, part, s); break;
        default: launch_lowp<4, false>(pl, SX, B, d, m, key, nullptr, part, s); break;
      }
    } else {
      switch (pl.nb) {
        case 1: launch_lowp<1, true>(pl, SX, B, d, m, key, (float2*)scales, part, s, scales_ready); break;
        case 2: launch_lowp<2, true>(pl, SX, B, d, m, key, (float2*)scales, part, s, scales_ready); break;
        case 3: launch_lowp<3, true>(pl, SX, B, d, m, key, (float2*)scales, part, s, scales_ready); break;
        default: launch_lowp<4, true>(pl, SX, B, d, m, key, (float2*)scales, part, s, scales_ready); break;
      }
    }
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_splitk_reduce(const T* part, int64_t parts, int64_t md, T* Y, hipStream_t s) {
  splitk_reduce_kernel<T><<<(unsigned)((md + 63) / 64), 64 * kRedWaves, 0, s>>>(part, parts, md, Y);
  return hipGetLastError();
}

template <int TAG>
static void launch_rows(const GsxArgs& a, int nb, dim3 grid, hipStream_t s) {
  switch (nb) {
    case 1: gx_rows_kernel<1, TAG><<<grid, kThreads, 0, s>>>(a); break;
    case 2: gx_rows_kernel<2, TAG><<<grid, kThreads, 0, s>>>(a); break;
    case 3: gx_rows_kernel<3, TAG><<<grid, kThreads, 0, s>>>(a); break;
    default: gx_rows_kernel<4, TAG><<<grid, kThreads, 0, s>>>(a); break;
  }
}

hipError_t launch_rows_partials(const GsxArgs& a0, hipStream_t s, bool dense_gaussian) {
  GsxArgs a = a0;
  a.kc = rows_per_wave(a.n);
  const int64_t parts = rows_parts(a.n, a.kc);
  const int nb = a.d >= 64 ? 4 : (a.d + 15) / 16;
  const int mgroups = (a.m + 63) / 64, ngroups = (a.d + 16 * nb - 1) / (16 * nb);
  dim3 grid((unsigned)parts, (unsigned)mgroups, (unsigned)ngroups);
  if (dense_gaussian)
    launch_rows<2>(a, nb, grid, s);
  else
    launch_rows<1>(a, nb, grid, s);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dense_gaussian_partials(const GsxPlan& pl, const T* X, int64_t ldx, int64_t n,
                                          int d, int m, Key key, uint64_t row_offset, T* part,
                                          hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    if (pl.nb == 1)
      launch_native<T, 1, 2>(pl, X, n, d, m, key, part, s, ldx, row_offset);
    else
      launch_native<T, 2, 2>(pl, X, n, d, m, key, part, s, ldx, row_offset);
  } else {
    switch (pl.nb) {
      case 1: launch_native<T, 1, 2>(pl, X, n, d, m, key, part, s, ldx, row_offset); break;
      case 2: launch_native<T, 2, 2>(pl, X, n, d, m, key, part, s, ldx, row_offset); break;
      case 3: launch_native<T, 3, 2>(pl, X, n, d, m, key, part, s, ldx, row_offset); break;
      default: launch_native<T, 4, 2>(pl, X, n, d, m, key, part, s, ldx, row_offset); break;
    }
  }
  return hipGetLastError();
}

template hipError_t launch_dense_gaussian_partials<float>(const GsxPlan&, const float*, int64_t,
                                                          int64_t, int, int, Key, uint64_t, float*,
                                                          hipStream_t);
template hipError_t launch_dense_gaussian_partials<double>(const GsxPlan&, const double*, int64_t,
                                                           int64_t, int, int, Key, uint64_t,
                                                           double*, hipStream_t);

hipError_t launch_gsx_batched(const GsxArgs* args, const int32_t* gsx_inst,
                              const int32_t* gsx_first, const int64_t items_by_nb[4],
                              hipStream_t s) {
  int64_t base = 0;
  for (int k = 0; k < 4; ++k) {
    const int64_t n = items_by_nb[k];
    if (n > 0) {
      switch (k) {
        case 0: gsx_batched_kernel<1><<<(unsigned)n, kThreads, 0, s>>>(args, gsx_inst, gsx_first, base); break;
        case 1: gsx_batched_kernel<2><<<(unsigned)n, kThreads, 0, s>>>(args, gsx_inst, gsx_first, base); break;
        case 2: gsx_batched_kernel<3><<<(unsigned)n, kThreads, 0, s>>>(args, gsx_inst, gsx_first, base); break;
        default: gsx_batched_kernel<4><<<(unsigned)n, kThreads, 0, s>>>(args, gsx_inst, gsx_first, base); break;
      }
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    base += n;
  }
  return hipSuccess;
}

hipError_t launch_splitk_batched(const GsxArgs* args, const int32_t* red_inst,
                                 const int32_t* red_first, int64_t items, hipStream_t s) {
  if (items > 0)
    splitk_batched_kernel<<<(unsigned)items, 64 * kRedWaves, 0, s>>>(args, red_inst, red_first);
  return hipGetLastError();
}

template hipError_t launch_gsx_partials<float>(const GsxPlan&, Prec, const float*, int64_t, int,
                                               int, Key, float*, hipStream_t, void*, bool);
template hipError_t launch_gsx_partials<double>(const GsxPlan&, Prec, const double*, int64_t, int,
                                                int, Key, double*, hipStream_t, void*, bool);
template hipError_t launch_splitk_reduce<float>(const float*, int64_t, int64_t, float*,
                                                hipStream_t);
template hipError_t launch_splitk_reduce<double>(const double*, int64_t, int64_t, double*,
                                                 hipStream_t);

}  // namespace cg
