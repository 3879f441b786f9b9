// Device-side random source of the CountGauss transform.
//
// The paper asks for a CountSketch S with independent uniform buckets and
// fair +-1 signs and a Gaussian G with i.i.d. unit-variance entries
// (Section 1.1; Theorem 1).  It names no generator.  Both are produced here
// as pure functions of (seed, index) by the counter-based Philox4x32-10
// generator of Salmon, Moraes, Dror and Shaw (SC'11), so that S and G are
// never stored and any row range or column block can be regenerated where
// it is consumed:
//
//   key                = (lo32(seed), hi32(seed))
//   row hash, tag 0    : counter (lo32(r>>2), hi32(r>>2), 0, 0); the four
//                        output words serve rows 4q..4q+3.  For word w:
//                        sigma = bit 31 of w ? -1 : +1,
//                        h     = ((w & 0x7fffffff) * B) >> 31
//   Gaussian, tag 1    : G[i][b] from counter (b, i>>2, 1, 0); the four
//                        words give four normals by Box-Muller for rows
//                        4q..4q+3 of column b.
//   uniform            : u = ((w >> 9) + 1/2) * 2^-23 in (0, 1), exact in
//                        FP32 and FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cg {

struct Words4 {
  uint32_t x, y, z, w;
};

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// a ^ b ^ c in one gfx950 v_bitop3_b32 (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Ten Philox rounds.  The key words are wave-uniform in every caller, so the
// compiler keeps the key schedule in scalar registers.  Each round is two
// 32 x 32 -> 64-bit products and two three-way xors.
__device__ __forceinline__ Words4 philox10(Words4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
    const Words4 n = {xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                      xor3((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0};
    c = n;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return c;
}

__device__ __forceinline__ uint32_t word_at(const Words4& w, int i) {
  return i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w;
}

// Words for row quad q (tag 0).  The empty asm makes the key words opaque
// here, so the round keys are formed with scalar adds at each call instead
// of being hoisted out of the caller's loop into twenty scalar registers
// (which the row-splitting kernels would spill).
__device__ __forceinline__ Words4 hash_block(uint64_t q, uint32_t k0, uint32_t k1) {
  asm volatile("" : "+s"(k0), "+s"(k1));
  return philox10(Words4{(uint32_t)q, (uint32_t)(q >> 32), 0u, 0u}, k0, k1);
}

// Packed (bucket | sign << 31) of one hash word; bucket < B <= 2^31 - 1.
__device__ __forceinline__ uint32_t pack_hash(uint32_t w, uint32_t B) {
  const uint32_t bucket = (uint32_t)(((uint64_t)(w & 0x7fffffffu) * B) >> 31);
  return bucket | (w & 0x80000000u);
}

// Packed hashes of the four consecutive global rows g, g+1, g+2, g+3.
// One Philox call when g is a multiple of four, two otherwise.
__device__ __forceinline__ void hash4(uint64_t g, uint32_t B, uint32_t k0, uint32_t k1,
                                      uint32_t out[4]) {
  const uint64_t q = g >> 2;
  const int s = (int)(g & 3);
  const Words4 a = hash_block(q, k0, k1);
  if (s == 0) {
    out[0] = pack_hash(a.x, B);
    out[1] = pack_hash(a.y, B);
    out[2] = pack_hash(a.z, B);
    out[3] = pack_hash(a.w, B);
  } else {
    const Words4 b = hash_block(q + 1, k0, k1);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = s + t;
      out[t] = pack_hash(j < 4 ? word_at(a, j) : word_at(b, j - 4), B);
    }
  }
}

__device__ __forceinline__ uint32_t hash_bucket(uint32_t packed) { return packed & 0x7fffffffu; }
__device__ __forceinline__ bool hash_negative(uint32_t packed) { return (packed >> 31) != 0u; }

// Words of Gaussian column b, row quad q (tag 1).
__device__ __forceinline__ Words4 gauss_block(uint32_t b, uint32_t q, uint32_t k0, uint32_t k1) {
  return philox10(Words4{b, q, 1u, 0u}, k0, k1);
}

// Words of the dense Gaussian G~ (m x n, the product T X stands in for)
// column r -- a global row index of X -- row quad q (tag 2): counter
// (lo32(r), q, 2, hi32(r)).
__device__ __forceinline__ Words4 dense_gauss_block(uint64_t r, uint32_t q, uint32_t k0,
                                                    uint32_t k1) {
  return philox10(Words4{(uint32_t)r, q, 2u, (uint32_t)(r >> 32)}, k0, k1);
}

// 0x3f800000 | (w >> 9) is 1 + (w >> 9) 2^-23 (one v_alignbit_b32);
// subtracting 1 - 2^-24 leaves ((w >> 9) + 1/2) 2^-23 exactly (both
// operands and the difference are representable: Sterbenz).
__device__ __forceinline__ float unit_f32(uint32_t w) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, w, 9u)) - 0x1.fffffep-1f;
}
__device__ __forceinline__ double unit_f64(uint32_t w) {
  return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

// Box-Muller, FP32, on the hardware transcendental units: v_log_f32
// (log2, so -2 ln u = -2 ln 2 log2 u), v_sqrt_f32, and v_sin_f32 /
// v_cos_f32, whose argument is in revolutions (sin(2 pi u) = v_sin(u)).
// Measured on gfx950 against FP64 over 2^22 (u0, u1) pairs: largest
// absolute error 8.5e-7, rms 6.1e-8 -- about what the device library's
// logf/sqrtf/sincospif give (7.4e-7, 5.1e-8), since the error is dominated
// by u itself being FP32 -- at three times the rate.
// `rscale` (a power of two) scales the radii, and so the four normals,
// exactly: the reduced-precision contraction draws G 2^6 for its FP8
// operand at the cost of two multiplies instead of four.
__device__ __forceinline__ void box_muller(const Words4& w, float z[4], float rscale = 1.0f) {
  constexpr float kNeg2Ln2 = -1.3862943611198906f;
  const float r0 = rscale * __builtin_amdgcn_sqrtf(kNeg2Ln2 * __builtin_amdgcn_logf(unit_f32(w.x)));
  const float r1 = rscale * __builtin_amdgcn_sqrtf(kNeg2Ln2 * __builtin_amdgcn_logf(unit_f32(w.z)));
  const float u1 = unit_f32(w.y), u3 = unit_f32(w.w);
  z[0] = r0 * __builtin_amdgcn_cosf(u1);
  z[1] = r0 * __builtin_amdgcn_sinf(u1);
  z[2] = r1 * __builtin_amdgcn_cosf(u3);
  z[3] = r1 * __builtin_amdgcn_sinf(u3);
}

// Box-Muller, FP64.
__device__ __forceinline__ void box_muller(const Words4& w, double z[4]) {
  const double r0 = sqrt(-2.0 * log(unit_f64(w.x)));
  const double r1 = sqrt(-2.0 * log(unit_f64(w.z)));
  double s0, c0, s1, c1;
  sincospi(2.0 * unit_f64(w.y), &s0, &c0);
  sincospi(2.0 * unit_f64(w.w), &s1, &c1);
  z[0] = r0 * c0;
  z[1] = r0 * s0;
  z[2] = r1 * c1;
  z[3] = r1 * s1;
}

}  // namespace cg
