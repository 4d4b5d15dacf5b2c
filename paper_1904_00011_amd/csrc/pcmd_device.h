// Device-side building blocks shared by the gfx950 kernels: the counter-based generator, the
// FP32 logarithm and ln k! used by the rejection sampler, and the sampler rules themselves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcmd {

// Philox4x32-10 (Salmon et al., SC'11): multipliers and Weyl key increments.
constexpr uint32_t PH_M0 = 0xD2511F53u;
constexpr uint32_t PH_M1 = 0xCD9E8D57u;
constexpr uint32_t PH_W0 = 0x9E3779B9u;
constexpr uint32_t PH_W1 = 0xBB67AE85u;

// Stream tags (counter word 2).
constexpr uint32_t TAG_MAIN = 0, TAG_SPLIT = 1, TAG_SPLIT_X = 2, TAG_PTRS = 3, TAG_DUST = 4, TAG_NOISE = 5;
// block-skip sampler: block total by inversion / rejection, star placement, star dust screen
constexpr uint32_t TAG_BLOCK = 6, TAG_BLOCK_PTRS = 7, TAG_STAR = 8, TAG_STAR_SPLIT = 9;
// thinned entries: the reddened part's word (p, i / 4, TAG_RED, 0) and rejection attempts
constexpr uint32_t TAG_RED = 10, TAG_PTRS_RED = 11;

// Entry kinds written by the preparation kernel (low four bits of a record's kk), and the flag of
// a table entry whose unreddened and reddened counts are drawn as two thinned parts.
constexpr uint32_t KIND_ZERO = 0, KIND_INV = 1, KIND_PTRS = 2, KIND_ALIAS = 3;
constexpr uint32_t KIND_MASK = 0x0Fu, FLAG_THIN = 0x80u;
// Dust split F = 1/2: table entries at or above this lambda are thinned; the others keep one bit
// per star.  4 is the lowest lambda whose halves (>= ALIAS_MIN) still take the alias rule, and
// from about there on nearly every 64-pixel wave has a lane with more than the 8 stars that the
// shared split block covers, so a bit per star would cost a Philox block per entry, where the
// thinned entry costs a quarter block and a second table read.
constexpr double LAM_THIN_HALF = 4.0;
// Alias rule for ALIAS_MIN <= lambda < ALIAS_MAX: M = 2^b <= ALIAS_COLS columns of 2^(32-b) words
// each (column = top b bits of the inversion word), one packed word per column:
// height << b | alias.  Each entry's table has room for ALIAS_COLS columns.
constexpr double ALIAS_MIN = 2.0, ALIAS_MAX = 512.0;
constexpr int ALIAS_COLS = 512;
constexpr int THR_STRIDE = 64;       // thresholds per entry slot (K <= 63)
constexpr int CHUNK = 1024;          // entries per slice, at most (sample_slices)
constexpr int PTRS_MAX_ATTEMPTS = 64;

// Slices of the sampler for E entries over npx pixels: one per CHUNK entries, more for small
// images (up to one per 16-entry block) until the 256-pixel blocks x slices reach 512 workgroups,
// so that a small image still spreads over the chip.  A function of (E, npx) alone: a batch job
// gets the slices of the same single call, and so the same partial sums.
__host__ __device__ inline int sample_slices(int E, int64_t npx) {
  const int64_t base = (E + CHUNK - 1) / CHUNK, blocks16 = (E + 15) / 16;
  const int64_t pblocks = (npx + 255) / 256, want = (512 + pblocks - 1) / pblocks;
  const int64_t small = blocks16 < want ? blocks16 : want;
  return (int)(base > small ? base : small);
}

struct u4 { uint32_t x, y, z, w; };

// Every counter used here is (lane-varying word, uniform, uniform, uniform), so the first three
// rounds still mix uniform words (their XORs go to the scalar unit); from the fourth round on all
// three XOR inputs are per lane and one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c) replaces two
// v_xor_b32.  The XOR order does not change the result.
__device__ __forceinline__ uint32_t xor3_lane(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96u);
}

__device__ __forceinline__ u4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)PH_M0 * c0;
    const uint64_t p1 = (uint64_t)PH_M1 * c2;
    uint32_t n0, n2;
    if (r < 2) {
      n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
      n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    } else if (r == 2) {
      // c3 is still uniform here (the low half of a product of uniform words): XOR it into the
      // key on the scalar unit first, since a vector instruction reads at most one scalar
      // operand and a three-input XOR of two would need a v_mov
      n0 = xor3_lane((uint32_t)(p1 >> 32), c1, k0);
      n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
    } else {
      n0 = xor3_lane((uint32_t)(p1 >> 32), c1, k0);
      n2 = xor3_lane((uint32_t)(p0 >> 32), c3, k1);
    }
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += PH_W0;
    k1 += PH_W1;
  }
  return u4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t word_of(const u4 &w, int q) {
  return q == 0 ? w.x : q == 1 ? w.y : q == 2 ? w.z : w.w;
}

// 32-bit word -> (0,1) with 24 significant bits, exact in FP32.
__device__ __forceinline__ float u01_f32(uint32_t w) {
  return ((float)(w >> 9) + 0.5f) * 1.1920928955078125e-07f;  // 2^-23
}
// 32-bit word -> (0,1), exact in FP64.
__device__ __forceinline__ double u01_f64(uint32_t w) {
  return ((double)w + 0.5) * 2.3283064365386963e-10;  // 2^-32
}

__device__ __forceinline__ double box_muller(uint32_t w0, uint32_t w1) {
  const double u1 = u01_f64(w0), u2 = u01_f64(w1);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// ---------------------------------------------------------------------------------------
// FP32 decision path of the rejection sampler.  Every step is a single correctly rounded
// IEEE operation; contraction into fused multiply-adds is off so that the result is the same
// integer on every IEEE implementation that takes the same steps.
// ---------------------------------------------------------------------------------------
#pragma clang fp contract(off)

// ln x for positive normal x: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s) = s (2 + s^2 (2/3 + s^2 (2/5 + ...))), s = (m - 1)/(m + 1).
__device__ __forceinline__ float ln_f32(float x) {
  const uint32_t bits = __float_as_uint(x);
  int e = (int)((bits >> 23) & 0xFFu) - 127;
  float m = __uint_as_float((bits & 0x007FFFFFu) | 0x3F800000u);
  if (m > 1.41421353816986083984375f) {
    m = m * 0.5f;
    e += 1;
  }
  const float s = (m - 1.0f) / (m + 1.0f);
  const float z = s * s;
  float P = (float)(2.0 / 11.0);
  P = P * z + (float)(2.0 / 9.0);
  P = P * z + (float)(2.0 / 7.0);
  P = P * z + (float)(2.0 / 5.0);
  P = P * z + (float)(2.0 / 3.0);
  P = P * z + 2.0f;
  const float ef = (float)e;
  const float ln2_hi = 0.693145751953125f;
  const float ln2_lo = 1.428606765330187e-06f;
  return ef * ln2_hi + (ef * ln2_lo + s * P);
}

// ln k! : table below 256 (FP64-built, rounded), Stirling series in x = k + 1 above.
__device__ __forceinline__ float lnfact_f32(float kf, const float *__restrict__ table) {
  if (kf < 256.0f) return table[(int)kf];
  const float x = kf + 1.0f;
  const float lx = ln_f32(x);
  float t = (x - 0.5f) * lx;
  t = t - x;
  t = t + 0.9189385332046727f;
  const float r = 1.0f / x;
  t = t + r * (float)(1.0 / 12.0);
  const float r3 = (r * r) * r;
  t = t - r3 * (float)(1.0 / 360.0);
  return t;
}

// Per-entry constants of the transformed rejection (Hormann 1993), FP32.
struct PtrsConst {
  float mu, lnmu, b, a, twoa, lninva, vr, pad;
};

// One attempt.  Returns true if accepted and writes k.
__device__ __forceinline__ bool ptrs_attempt(const PtrsConst &c, uint32_t wu, uint32_t wv,
                                             const float *__restrict__ lnfact_table, int &k_out) {
  const float u = u01_f32(wu);
  const float V = u01_f32(wv);
  const float U = u - 0.5f;
  const float us = 0.5f - fabsf(U);
  float t = c.twoa / us;
  t = t + c.b;
  t = t * U;
  t = t + c.mu;
  t = t + 0.43f;
  const float kf = floorf(t);
  k_out = (int)kf;
  if (us >= 0.07f && V <= c.vr) return true;
  if (kf < 0.0f || (us < 0.013f && V > us)) return false;
  float q = c.a / (us * us);
  q = q + c.b;
  const float lhs = (ln_f32(V) + c.lninva) - ln_f32(q);
  const float rhs = ((-c.mu) + kf * c.lnmu) - lnfact_f32(kf, lnfact_table);
  return lhs <= rhs;
}

// Tables that are only read while sampling: reading them through the constant address space
// lets the wave-uniform loads go through the scalar cache.
#define PCMD_CONST __attribute__((address_space(4)))

// Copy a struct out of constant-address-space memory word by word (scalar loads).
template <typename T>
__device__ __forceinline__ T ld_const(const PCMD_CONST T *p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized structs only");
  T v;
  uint32_t *d = reinterpret_cast<uint32_t *>(&v);
  const PCMD_CONST uint32_t *s = reinterpret_cast<const PCMD_CONST uint32_t *>(p);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) d[k] = s[k];
  return v;
}

__device__ __forceinline__ bool wave_any(bool v) { return __ballot(v) != 0ull; }

// Transformed-rejection draw of stream (p, i, tag): attempts 2j, 2j+1 use words (0,1), (2,3) of
// Philox(p, i, tag, j).  A lane that exhausts PTRS_MAX_ATTEMPTS draws 0 and sets `failed`
// (reported once per wave by the caller, so the loop holds no store).
__device__ __forceinline__ uint32_t ptrs_draw(const PtrsConst &c, uint32_t p, uint32_t i, uint32_t tag, uint32_t k0,
                                              uint32_t k1, const float *__restrict__ lnfact, uint32_t &failed) {
  int k = 0;
  bool done = false;
  for (uint32_t j = 0; j < (uint32_t)(PTRS_MAX_ATTEMPTS / 2); ++j) {
    const u4 w = philox10(p, i, tag, j, k0, k1);
    int kk;
    if (!done && ptrs_attempt(c, w.x, w.y, lnfact, kk)) {
      k = kk;
      done = true;
    }
    if (!done && ptrs_attempt(c, w.z, w.w, lnfact, kk)) {
      k = kk;
      done = true;
    }
    if (!wave_any(!done)) break;
  }
  if (!done) {
    failed = 1u;
    k = 0;
  }
  return (uint32_t)k;
}

// C1 table of a Poisson(l) count, 0 < l < 10: T_k = floor(2^32 F(k)) for k = 0, 1, ... while
// T_k < 2^32 - 1 (at most THR_STRIDE - 1 values), the cdf F built in FP64 by the pmf recurrence
// p_k = p_{k-1} l / k from p_0 = e^-l.  The first threshold that reaches 2^32 - 1 counts as 2^32
// and is not stored: its outcome K takes the last word too.  (The FP64 sum can stall just below
// 1, where floor(2^32 F) = 2^32 - 1; a table that ran on there would give word 2^32 - 1 the
// 63-star cap.)  T_k goes to t[k * stride] and, for k < 3, also to first[k].  Returns K, the
// number of thresholds written; K = 0 (l below about 2^-32) draws no star.
__device__ inline uint32_t inversion_table(double l, uint32_t *t, size_t stride, uint32_t first[3]) {
  double pk = exp(-l);
  double F = pk;
  uint32_t K = 0;
  for (int k = 0; k < THR_STRIDE - 1; ++k) {
    if (k > 0) {
      pk = pk * l / (double)k;
      F = F + pk;
    }
    const double tk = floor(F * 4294967296.0);
    if (tk >= 4294967295.0) break;
    const uint32_t tv = (uint32_t)tk;
    t[(size_t)k * stride] = tv;
    if (k < 3) first[k] = tv;
    K = (uint32_t)(k + 1);
  }
  return K;
}

// C2 constants of a Poisson(l) count (entries with l >= ALIAS_MAX, block totals with l >= 10):
// computed in FP64 and rounded to FP32.
__device__ inline PtrsConst ptrs_constants(double l) {
  const double slam = sqrt(l);
  const double bb = 0.931 + 2.53 * slam;
  const double aa = -0.059 + 0.02483 * bb;
  const double inv_alpha = 1.1239 + 1.1328 / (bb - 3.4);
  const double vr = 0.9277 - 3.6224 / (bb - 2.0);
  PtrsConst c;
  c.mu = (float)l;
  c.lnmu = (float)log(l);
  c.b = (float)bb;
  c.a = (float)aa;
  c.twoa = (float)(2.0 * aa);
  c.lninva = (float)log(inv_alpha);
  c.vr = (float)vr;
  c.pad = 0.0f;
  return c;
}

#pragma clang fp contract(on)

}  // namespace pcmd
