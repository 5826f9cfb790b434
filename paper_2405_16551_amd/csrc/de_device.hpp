// de_device.hpp -- device-side building blocks of the gfx950 DE/rand/1/bin
// kernels: counter-based random draws, the donor sampler of eq. 2, the
// crossover test of eq. 3, bound repair, ordered (f, index) keys and
// wave64 reductions.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  The
// 128-bit counter is (q, i, gen, tag << 24 | run) and the key is the 64-bit
// seed, so every draw is a pure function of its coordinates and no
// generator state lives in memory.  Integer-only conversions keep every
// index and every crossover decision independent of floating point.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace de {

enum : uint32_t {
  kTagInit = 1u,
  kTagIdx = 2u,
  kTagXover = 3u,
  kTagJde = 4u,
  kTagTrain = 5u,   // surrogate: minibatch rows
  kTagModel = 6u    // surrogate: initial weights
};

// Philox4x32-10 multipliers and Weyl key increments (Salmon et al., Sec. 4).
constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeylA = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeylB = 0xBB67AE85u;

struct Words4 {
  uint32_t w[4];
};

// Three-way XOR; on gfx950 one v_bitop3_b32 (truth table 0x96) instead of
// two v_xor_b32.
__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b,
                                                  uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
  return a ^ b ^ c;
#endif
}

// One S-box round: two 32x32->64 products (v_mad_u64_u32 on CDNA), the
// high halves mixed with the other two counter words and the round key.
__host__ __device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1,
                                             uint32_t& c2, uint32_t& c3,
                                             uint32_t k0, uint32_t k1) {
  const uint64_t pa = (uint64_t)kPhiloxMulA * c0;
  const uint64_t pb = (uint64_t)kPhiloxMulB * c2;
  const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
  const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
  c1 = (uint32_t)pb;
  c3 = (uint32_t)pa;
  c0 = n0;
  c2 = n2;
}

__host__ __device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1,
                                                uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c0, c1, c2, c3, k0 + (uint32_t)r * kPhiloxWeylA,
                 k1 + (uint32_t)r * kPhiloxWeylB);
  }
  Words4 out;
  out.w[0] = c0;
  out.w[1] = c1;
  out.w[2] = c2;
  out.w[3] = c3;
  return out;
}

// Draw block for (tag, run, gen, individual, group q).
__host__ __device__ __forceinline__ Words4 draw_block(uint32_t tag, uint32_t run,
                                             uint32_t gen, uint32_t indiv,
                                             uint32_t q, uint32_t key_lo,
                                             uint32_t key_hi) {
  return philox4x32_10(q, indiv, gen, (tag << 24) | run, key_lo, key_hi);
}

// Uniform integer in [0, n) from one 32-bit word: floor(w * n / 2^32).
__host__ __device__ __forceinline__ int uniform_below(uint32_t w, uint32_t n) {
  return (int)(((uint64_t)w * n) >> 32);
}

// Donor triple and j_rand of eq. 2 / eq. 3 for target i.  a, b, c are
// uniform over NP-1, NP-2, NP-3 values; each is lifted over the indices
// already taken (target first, then earlier donors), in ascending order, so
// (a, b, c) maps one-to-one onto ordered triples of distinct indices != i.
struct Donors {
  int r1, r2, r3, jrand;
};

// ctr_i is the counter's individual field (i itself, or i | c << 24 for
// candidate c of the surrogate-assisted step); i is the target to avoid.
__host__ __device__ __forceinline__ Donors pick_donors_ctr(
    uint32_t run, uint32_t gen, uint32_t ctr_i, int i, int NP, int D,
    uint32_t key_lo, uint32_t key_hi) {
  const Words4 w = draw_block(kTagIdx, run, gen, ctr_i, 0u, key_lo, key_hi);
  Donors d;
  const int a = uniform_below(w.w[0], (uint32_t)(NP - 1));
  d.r1 = a + (a >= i ? 1 : 0);
  const int lo2 = min(i, d.r1), hi2 = max(i, d.r1);
  int b = uniform_below(w.w[1], (uint32_t)(NP - 2));
  b += (b >= lo2 ? 1 : 0);
  b += (b >= hi2 ? 1 : 0);
  d.r2 = b;
  // ascending order of {i, r1, r2}
  int s0 = lo2, s1 = hi2, s2 = b;
  if (s2 < s1) { const int t = s1; s1 = s2; s2 = t; }
  if (s1 < s0) { const int t = s0; s0 = s1; s1 = t; }
  int c = uniform_below(w.w[2], (uint32_t)(NP - 3));
  c += (c >= s0 ? 1 : 0);
  c += (c >= s1 ? 1 : 0);
  c += (c >= s2 ? 1 : 0);
  d.r3 = c;
  d.jrand = uniform_below(w.w[3], (uint32_t)D);
  return d;
}

__host__ __device__ __forceinline__ Donors pick_donors(uint32_t run, uint32_t gen,
                                              int i, int NP, int D,
                                              uint32_t key_lo,
                                              uint32_t key_hi) {
  return pick_donors_ctr(run, gen, (uint32_t)i, i, NP, D, key_lo, key_hi);
}

// Crossover test of eq. 3 for coordinate j = 4q + b: rand_j = (w >> 8) 2^-24
// and rand_j <= CR  <=>  (w >> 8) <= floor(CR 2^24) = cr_threshold
// <=>  w <= 256 cr_threshold + 255 (all words when cr_threshold >= 2^24 - 1),
// one comparison of the whole word.  The limit depends on the threshold
// only, so loops compute it once.
__host__ __device__ __forceinline__ uint32_t xover_word_limit(
    uint32_t cr_threshold) {
  return cr_threshold >= 0xFFFFFFu ? 0xFFFFFFFFu
                                   : (cr_threshold << 8) | 0xFFu;
}

__host__ __device__ __forceinline__ bool take_mutant(uint32_t word, int j, int jrand,
                                            uint32_t cr_threshold) {
  return (j == jrand) | (word <= xover_word_limit(cr_threshold));
}

// Mutant coordinate of eq. 2 with clamping to the box; NaN passes through.
__host__ __device__ __forceinline__ float mutant_coord(float x1, float x2, float x3,
                                              float F, float lo, float hi) {
  float v = fmaf(F, x2 - x3, x1);
  v = v < lo ? lo : v;
  v = v > hi ? hi : v;
  return v;
}

// jDE control values of individual i for this generation (self-adaptation
// of Brest et al., 2006): one Philox block (tag 4, group 0) gives u1..u4 on
// the 2^-24 lattice; F' = F_lo + u1 F_span (one fused rounding) if
// u2 < tau_F, else the stored F; CR' = u3 if u4 < tau_CR, else the stored
// CR.  tau thresholds are floor(tau 2^24), compared in integers.
struct Control {
  float F, CR;
};

__host__ __device__ __forceinline__ Control jde_control(
    uint32_t run, uint32_t gen, int i, uint32_t key_lo, uint32_t key_hi,
    float F_lo, float F_span, uint32_t tau_F, uint32_t tau_CR, Control cur) {
  const Words4 w = draw_block(kTagJde, run, gen, (uint32_t)i, 0u, key_lo,
                              key_hi);
  Control c = cur;
  if ((w.w[1] >> 8) < tau_F)
    c.F = fmaf((float)(w.w[0] >> 8) * 0x1.0p-24f, F_span, F_lo);
  if ((w.w[3] >> 8) < tau_CR) c.CR = (float)(w.w[2] >> 8) * 0x1.0p-24f;
  return c;
}

// floor(CR 2^24) for a float CR in [0, 1] (the scaling is exact).
__host__ __device__ __forceinline__ uint32_t cr_threshold_of(float CR) {
  return (uint32_t)(CR * 16777216.0f);
}

// Totally ordered 64-bit key: order-preserving image of the float in the high
// half (NaN sorts above +inf), individual index in the low half, so
// atomicMin yields the lowest value with ties to the lowest index.
__host__ __device__ __forceinline__ unsigned long long fit_key(float f, int idx) {
  const uint32_t b = __builtin_bit_cast(uint32_t, f);
  const uint32_t ord = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((unsigned long long)ord << 32) | (uint32_t)idx;
}

// sin^2(t), t in FP32.  t = k (pi/2) + r with |r| <= pi/4: k = rint(t 2/pi),
// r by Cody-Waite reduction with pi/2 split into three FP32 parts (each
// product k * part folded in with one FMA).  sin^2(t) = sin^2(r) for even k
// and 1 - sin^2(r) for odd k.  sin^2(r) from its Taylor series
// sum_{n>=1} (-1)^(n+1) 2^(2n-1) r^(2n) / (2n)!, six terms: the first
// omitted term is below 4e-9 on |r| <= pi/4, under half an FP32 ulp of 0.5.
__host__ __device__ __forceinline__ float sin_squared(float t) {
  constexpr float kTwoOverPi = 0x1.45f306p-1f;
  constexpr float kHalfPiA = 0x1.921fb6p+0f;
  constexpr float kHalfPiB = -0x1.777a5cp-25f;
  constexpr float kHalfPiC = -0x1.ee59dap-50f;
  const float k = rintf(t * kTwoOverPi);
  float r = fmaf(-k, kHalfPiA, t);
  r = fmaf(-k, kHalfPiB, r);
  r = fmaf(-k, kHalfPiC, r);
  const float s = r * r;
  float p = -2.0f / 467775.0f;
  p = fmaf(p, s, 2.0f / 14175.0f);
  p = fmaf(p, s, -1.0f / 315.0f);
  p = fmaf(p, s, 2.0f / 45.0f);
  p = fmaf(p, s, -1.0f / 3.0f);
  p = fmaf(p, s, 1.0f);
  p *= s;
  return ((int)k & 1) ? 1.0f - p : p;
}

// Sum over aligned groups of `width` lanes (power of two <= 64) by
// butterfly exchange; every lane of the group ends with the same total, and
// the order of additions is fixed.
template <int width>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int m = width / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Block index remapping so that consecutive logical blocks land on the same
// XCD (gfx950 dispatches block b to XCD b mod 8): logical block ranges, and
// the donor rows they share, then stay in one XCD's L2.  Bijective for any n.
__host__ __device__ __forceinline__ int xcd_logical_block(int b, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd;
  const int xcd = b % kXcd, k = b / kXcd;
  return xcd * q + min(xcd, r) + k;
}

}  // namespace de
