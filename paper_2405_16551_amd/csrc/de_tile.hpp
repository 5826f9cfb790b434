// de_tile.hpp -- device code shared by the per-problem and the batched
// generation kernels: vector helpers, the per-run statistics update and the
// rotated-objective tile (build trials into LDS, Z = Y R^T on MFMA with the
// objective fused, select and write).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "de_device.hpp"
#include "de_internal.h"

namespace de {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr unsigned long long kNoHit = ~0ull;

__device__ __forceinline__ float4 ld4(const float* p) {
  return *reinterpret_cast<const float4*>(p);
}
__device__ __forceinline__ void st4(float* p, float4 v) {
  *reinterpret_cast<float4*>(p) = v;
}
__device__ __forceinline__ float get(const float4& v, int b) {
  return b == 0 ? v.x : b == 1 ? v.y : b == 2 ? v.z : v.w;
}
__device__ __forceinline__ void set(float4& v, int b, float s) {
  if (b == 0) v.x = s; else if (b == 1) v.y = s; else if (b == 2) v.z = s;
  else v.w = s;
}

// Statistics after an accepted trial with value f of individual i in run r,
// which produced generation gen+1.
__device__ __forceinline__ void record_accept_at(const GenArgs& a, int run,
                                                 int i, float f,
                                                 uint32_t gen) {
  atomicAdd(&a.accepted[run], 1ull);
  atomicMin(&a.best_key[run], fit_key(f, i));
  if (f <= a.target) {
    const unsigned long long old =
        atomicMin(&a.hit_gen[run], (unsigned long long)gen + 1ull);
    if (old == kNoHit) atomicAdd(a.done, 1u);
  }
}

__device__ __forceinline__ void record_accept(const GenArgs& a, int run, int i,
                                              float f) {
  record_accept_at(a, run, i, f, a.gen);
}

// ---------------------------------------------------------------------------
// Rotated objective.  Tile of BM trial rows per workgroup of NT threads.
//   phase 1: donors of every row, then per row all target/donor loads in
//            flight before the crossover draws; trial rows -> LDS A tile as
//            y = u - o in the GEMM precision, crossover decisions -> bit
//            planes; padding rows and columns are zero.
//   phase 2: Z = Y R^T in 32x32 MFMA blocks, wave tile BM rows x one
//            32-column block per pass (two for FP32 tiles wider than 256),
//            R fragments prefetched four K-steps ahead from L2; the
//            objective z^2 + sin^2(3z) is summed per row in registers.
//   phase 3: row totals -> selection -> next generation rows (a rejected row
//            is rewritten only if the other buffer holds a stale copy),
//            statistics.
// Operand precision of the rotation product; kOneBlock: each wave owns one
// 32-column block per pass (BF16 always; FP32 at padded widths up to 256,
// where two blocks per wave would leave most waves without a block), else
// two.
struct PrecBF16 {
  using T = __bf16;
  static constexpr int kPad = 8;  // LDS row padding, elements
  static constexpr bool kOneBlock = true;
};
struct PrecF32 {
  using T = float;
  static constexpr int kPad = 4;
  static constexpr bool kOneBlock = false;
};
struct PrecF32Narrow : PrecF32 {
  static constexpr bool kOneBlock = true;
};
constexpr int kF32NarrowMaxDpad = 256;

// Slots of the per-row objective sums (see rot_tile).
constexpr int kRotSlots = 16;

template <class P, int BM, bool JDE = false>
__host__ __device__ constexpr size_t rot_lds_bytes(int dpad) {
  const int tq = (dpad / 4 + 63) / 64;
  return (size_t)BM * (dpad + P::kPad) * sizeof(typename P::T)  // A tile
         + (size_t)BM * tq * 4 * sizeof(unsigned long long)     // planes
         + (size_t)BM * 4 * sizeof(int)                         // donors
         + (size_t)kRotSlots * BM * sizeof(float)               // slot sums
         + (JDE ? (size_t)BM * sizeof(Control) : 0);            // F', CR'
}

// Position of coordinate k inside an LDS row.  BF16: natural order.  FP32:
// within each group of 8, k = 2s + h is stored at 4h + s so that one lane's
// four K-steps of the 32x32x2 MFMA are one 16-byte read.
template <class P>
__device__ __forceinline__ int lds_col(int k) {
  if constexpr (sizeof(typename P::T) == 2) {
    return k;
  } else {
    const int g = k & ~7, r = k & 7;
    return g + (r & 1) * 4 + (r >> 1);
  }
}

// One coordinate of the rotated oscillating objective: z^2 + sin^2(3z).
// FP32 product: sin^2 from the reduction and series of sin_squared.
// BF16 product (z already carries BF16 operand rounding, relative error
// ~2^-8): the hardware sine, which takes its argument in turns; 3z / (2 pi)
// is reduced to [-1/2, 1/2] turns first (exact), the remaining error is the
// FP32 rounding of 3z / (2 pi), about 2^-24 |3z| radians.
template <bool kFastSin>
__device__ __forceinline__ float osc_term(float z) {
  if constexpr (kFastSin) {
    constexpr float kTurnsPer3z = 0x1.e8ec8ap-2f;  // 3 / (2 pi)
    const float turns = z * kTurnsPer3z;
    const float s = __builtin_amdgcn_sinf(turns - rintf(turns));
    return fmaf(z, z, s * s);
  } else {
    return fmaf(z, z, sin_squared(3.0f * z));
  }
}

template <bool kFastSin>
__device__ __forceinline__ void osc_accumulate(floatx16& part,
                                               const floatx16& c) {
#pragma unroll
  for (int r = 0; r < 16; ++r) part[r] += osc_term<kFastSin>(c[r]);
}

// 256-coordinate chunks per producer step (rows per step: 8 / this).  One
// chunk of eight rows measured fastest at D = 1000 (BF16 and FP32 tiles).
constexpr int kProducerChunks = 1;
// Rows per producer step of BF16 tiles (128 registers per lane).
constexpr int kBf16Rows = 4;
// Threads of the BF16 rotated tile.  Each wave owns one column block per
// pass and four producer rows per step, within 128 registers, so four
// waves fit per SIMD.  The tile has 16 waves (measured faster at D = 1000
// than 8 waves with twice the registers each), or 8 when two tiles fit in
// a CU's LDS (padded width up to 512) and there are more tiles than CUs:
// then each CU holds two and one tile's loads overlap the other's MFMAs.
// The result does not depend on the choice (row sums add column blocks in
// a fixed order).
constexpr int kRotBf16Threads = 1024;
constexpr int kRotBf16ThreadsNarrow = 512;
constexpr int kRotBf16NarrowMaxDpad = 512;
__host__ __device__ constexpr bool rot_bf16_narrow(int dpad, long long tiles,
                                                   int cus) {
  return dpad <= kRotBf16NarrowMaxDpad && tiles > cus;
}

// R fragments of four consecutive K-steps of one column block.
struct BFrags {
  bf16x8 b0[4];
};

__device__ __forceinline__ void load_bfrags(BFrags& f, const bf16x8* rb0,
                                            int kb) {
#pragma unroll
  for (int u = 0; u < 4; ++u) f.b0[u] = rb0[(size_t)(kb + u) * 64];
}

// Scheduling pattern for one K-step: per row block one MFMA and its next A
// read (LDS), then the step's R load (L2), so the matrix unit keeps busy
// while the reads go out instead of waiting behind one burst.
template <int MB>
__device__ __forceinline__ void interleave_step() {
  __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
  __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
  if constexpr (MB == 2) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read
  __builtin_amdgcn_sched_barrier(0);
}

// Four FP32 K-steps (8 coordinates) of the wave tile, rows 0-31.
__device__ __forceinline__ void f32_step(const float* ar, int k8, float4 b0,
                                         float4 b1, floatx16& c00,
                                         floatx16& c01) {
  const float4 av = *reinterpret_cast<const float4*>(ar + k8 * 8);
  c00 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, b0.x, c00, 0, 0, 0);
  c01 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, b1.x, c01, 0, 0, 0);
  c00 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, b0.y, c00, 0, 0, 0);
  c01 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, b1.y, c01, 0, 0, 0);
  c00 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, b0.z, c00, 0, 0, 0);
  c01 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, b1.z, c01, 0, 0, 0);
  c00 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, b0.w, c00, 0, 0, 0);
  c01 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, b1.w, c01, 0, 0, 0);
}

// Two consecutive FP32 four-step groups (k8, k8 + 1) of one column block
// into two accumulators, interleaved.
__device__ __forceinline__ void f32_step2(const float* ar, int k8, float4 b0,
                                          float4 b1, floatx16& ce,
                                          floatx16& co) {
  const float4 a0 = *reinterpret_cast<const float4*>(ar + k8 * 8);
  const float4 a1 = *reinterpret_cast<const float4*>(ar + (k8 + 1) * 8);
  ce = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.x, b0.x, ce, 0, 0, 0);
  co = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.x, b1.x, co, 0, 0, 0);
  ce = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.y, b0.y, ce, 0, 0, 0);
  co = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.y, b1.y, co, 0, 0, 0);
  ce = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.z, b0.z, ce, 0, 0, 0);
  co = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.z, b1.z, co, 0, 0, 0);
  ce = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.w, b0.w, ce, 0, 0, 0);
  co = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.w, b1.w, co, 0, 0, 0);
}

// Widest padded row of the paired-row form: 32 quads, so that one row's
// quads fill half a wave and its crossover bits are one 32-bit half of a
// ballot.  Launchers refuse PAIR beyond it.
constexpr int kPairMaxDpad = 128;

// One tile: rows row0 .. row0 + nvalid - 1 of run `run` (EVAL: of the
// flattened row range).  Ends with every LDS access of the tile complete
// only for the calling thread: a caller that runs another tile in the same
// workgroup synchronises first.  PAIR (padded widths up to kPairMaxDpad
// only): the trials are built two rows per wave instruction.
template <class P, int BM, int NT, bool EVAL, bool JDE = false,
          bool PAIR = false>
__device__ __forceinline__ void rot_tile(const GenArgs& a, int run, int row0,
                                         int nvalid) {
  using T = typename P::T;
  constexpr int MB = BM / 32;
  constexpr int kRotThreads = NT;
  constexpr int kRotWaves = NT / 64;
  // BF16 tiles: one column block per wave and pass, four producer rows per
  // step (128 registers); FP32 tiles: one or two column blocks (P),
  // eight rows
  constexpr int NBW = P::kOneBlock ? 1 : 2;
  static_assert(MB == 1 || (MB == 2 && sizeof(T) == 2), "tile shape");
  extern __shared__ __align__(16) char smem[];
  const int dpad = a.dpad;
  const int stride = dpad + P::kPad;
  const int tq = (dpad / 4 + 63) / 64;
  T* At = reinterpret_cast<T*>(smem);
  unsigned long long* planes = reinterpret_cast<unsigned long long*>(
      smem + (size_t)BM * stride * sizeof(T));
  int* donors = reinterpret_cast<int*>(planes + (size_t)BM * tq * 4);
  float* fpart = reinterpret_cast<float*>(donors + BM * 4);
  // jDE: the F' and CR' of every row of the tile
  Control* ctl = reinterpret_cast<Control*>(fpart + kRotSlots * BM);

  const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
  const uint32_t rng_run = a.run_base + (uint32_t)run;
  const float* base = a.pop_cur + (EVAL ? 0 : (size_t)run * a.NP * a.ldx);

  // ---- phase 1: build the A tile
  if (!EVAL) {
    for (int rl = (int)threadIdx.x; rl < nvalid; rl += kRotThreads) {
      const Donors d = pick_donors(rng_run, a.gen, row0 + rl, a.NP, a.D,
                                   a.key_lo, a.key_hi);
      donors[rl * 4 + 0] = d.r1;
      donors[rl * 4 + 1] = d.r2;
      donors[rl * 4 + 2] = d.r3;
      donors[rl * 4 + 3] = d.jrand;
      if constexpr (JDE) {
        const float2 c = a.jp_cur[(size_t)run * a.NP + row0 + rl];
        ctl[rl] = jde_control(rng_run, a.gen, row0 + rl, a.key_lo, a.key_hi,
                              a.jF_lo, a.jF_span, a.jtau_F, a.jtau_CR,
                              Control{c.x, c.y});
      }
    }
    __syncthreads();
  }
  // Rows rl = wave + kRotWaves * k of this wave; each row is cut into groups
  // of four 256-coordinate chunks.  Items (row, group) are processed in
  // order with two register sets, so the loads of item s + 1 are in flight
  // while item s is drawn, mutated and stored.
  for (int rl = nvalid + (((wave - nvalid) % kRotWaves) + kRotWaves) %
                             kRotWaves;
       rl < BM; rl += kRotWaves) {
    T* arow = At + (size_t)rl * stride;
    for (int k = lane; k < dpad; k += 64) arow[k] = (T)0.0f;
  }
  if constexpr (PAIR) {
    // Padded widths up to 128 (at most 32 quads per row): lanes 32 h + q
    // build quad q of the h-th row of a pair of the wave's rows, so every
    // lane has a quad (one row per instruction would leave more than half
    // of them idle).  Same loads, draws, arithmetic and stores as below;
    // each row's crossover bits are its half of the ballot.
    static_assert(!EVAL, "paired form: generation step");
    constexpr int RBP = 4;  // pairs per step
    const int hl = lane / 32, ql = lane % 32;
    const int nrow_w = wave < nvalid ? (nvalid - 1 - wave) / kRotWaves + 1 : 0;
    const int dlast = ((a.D + 3) / 4 - 1) * 4;
    const int j0 = 4 * ql, jl = min(j0, dlast);
    const float4 ov = ld4(a.o + jl);
    for (int k = 0; k < nrow_w; k += 2 * RBP) {
      float4 xv[RBP], v1[RBP], v2[RBP], v3[RBP];
#pragma unroll
      for (int p = 0; p < RBP; ++p) {
        const int rl = wave + kRotWaves * min(k + 2 * p + hl, nrow_w - 1);
        xv[p] = ld4(base + (size_t)(row0 + rl) * a.ldx + jl);
        if (!EVAL) {
          v1[p] = ld4(base + (size_t)donors[rl * 4 + 0] * a.ldx + jl);
          v2[p] = ld4(base + (size_t)donors[rl * 4 + 1] * a.ldx + jl);
          v3[p] = ld4(base + (size_t)donors[rl * 4 + 2] * a.ldx + jl);
        }
      }
#pragma unroll
      for (int p = 0; p < RBP; ++p) {
        if (k + 2 * p >= nrow_w) break;
        const int kk = k + 2 * p + hl;
        const bool live = kk < nrow_w;  // the pair's second row may not exist
        const int rl = wave + kRotWaves * min(kk, nrow_w - 1);
        const int i = row0 + rl;
        uint32_t bits = 0;
        float4 uu = xv[p];
        if (!EVAL) {
          const int jrand = donors[rl * 4 + 3];
          float Fr = a.F;
          uint32_t crt = a.cr_threshold;
          if constexpr (JDE) {  // the row's own F', CR'
            const Control c = ctl[rl];
            Fr = c.F;
            crt = cr_threshold_of(c.CR);
          }
          const Words4 w = draw_block(kTagXover, rng_run, a.gen, (uint32_t)i,
                                      (uint32_t)ql, a.key_lo, a.key_hi);
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const bool tk = (j0 + b < a.D) &&
                            take_mutant(w.w[b], j0 + b, jrand, crt);
            const float mv = mutant_coord(get(v1[p], b), get(v2[p], b),
                                          get(v3[p], b), Fr, a.lo, a.hi);
            set(uu, b, tk ? mv : get(xv[p], b));
            bits |= (tk ? 1u : 0u) << b;
          }
        }
        float4 y;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          set(y, b, (j0 + b < a.D) ? get(uu, b) - get(ov, b) : 0.f);
        T* arow = At + (size_t)rl * stride;
        if (live && j0 < dpad) {
          if constexpr (sizeof(T) == 2) {
            bf16x4 yb;
            yb[0] = (__bf16)y.x;
            yb[1] = (__bf16)y.y;
            yb[2] = (__bf16)y.z;
            yb[3] = (__bf16)y.w;
            *reinterpret_cast<bf16x4*>(arow + j0) = yb;
          } else {
#pragma unroll
            for (int b = 0; b < 4; ++b) arow[lds_col<P>(j0 + b)] = get(y, b);
          }
        }
        if (!EVAL) {
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const unsigned long long m = __ballot((bits >> b) & 1u);
            if (ql == 0 && live)
              planes[(size_t)rl * tq * 4 + b] = hl ? (m >> 32) : (m & 0xFFFFFFFFull);
          }
        }
      }
    }
  } else
  {
    // Chunk-major: for each group of CG 256-coordinate chunks, the wave's
    // rows rl = wave + kRotWaves * k go RB at a time (CG * RB = 8 chunk
    // rows in flight): the target and donor chunks of the RB rows are
    // requested together, then drawn, mutated and stored.  All workgroups
    // walk the chunks in the same order, so an XCD's donor reads of one
    // step stay within one chunk of its runs' rows (a working set its L2
    // holds).  Loads past the end of a row go to its last chunk and rows
    // past the wave's last go to its last row (values unused), so no load
    // sits behind a per-lane branch.
    constexpr int CG = kProducerChunks;
    constexpr int RB = (sizeof(T) == 2 ? kBf16Rows : 8) / CG;
    const int nrow_w = wave < nvalid ? (nvalid - 1 - wave) / kRotWaves + 1 : 0;
    const int dlast = ((a.D + 3) / 4 - 1) * 4;
    for (int t0 = 0; t0 < tq; t0 += CG) {
      float4 ov[CG];
#pragma unroll
      for (int u = 0; u < CG; ++u)
        ov[u] = ld4(a.o + min(4 * (lane + 64 * (t0 + u)), dlast));
      for (int k = 0; k < nrow_w; k += RB) {
        float4 xv[RB][CG], v1[RB][CG], v2[RB][CG], v3[RB][CG];
#pragma unroll
        for (int h = 0; h < RB; ++h) {
          // row and donor indices are wave-uniform: scalar row pointers
          const int rl = __builtin_amdgcn_readfirstlane(
              wave + kRotWaves * min(k + h, nrow_w - 1));
          const float* xrow = base + (size_t)(row0 + rl) * a.ldx;
          const float *x1 = xrow, *x2 = xrow, *x3 = xrow;
          if (!EVAL) {
            x1 = base + (size_t)__builtin_amdgcn_readfirstlane(
                            donors[rl * 4 + 0]) * a.ldx;
            x2 = base + (size_t)__builtin_amdgcn_readfirstlane(
                            donors[rl * 4 + 1]) * a.ldx;
            x3 = base + (size_t)__builtin_amdgcn_readfirstlane(
                            donors[rl * 4 + 2]) * a.ldx;
          }
#pragma unroll
          for (int u = 0; u < CG; ++u) {
            const int jl = min(4 * (lane + 64 * (t0 + u)), dlast);
            xv[h][u] = ld4(xrow + jl);
            if (!EVAL) {
              v1[h][u] = ld4(x1 + jl);
              v2[h][u] = ld4(x2 + jl);
              v3[h][u] = ld4(x3 + jl);
            }
          }
        }
        // every gather of the step is issued before any of it is used:
        // keeps the compiler from sinking a row's loads into the guarded
        // code that consumes them
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int h = 0; h < RB; ++h) {
          if (k + h >= nrow_w) break;
          const int rl = wave + kRotWaves * (k + h);
          const int i = row0 + rl;
          const int jrand = EVAL ? 0 : donors[rl * 4 + 3];
          float Fr = a.F;
          uint32_t crt = a.cr_threshold;
          if constexpr (JDE && !EVAL) {
            const Control c = ctl[rl];
            Fr = c.F;
            crt = cr_threshold_of(c.CR);
          }
          T* arow = At + (size_t)rl * stride;
#pragma unroll
          for (int u = 0; u < CG; ++u) {
            const int t = t0 + u;
            if (t >= tq) break;
            const int q = lane + 64 * t, j0 = 4 * q;
            bool tk[4] = {false, false, false, false};
            float4 uu = xv[h][u];
            if (!EVAL) {
              const Words4 w = draw_block(kTagXover, rng_run, a.gen,
                                          (uint32_t)i, (uint32_t)q, a.key_lo,
                                          a.key_hi);
#pragma unroll
              for (int b = 0; b < 4; ++b) {
                // bitwise &: both tests are lane masks, no branch
                tk[b] = (j0 + b < a.D) &
                        take_mutant(w.w[b], j0 + b, jrand, crt);
                const float mv =
                    mutant_coord(get(v1[h][u], b), get(v2[h][u], b),
                                 get(v3[h][u], b), Fr, a.lo, a.hi);
                set(uu, b, tk[b] ? mv : get(xv[h][u], b));
              }
            }
            float4 y;
#pragma unroll
            for (int b = 0; b < 4; ++b)
              set(y, b, (j0 + b < a.D) ? get(uu, b) - get(ov[u], b) : 0.f);
            if (j0 < dpad) {
              if constexpr (sizeof(T) == 2) {
                bf16x4 yb;
                yb[0] = (__bf16)y.x;
                yb[1] = (__bf16)y.y;
                yb[2] = (__bf16)y.z;
                yb[3] = (__bf16)y.w;
                *reinterpret_cast<bf16x4*>(arow + j0) = yb;
              } else {
#pragma unroll
                for (int b = 0; b < 4; ++b)
                  arow[lds_col<P>(j0 + b)] = get(y, b);
              }
            }
            if (!EVAL) {
              // the four crossover planes of the chunk are the ballots of
              // the decisions (the compare masks themselves), stored by
              // lane 0 as two 16-byte writes
              const unsigned long long m0 = __ballot(tk[0]);
              const unsigned long long m1 = __ballot(tk[1]);
              const unsigned long long m2 = __ballot(tk[2]);
              const unsigned long long m3 = __ballot(tk[3]);
              if (lane == 0) {
                ulonglong2* pp = reinterpret_cast<ulonglong2*>(
                    planes + ((size_t)rl * tq + t) * 4);
                pp[0] = make_ulonglong2(m0, m1);
                pp[1] = make_ulonglong2(m2, m3);
              }
            }
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- phase 2: Z = Y R^T with the objective fused into the epilogue
  // Accumulators c{m}{n}: 32x32 block (row block m, column block nb0 + n),
  // named values rather than arrays so that every index is static.
  // Wave w of every workgroup streams the same R fragments at about the same
  // time, so concurrent requests from the CUs of an XCD share L2 lines.
  const int nblk = dpad / 32;
  // Row sums of the objective go to kRotSlots slots: slot s adds column
  // blocks s, s + 16, s + 32, ... in increasing order, so the result does
  // not depend on how blocks are dealt to waves (the number of threads).
  // A wave's blocks fall into SPW slots, its pass p into sacc[p % SPW].
  constexpr int SPW = kRotSlots / (kRotWaves * NBW) > 1
                          ? kRotSlots / (kRotWaves * NBW)
                          : 1;
  static_assert(kRotSlots % (kRotWaves * NBW) == 0 ||
                    (kRotWaves * NBW) % kRotSlots == 0,
                "slots and waves");
  float sacc[SPW];
#pragma unroll
  for (int q = 0; q < SPW; ++q) sacc[q] = 0.f;
  int pass = 0;
  for (int nb0 = wave * NBW; nb0 < nblk;
       nb0 += kRotWaves * NBW, ++pass) {
    floatx16 c00 = {}, c01 = {}, c10 = {};
    if constexpr (sizeof(T) == 2) {
      // R as [nblk][dpad/16][64 lanes][8]: one 16-byte load per lane per
      // block and K-step; dpad / 16 is a multiple of 4.
      const bf16x8* rop = reinterpret_cast<const bf16x8*>(a.rop);
      const int kbn = dpad / 16;
      const bf16x8* rb0 = rop + ((size_t)nb0 * kbn) * 64 + lane;
      const T* ar = At + (size_t)(lane % 32) * stride + 8 * (lane / 32);
      // Software pipeline at K-step granularity: the A fragments of step
      // k + 1 are read from LDS while step k's MFMAs run (two slots), and
      // the R fragments of the next four-step group are loaded from L2 one
      // per step into the other of two register sets.  Each step's reads
      // are interleaved with its MFMAs (one per row block).  dpad / 16 is a
      // multiple of 8.
      const T* ar1 = ar + (size_t)32 * stride;
      bf16x8 a0s[2], a1s[2];
      BFrags fa, fb;
      a0s[0] = *reinterpret_cast<const bf16x8*>(ar);
      if constexpr (MB == 2) a1s[0] = *reinterpret_cast<const bf16x8*>(ar1);
      load_bfrags(fa, rb0, 0);
      for (int kb = 0; kb < kbn; kb += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = kb + u;
          const int cur = u & 1, nxt = cur ^ 1;
          if (u < 7 || k + 1 < kbn) {
            a0s[nxt] = *reinterpret_cast<const bf16x8*>(ar + (k + 1) * 16);
            if constexpr (MB == 2)
              a1s[nxt] = *reinterpret_cast<const bf16x8*>(ar1 + (k + 1) * 16);
          }
          if (u < 4) {
            fb.b0[u] = rb0[(size_t)(kb + 4 + u) * 64];
          } else if (kb + 8 < kbn) {
            fa.b0[u - 4] = rb0[(size_t)(kb + 8 + u - 4) * 64];
          }
          const bf16x8 b0 = u < 4 ? fa.b0[u & 3] : fb.b0[u & 3];
          c00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0s[cur], b0, c00, 0, 0,
                                                        0);
          if constexpr (MB == 2) {
            c10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1s[cur], b0, c10, 0,
                                                          0, 0);
          }
          interleave_step<MB>();
        }
      }
    } else {
      // R as [nblk][dpad/8][64 lanes][4]: one float4 = four K-steps;
      // dpad / 8 is a multiple of 2.
      const float4* rop = reinterpret_cast<const float4*>(a.rop);
      const int k8n = dpad / 8;
      const float4* rb0 = rop + ((size_t)nb0 * k8n) * 64 + lane;
      const float* ar = reinterpret_cast<const float*>(At) +
                        (size_t)(lane % 32) * stride + 4 * (lane / 32);
      if constexpr (NBW == 2) {
        const float4* rb1 = rb0 + (size_t)k8n * 64;
        float4 p00 = rb0[0], p01 = rb0[64], p10 = rb1[0], p11 = rb1[64];
        for (int k8 = 0; k8 < k8n; k8 += 2) {
          const float4 q00 = p00, q01 = p01, q10 = p10, q11 = p11;
          if (k8 + 2 < k8n) {
            const size_t nx = (size_t)(k8 + 2) * 64;
            p00 = rb0[nx];
            p01 = rb0[nx + 64];
            p10 = rb1[nx];
            p11 = rb1[nx + 64];
          }
          f32_step(ar, k8 + 0, q00, q10, c00, c01);
          f32_step(ar, k8 + 1, q01, q11, c00, c01);
        }
      } else {
        // one block: even and odd four-step groups accumulate apart (two
        // independent MFMA chains), then add
        float4 p0 = rb0[0], p1 = rb0[64];
        for (int k8 = 0; k8 < k8n; k8 += 2) {
          const float4 q0 = p0, q1 = p1;
          if (k8 + 2 < k8n) {
            const size_t nx = (size_t)(k8 + 2) * 64;
            p0 = rb0[nx];
            p1 = rb0[nx + 64];
          }
          f32_step2(ar, k8, q0, q1, c00, c01);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) c00[r] += c01[r];
      }
    }
    // The objective of each 32-column block, summed per row and written to
    // the block's LDS slot; rows then add the slots in block order, so the
    // result does not depend on how blocks are dealt to waves (the number
    // of threads).  32x32 accumulator layout: register r of lane l holds
    // row 8 (r / 4) + 4 (l / 32) + r % 4 and column l % 32 of the block.
    // Each lane has 32 values (BF16: rows of row blocks 0 and 1; FP32: one
    // row block, column blocks nb0 and nb0 + 1); a reduce-scatter butterfly
    // over the 32 lanes of each half-wave leaves lane l with the total of
    // value l % 32 (31 exchanges instead of 5 per value).
    constexpr bool kFastSin = sizeof(T) == 2;
    floatx16& lo = c00;
    floatx16& hi = MB == 2 ? c10 : c01;
    // FP32 one-block tiles: values 16-31 (a second block) are empty
    constexpr bool kHi = MB == 2 || NBW == 2;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      lo[r] = osc_term<kFastSin>(lo[r]);
      hi[r] = kHi ? osc_term<kFastSin>(hi[r]) : 0.f;
    }
    {  // first exchange: values 0-15 keep lo or hi, the other half goes over
      const bool upper = (lane & 16) != 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const float send = upper ? lo[k] : hi[k];
        const float keep = upper ? hi[k] : lo[k];
        lo[k] = keep + __shfl_xor(send, 16, 64);
      }
    }
#pragma unroll
    for (int m = 8, n = 16; m >= 1; m >>= 1, n >>= 1) {
      const bool upper = (lane & m) != 0;
#pragma unroll
      for (int k = 0; k < n / 2; ++k) {
        const float send = upper ? lo[k] : lo[k + n / 2];
        const float keep = upper ? lo[k + n / 2] : lo[k];
        lo[k] = keep + __shfl_xor(send, m, 64);
      }
    }
#pragma unroll
    for (int q = 0; q < SPW; ++q)
      if (pass % SPW == q) sacc[q] += lo[0];
  }
  // lane l holds value l % 32: BF16 row (l % 32 / 16) * 32 + rin of the
  // wave's blocks; FP32 row rin of block nb0 + (l % 32) / 16 (one-block
  // tiles: block nb0 in lanes with l % 32 < 16)
  {
    const int idx = lane % 32, hb = idx / 16, r = idx % 16;
    const int rin = 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
      const int b0 = wave * NBW + q * kRotWaves * NBW;  // first block of q
      if constexpr (MB == 2) {
        if (b0 < kRotSlots) fpart[(size_t)b0 * BM + hb * 32 + rin] = sacc[q];
      } else if constexpr (NBW == 1) {
        if (hb == 0 && b0 < kRotSlots) fpart[(size_t)b0 * BM + rin] = sacc[q];
      } else {
        if (b0 + hb < kRotSlots)
          fpart[(size_t)(b0 + hb) * BM + rin] = sacc[q];
      }
    }
  }
  __syncthreads();

  // ---- phase 3: selection and the next generation
  if constexpr (PAIR) {
    // two rows per wave instruction as in the build: lanes 32 h + q handle
    // quad q of the h-th row of a pair; lanes 0 and 32 each write their
    // row's value, flag and statistics
    const int hl = lane / 32, ql = lane % 32;
    const int nrow_w = wave < nvalid ? (nvalid - 1 - wave) / kRotWaves + 1 : 0;
    const int dlast = ((a.D + 3) / 4 - 1) * 4;
    const int j0 = 4 * ql, jl = min(j0, dlast);
    for (int k = 0; k < nrow_w; k += 2) {
      const int kk = k + hl;
      const bool live = kk < nrow_w;
      const int rl = wave + kRotWaves * min(kk, nrow_w - 1);
      float f = 0.f;
#pragma unroll
      for (int sl = 0; sl < kRotSlots; ++sl) f += fpart[sl * BM + rl];
      const int i = row0 + rl;
      const size_t g = (size_t)run * a.NP + i;
      const float fx = a.fit_cur[g];
      const bool accept = f < fx;
      const bool refresh = !accept && a.changed[g] != 0;
      const float Fr = JDE ? ctl[rl].F : a.F;
      if (live && (accept || refresh)) {
        const float4 xv = ld4(base + (size_t)i * a.ldx + jl);
        float4 out = xv;
        if (accept) {
          const float4 v1 = ld4(base + (size_t)donors[rl * 4 + 0] * a.ldx + jl);
          const float4 v2 = ld4(base + (size_t)donors[rl * 4 + 1] * a.ldx + jl);
          const float4 v3 = ld4(base + (size_t)donors[rl * 4 + 2] * a.ldx + jl);
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const unsigned long long m = planes[(size_t)rl * tq * 4 + b];
            const float mv = mutant_coord(get(v1, b), get(v2, b), get(v3, b),
                                          Fr, a.lo, a.hi);
            set(out, b, ((m >> ql) & 1ull) ? mv : get(xv, b));
          }
        }
        if (j0 < a.D) st4(a.pop_next + g * a.ldx + j0, out);
      }
      if (live && ql == 0) {
        a.fit_next[g] = accept ? f : fx;
        a.changed[g] = accept ? 1 : 0;
        if constexpr (JDE) {
          // the trial's F', CR' survive only with the trial
          a.jp_next[g] = accept ? make_float2(ctl[rl].F, ctl[rl].CR)
                                : a.jp_cur[g];
        }
        if (accept) record_accept(a, run, i, f);
      }
    }
    return;
  }
  for (int rl = wave; rl < nvalid; rl += kRotWaves) {
    float f = 0.f;
#pragma unroll
    for (int sl = 0; sl < kRotSlots; ++sl) f += fpart[sl * BM + rl];
    const int i = row0 + rl;
    if (EVAL) {
      if (lane == 0) a.fit_next[i] = f;
      continue;
    }
    const size_t g = (size_t)run * a.NP + i;
    const float fx = a.fit_cur[g];
    const bool accept = f < fx;
    const bool refresh = !accept && a.changed[g] != 0;
    const float Fr = JDE ? ctl[rl].F : a.F;
    if (accept || refresh) {
      const float* xrow = base + (size_t)i * a.ldx;
      float* nrow = a.pop_next + g * a.ldx;
      const float* x1 = base + (size_t)donors[rl * 4 + 0] * a.ldx;
      const float* x2 = base + (size_t)donors[rl * 4 + 1] * a.ldx;
      const float* x3 = base + (size_t)donors[rl * 4 + 2] * a.ldx;
      const int dlast = ((a.D + 3) / 4 - 1) * 4;
      for (int t0 = 0; t0 < tq; t0 += 4) {
        float4 xv[4], v1[4], v2[4], v3[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int jl = min(4 * (lane + 64 * (t0 + u)), dlast);
          xv[u] = ld4(xrow + jl);
          if (accept) {
            v1[u] = ld4(x1 + jl);
            v2[u] = ld4(x2 + jl);
            v3[u] = ld4(x3 + jl);
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = t0 + u;
          if (t >= tq) break;
          const int j0 = 4 * (lane + 64 * t);
          float4 out = xv[u];
          if (accept) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const unsigned long long m = planes[((size_t)rl * tq + t) * 4 + b];
              const float mv = mutant_coord(get(v1[u], b), get(v2[u], b),
                                            get(v3[u], b), Fr, a.lo, a.hi);
              set(out, b, ((m >> lane) & 1ull) ? mv : get(xv[u], b));
            }
          }
          if (j0 < a.D) st4(nrow + j0, out);
        }
      }
    }
    if (lane == 0) {
      a.fit_next[g] = accept ? f : fx;
      a.changed[g] = accept ? 1 : 0;
      if constexpr (JDE) {
        // the trial's F', CR' survive only with the trial
        a.jp_next[g] = accept ? make_float2(ctl[rl].F, ctl[rl].CR)
                              : a.jp_cur[g];
      }
      if (accept) record_accept(a, run, i, f);
    }
  }
}

}  // namespace de
