// de_kernels.hip -- gfx950 kernels of the DE/rand/1/bin generation step.
//
// One launch advances every run by one synchronous generation (Section 2 of
// arXiv 2405.16551): draws, DE/rand/1 mutation (eq. 2) with clamping,
// binomial crossover (eq. 3), fitness of the trial vector, greedy selection,
// write of generation g+1 into the other ping-pong buffer and the per-run
// statistics.  Two fused kernels cover the two objective families of
// Section 7.3.1:
//
//   k_sep   separable objective (shifted sphere).  A group of LPI lanes owns
//           one individual; each lane owns 4 consecutive coordinates per
//           step (one Philox block, one float4 of each row).  Rows of more
//           than 256 coordinates take k_sep_row (one wave per row, donors
//           drawn once per workgroup, scalar row pointers).
//   k_rot   rotated objective z = R (x - o), f = sum z^2 + sin^2(3z).  A
//           workgroup owns a tile of BM trial rows: it builds them into LDS
//           as the A operand, runs Z = Y R^T on MFMA with the objective and
//           row sum fused into the epilogue, then selects and writes.  R is
//           read from L2 in a fragment-major layout prepared once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <mutex>

#include "de_device.hpp"
#include "de_internal.h"
#include "de_tile.hpp"

namespace de {

// ---------------------------------------------------------------------------
// Separable objective.  EVAL: f of rows pop_cur[0..nrows) into fit_next.
template <int LPI, int ITER, bool EVAL, bool JDE>
__global__ __launch_bounds__(256) void k_sep(GenArgs a) {
  constexpr int IPB = 256 / LPI;
  const int lb = xcd_logical_block((int)blockIdx.x, (int)gridDim.x);
  const int slot = (int)threadIdx.x / LPI, ln = (int)threadIdx.x % LPI;
  const int g = lb * IPB + slot;
  if (g >= a.nrows) return;  // whole LPI-groups leave together
  const int run = EVAL ? 0 : g / a.NP;
  const int i = EVAL ? g : g - run * a.NP;
  const float* xrow = a.pop_cur + (size_t)g * a.ldx;
  // Last 4-coordinate chunk that lies inside every row: loads past the end
  // of a row are redirected there (and their values ignored), so no load
  // sits behind a per-lane branch and all of them stay in flight together.
  const int dlast = ((a.D + 3) / 4 - 1) * 4;

  Donors d{0, 0, 0, 0};
  const float *x1 = xrow, *x2 = xrow, *x3 = xrow;
  float F = a.F;
  uint32_t crt = a.cr_threshold;
  Control ctl{0.f, 0.f};
  if (JDE && !EVAL) {
    const float2 c = a.jp_cur[g];
    ctl = jde_control((uint32_t)run, a.gen, i, a.key_lo, a.key_hi, a.jF_lo,
                      a.jF_span, a.jtau_F, a.jtau_CR, Control{c.x, c.y});
    F = ctl.F;
    crt = cr_threshold_of(ctl.CR);
  }
  if (!EVAL) {
    d = pick_donors((uint32_t)run, a.gen, i, a.NP, a.D, a.key_lo, a.key_hi);
    const float* base = a.pop_cur + (size_t)run * a.NP * a.ldx;
    x1 = base + (size_t)d.r1 * a.ldx;
    x2 = base + (size_t)d.r2 * a.ldx;
    x3 = base + (size_t)d.r3 * a.ldx;
  }
  float4 xv[ITER], uv[ITER], v1[ITER], v2[ITER], v3[ITER], ov[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int jl = min(4 * (ln + it * LPI), dlast);
    xv[it] = ld4(xrow + jl);
    ov[it] = ld4(a.o + jl);
    if (!EVAL) {
      v1[it] = ld4(x1 + jl);
      v2[it] = ld4(x2 + jl);
      v3[it] = ld4(x3 + jl);
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int q = ln + it * LPI, j0 = 4 * q;
    uv[it] = xv[it];
    if (!EVAL) {
      const Words4 w = draw_block(kTagXover, (uint32_t)run, a.gen,
                                  (uint32_t)i, (uint32_t)q, a.key_lo,
                                  a.key_hi);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const bool tk = (j0 + b < a.D) &&
                        take_mutant(w.w[b], j0 + b, d.jrand, crt);
        const float mv = mutant_coord(get(v1[it], b), get(v2[it], b),
                                      get(v3[it], b), F, a.lo, a.hi);
        set(uv[it], b, tk ? mv : get(xv[it], b));
      }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float y = get(uv[it], b) - get(ov[it], b);
      acc = (j0 + b < a.D) ? fmaf(y, y, acc) : acc;
    }
  }
  const float f = group_sum<LPI>(acc);
  if (EVAL) {
    if (ln == 0) a.fit_next[g] = f;
    return;
  }
  const float fx = a.fit_cur[g];
  const bool accept = f < fx;
  // a rejected row is rewritten only if the other buffer holds a stale copy
  // (the row changed in the previous generation)
  if (accept || a.changed[g] != 0) {
    float* nrow = a.pop_next + (size_t)g * a.ldx;
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int j0 = 4 * (ln + it * LPI);
      if (j0 < a.D) st4(nrow + j0, accept ? uv[it] : xv[it]);
    }
  }
  if (ln == 0) {
    a.fit_next[g] = accept ? f : fx;
    a.changed[g] = accept ? 1 : 0;
    if constexpr (JDE) {
      a.jp_next[g] = accept ? make_float2(ctl.F, ctl.CR) : a.jp_cur[g];
    }
    if (accept) record_accept(a, run, i, f);
  }
}

// BF16 tiles of fewer than 1024 threads: two workgroups per CU (four
// waves per SIMD, 128 registers).
template <class P, int BM, int NT, bool EVAL, bool JDE, bool PAIR = false>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(
    (sizeof(typename P::T) == 2 && NT < 1024) ? 4 : 1)))
void k_rot(GenArgs a) {
  const int lb = xcd_logical_block((int)blockIdx.x, (int)gridDim.x);
  int run = 0, row0 = 0, nvalid = 0;
  if (EVAL) {
    row0 = lb * BM;
    nvalid = min(BM, a.nrows - row0);
  } else {
    const int tiles = (a.NP + BM - 1) / BM;
    run = lb / tiles;
    row0 = (lb - run * tiles) * BM;
    nvalid = min(BM, a.NP - row0);
  }
  rot_tile<P, BM, NT, EVAL, JDE, PAIR>(a, run, row0, nvalid);
}

// jDE: every individual starts from the same (F, CR).
__global__ __launch_bounds__(256) void k_fill_control(float2* jp, int n,
                                                      float F, float CR) {
  for (int t = blockIdx.x * 256 + threadIdx.x; t < n; t += gridDim.x * 256)
    jp[t] = make_float2(F, CR);
}

// ---------------------------------------------------------------------------
// Initial population (Section 2): x = lo + u (hi - lo), u = k 2^-24.
__global__ __launch_bounds__(256) void k_init(GenArgs a) {
  const int nq = (a.D + 3) / 4;
  const size_t total = (size_t)a.nrows * nq;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (size_t)gridDim.x * 256) {
    const int g = (int)(t / nq), q = (int)(t % nq);
    const int run = g / a.NP, i = g - run * a.NP;
    const Words4 w = draw_block(kTagInit, (uint32_t)run, 0u, (uint32_t)i,
                                (uint32_t)q, a.key_lo, a.key_hi);
    const float span = a.hi - a.lo;
    float4 v;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float u = (float)(w.w[b] >> 8) * 0x1.0p-24f;
      set(v, b, fmaf(u, span, a.lo));
    }
    float* p = a.pop_next + (size_t)g * a.ldx + 4 * q;
    if (4 * q + 4 <= a.D) {
      st4(p, v);
    } else {
      for (int b = 0; 4 * q + b < a.D; ++b) p[b] = get(v, b);
    }
  }
}

// o -> zero-padded copy; R -> MFMA B-operand layout (zero-padded).
// Waits on the constant 100 MHz clock (s_memrealtime) for `ticks` ticks;
// the loop ends once the clock has advanced that far, whatever the shader
// clock does.
__global__ __launch_bounds__(64) void k_delay(uint64_t ticks) {
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  while (__builtin_amdgcn_s_memrealtime() - t0 < ticks)
    __builtin_amdgcn_s_sleep(2);
}

__global__ __launch_bounds__(256) void k_prep_shift(const float* o, int D,
                                                    int dpad, float* o_pad) {
  for (int k = blockIdx.x * 256 + threadIdx.x; k < dpad; k += gridDim.x * 256)
    o_pad[k] = k < D ? o[k] : 0.f;
}

// BF16 layout: element (n, k) of R (z_n = sum_k R[n][k] y_k) goes to block
// nb = n / 32, k-step kb = k / 16, lane (n % 32) + 32 ((k % 16) / 8),
// slot k % 8.
__global__ __launch_bounds__(256) void k_prep_rot_bf16(const float* R, int ldr,
                                                       int D, int dpad,
                                                       __bf16* rop) {
  const size_t total = (size_t)dpad * dpad;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (size_t)gridDim.x * 256) {
    const int n = (int)(t / dpad), k = (int)(t % dpad);
    const float v = (n < D && k < D) ? R[(size_t)n * ldr + k] : 0.f;
    const size_t nb = n / 32, kb = k / 16;
    const int ln = (n % 32) + 32 * ((k % 16) / 8);
    rop[((nb * (dpad / 16) + kb) * 64 + ln) * 8 + (k % 8)] = (__bf16)v;
  }
}

// FP32 layout: block nb = n / 32, group k8 = k / 8, lane (n % 32) + 32 (k % 2),
// slot (k % 8) / 2.
__global__ __launch_bounds__(256) void k_prep_rot_f32(const float* R, int ldr,
                                                      int D, int dpad,
                                                      float* rop) {
  const size_t total = (size_t)dpad * dpad;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (size_t)gridDim.x * 256) {
    const int n = (int)(t / dpad), k = (int)(t % dpad);
    const float v = (n < D && k < D) ? R[(size_t)n * ldr + k] : 0.f;
    const size_t nb = n / 32, k8 = k / 8;
    const int ln = (n % 32) + 32 * (k % 2);
    rop[((nb * (dpad / 8) + k8) * 64 + ln) * 4 + (k % 8) / 2] = v;
  }
}

// ---------------------------------------------------------------------------
// Statistics.
__global__ void k_stats_reset(GenArgs a, int reset_accepted) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < a.runs;
       r += gridDim.x * blockDim.x) {
    a.best_key[r] = ~0ull;
    a.hit_gen[r] = kNoHit;
    if (reset_accepted) a.accepted[r] = 0ull;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.done = 0u;
}

// Every row of the other buffer is stale (after initialisation or a load).
__global__ __launch_bounds__(256) void k_mark_changed(unsigned char* changed,
                                                      int n) {
  for (int t = blockIdx.x * 256 + threadIdx.x; t < n; t += gridDim.x * 256)
    changed[t] = 1;
}

// best_key[r] = min over i of key(fit[r][i], i); one wave per run slice.
__global__ __launch_bounds__(256) void k_best_from_fit(GenArgs a) {
  const int run = blockIdx.y;
  unsigned long long best = ~0ull;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < a.NP; i += gridDim.x * 256)
    best = min(best, fit_key(a.fit_cur[(size_t)run * a.NP + i], i));
  for (int m = 32; m >= 1; m >>= 1) {
    const unsigned long long o =
        ((unsigned long long)__shfl_xor((unsigned)(best >> 32), m, 64) << 32) |
        (unsigned long long)__shfl_xor((unsigned)best, m, 64);
    best = min(best, o);
  }
  if ((threadIdx.x % 64) == 0) atomicMin(&a.best_key[run], best);
}

// FP64 re-evaluation of each run's current best row (one workgroup per
// run): the row is taken as the FP32 values it holds, y = x - o and, for the
// rotated objective, z = R y with R the FP32 matrix the caller supplied, are
// formed in FP64, and f is summed in a fixed order.  rf32 is R row-major
// [D][D]; f64 and idx receive one value per run.
__global__ __launch_bounds__(256) void k_best_f64(GenArgs a, int kind,
                                                  const float* rf32,
                                                  double* f64, int* idx) {
  __shared__ double ys[4096];
  __shared__ double red[256];
  const int run = blockIdx.x;
  const unsigned long long key = a.best_key[run];
  const int i = (int)(key & 0xFFFFFFFFu);
  const float* x = a.pop_cur + ((size_t)run * a.NP + i) * a.ldx;
  double part = 0.0;
  if (kind == kObjSphere) {
    for (int j = threadIdx.x; j < a.D; j += 256) {
      const double y = (double)x[j] - (double)a.o[j];
      part = fma(y, y, part);
    }
  } else {
    for (int j = threadIdx.x; j < a.D; j += 256)
      ys[j] = (double)x[j] - (double)a.o[j];
    __syncthreads();
    for (int r = threadIdx.x; r < a.D; r += 256) {
      double z = 0.0;
      for (int j = 0; j < a.D; ++j)
        z = fma((double)rf32[(size_t)j * a.D + r], ys[j], z);
      const double sz = sin(3.0 * z);
      part += fma(z, z, sz * sz);
    }
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int m = 128; m >= 1; m >>= 1) {
    if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    f64[run] = red[0];
    idx[run] = i;
  }
}

// Transposed FP32 copy of R (for the FP64 re-evaluation).
__global__ __launch_bounds__(256) void k_copy_rot(const float* R, int ldr,
                                                  int D, float* rf32) {
  const size_t total = (size_t)D * D;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (size_t)gridDim.x * 256)
    rf32[t] = R[(t % D) * ldr + t / D];
}

// Runs whose current best is already <= target hit at generation `gen`.
__global__ void k_hit_check(GenArgs a, unsigned long long target_key) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < a.runs;
       r += gridDim.x * blockDim.x) {
    if ((a.best_key[r] >> 32) <= (target_key >> 32) &&
        a.best_key[r] != ~0ull) {
      const unsigned long long old = atomicMin(&a.hit_gen[r],
                                               (unsigned long long)a.gen);
      if (old == kNoHit) atomicAdd(a.done, 1u);
    }
  }
}

// Draws of generation a.gen: idx4 [runs][NP][4], mask [runs][NP][ceil(D/32)].
__global__ __launch_bounds__(256) void k_debug_draws(GenArgs a, int* idx4,
                                                     uint32_t* mask) {
  const int nw = (a.D + 31) / 32;
  const size_t total = (size_t)a.runs * a.NP * (size_t)(nw + 1);
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (size_t)gridDim.x * 256) {
    const size_t g = t / (nw + 1);
    const int wsel = (int)(t % (nw + 1));
    const int run = (int)(g / a.NP), i = (int)(g % a.NP);
    const Donors d = pick_donors((uint32_t)run, a.gen, i, a.NP, a.D, a.key_lo,
                                 a.key_hi);
    if (wsel == nw) {
      if (idx4) {
        idx4[g * 4 + 0] = d.r1;
        idx4[g * 4 + 1] = d.r2;
        idx4[g * 4 + 2] = d.r3;
        idx4[g * 4 + 3] = d.jrand;
      }
      continue;
    }
    if (!mask) continue;
    uint32_t word = 0;
    for (int qq = 0; qq < 8; ++qq) {
      const int q = wsel * 8 + qq;
      if (4 * q >= a.D) break;
      const Words4 w = draw_block(kTagXover, (uint32_t)run, a.gen, (uint32_t)i,
                                  (uint32_t)q, a.key_lo, a.key_hi);
      for (int b = 0; b < 4; ++b) {
        const int j = 4 * q + b;
        if (j < a.D && take_mutant(w.w[b], j, d.jrand, a.cr_threshold))
          word |= 1u << (j % 32);
      }
    }
    mask[g * nw + wsel] = word;
  }
}

// ---------------------------------------------------------------------------
// Launchers.

// ---------------------------------------------------------------------------
// Separable objective, resident form for small problems (rows of at most 256
// coordinates, a run's two population buffers within the LDS limit): one
// workgroup per run keeps the population, fitness and shift in LDS for
// n_gens generations.  Each generation is computed exactly as k_sep<LPI, 1>
// computes it (same lanes per individual, draws, operations and summation
// order), so the result equals n_gens launches of k_sep bit for bit; what
// is saved is the launch and the global round trip per generation.  The
// final generation goes to pop_final / fit_final, and every row is marked
// changed (the other global buffer is stale).
template <int LPI>
__global__ __launch_bounds__(1024) void k_sep_resident(GenArgs a, int n_gens,
                                                       float* pop_final,
                                                       float* fit_final) {
  extern __shared__ __align__(16) float rs[];
  const int run = (int)blockIdx.x;
  const int NP = a.NP, ldx = a.ldx, D = a.D;
  const int dq = (D + 3) / 4 * 4;  // shift floats used
  // P0, P1 [NP][ldx] and the shift (16-byte aligned: ldx % 4 == 0), then
  // F0, F1 [NP]
  float* P0 = rs;
  float* P1 = P0 + (size_t)NP * ldx;
  float* so = P1 + (size_t)NP * ldx;
  float* F0 = so + dq;
  float* F1 = F0 + NP;
  const size_t row0 = (size_t)run * NP;
  {
    const float4* src =
        reinterpret_cast<const float4*>(a.pop_cur + row0 * ldx);
    const int n4 = NP * ldx / 4;
    for (int t = (int)threadIdx.x; t < n4; t += (int)blockDim.x) {
      const float4 v = src[t];
      reinterpret_cast<float4*>(P0)[t] = v;
      reinterpret_cast<float4*>(P1)[t] = v;  // padding alike in both
    }
    for (int t = (int)threadIdx.x; t < NP; t += (int)blockDim.x)
      F0[t] = a.fit_cur[row0 + t];
    for (int t = (int)threadIdx.x; t < dq; t += (int)blockDim.x)
      so[t] = a.o[t];
  }
  __syncthreads();
  const int groups = (int)blockDim.x / LPI;
  const int slot = (int)threadIdx.x / LPI, ln = (int)threadIdx.x % LPI;
  const int dlast = ((D + 3) / 4 - 1) * 4;
  const int jl = min(4 * ln, dlast), j0 = 4 * ln;
  const float4 ov = ld4(so + jl);
  for (int gi = 0; gi < n_gens; ++gi) {
    const uint32_t gen = a.gen + (uint32_t)gi;
    const float* Pc = (gi & 1) ? P1 : P0;
    float* Pn = (gi & 1) ? P0 : P1;
    const float* Fc = (gi & 1) ? F1 : F0;
    float* Fn = (gi & 1) ? F0 : F1;
    for (int i = slot; i - slot < NP; i += groups) {
      if (i >= NP) continue;  // whole LPI-groups, whose shuffles stay inside
      const Donors d = pick_donors((uint32_t)run, gen, i, NP, D, a.key_lo,
                                   a.key_hi);
      const float4 xv = ld4(Pc + (size_t)i * ldx + jl);
      const float4 v1 = ld4(Pc + (size_t)d.r1 * ldx + jl);
      const float4 v2 = ld4(Pc + (size_t)d.r2 * ldx + jl);
      const float4 v3 = ld4(Pc + (size_t)d.r3 * ldx + jl);
      const Words4 w = draw_block(kTagXover, (uint32_t)run, gen, (uint32_t)i,
                                  (uint32_t)ln, a.key_lo, a.key_hi);
      float4 uv = xv;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const bool tk = (j0 + b < D) &&
                        take_mutant(w.w[b], j0 + b, d.jrand, a.cr_threshold);
        const float mv = mutant_coord(get(v1, b), get(v2, b), get(v3, b), a.F,
                                      a.lo, a.hi);
        set(uv, b, tk ? mv : get(xv, b));
      }
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const float y = get(uv, b) - get(ov, b);
        acc = (j0 + b < D) ? fmaf(y, y, acc) : acc;
      }
      const float f = group_sum<LPI>(acc);
      const float fx = Fc[i];
      const bool accept = f < fx;
      if (j0 < D) st4(Pn + (size_t)i * ldx + j0, accept ? uv : xv);
      if (ln == 0) {
        Fn[i] = accept ? f : fx;
        if (accept) record_accept_at(a, run, i, f, gen);
      }
    }
    __syncthreads();
  }
  const float* Pf = (n_gens & 1) ? P1 : P0;
  const float* Ff = (n_gens & 1) ? F1 : F0;
  {
    float4* dst = reinterpret_cast<float4*>(pop_final + row0 * ldx);
    const int n4 = NP * ldx / 4;
    for (int t = (int)threadIdx.x; t < n4; t += (int)blockDim.x)
      dst[t] = reinterpret_cast<const float4*>(Pf)[t];
    for (int t = (int)threadIdx.x; t < NP; t += (int)blockDim.x) {
      fit_final[row0 + t] = Ff[t];
      a.changed[row0 + t] = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Separable objective, one wave per row, rows of more than 256 coordinates
// (ITER float4 per lane).  The work per row is mostly VALU, so this form
// trims instructions without changing any result:
//   - wave 0 draws the donors (and jDE controls) of the workgroup's four
//     rows in four lanes and hands them over in LDS (one Philox block per
//     four rows instead of one per row); the other waves issue their target
//     and shift loads meanwhile;
//   - row pointers are wave-uniform, so loads take a scalar base and one
//     32-bit lane offset;
//   - the crossover test compares the raw word with a precomputed bound:
//     (w >> 8) <= t  <=>  w <= t * 256 + 255 (every word when t = 2^24);
//   - the end-of-row checks run only on the chunk that holds the end.
// Rows of up to 1024 coordinates fit in 96 registers: five waves per SIMD
// (one more than the compiler picks unasked) keep more loads in flight.
template <int ITER, bool JDE>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(ITER <= 4 ? 5 : 1)))
void k_sep_row(GenArgs a) {
  __shared__ int sd[4][4];
  __shared__ Control sc[4];
  const int lb = xcd_logical_block((int)blockIdx.x, (int)gridDim.x);
  const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
  const int g0 = lb * 4;
  if (wave == 0 && lane < 4 && g0 + lane < a.nrows) {
    const int gl = g0 + lane;
    const int run = gl / a.NP, i = gl - run * a.NP;
    const Donors d =
        pick_donors((uint32_t)run, a.gen, i, a.NP, a.D, a.key_lo, a.key_hi);
    sd[lane][0] = d.r1;
    sd[lane][1] = d.r2;
    sd[lane][2] = d.r3;
    sd[lane][3] = d.jrand;
    if constexpr (JDE) {
      const float2 c = a.jp_cur[gl];
      sc[lane] = jde_control((uint32_t)run, a.gen, i, a.key_lo, a.key_hi,
                             a.jF_lo, a.jF_span, a.jtau_F, a.jtau_CR,
                             Control{c.x, c.y});
    }
  }
  const int g = __builtin_amdgcn_readfirstlane(g0 + wave);
  const bool live = g < a.nrows;
  const int run = live ? g / a.NP : 0, i = live ? g - run * a.NP : 0;
  const int dlast = ((a.D + 3) / 4 - 1) * 4;
  const float* xrow = a.pop_cur + (size_t)(live ? g : 0) * a.ldx;
  float4 xv[ITER], v1[ITER], v2[ITER], v3[ITER], ov[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const uint32_t jl = (uint32_t)min(4 * (lane + 64 * it), dlast);
    xv[it] = ld4(xrow + jl);
    ov[it] = ld4(a.o + jl);
  }
  float fx = 0.f;
  int chg = 0;
  if (live) {
    fx = a.fit_cur[g];
    chg = a.changed[g];
  }
  __syncthreads();
  if (!live) return;  // wave-uniform, after the only barrier
  const int r1 = __builtin_amdgcn_readfirstlane(sd[wave][0]);
  const int r2 = __builtin_amdgcn_readfirstlane(sd[wave][1]);
  const int r3 = __builtin_amdgcn_readfirstlane(sd[wave][2]);
  const int jrand = __builtin_amdgcn_readfirstlane(sd[wave][3]);
  float F = a.F;
  uint32_t crt = a.cr_threshold;
  Control ctl{0.f, 0.f};
  if constexpr (JDE) {
    ctl = sc[wave];
    F = ctl.F;
    crt = cr_threshold_of(ctl.CR);
  }
  const uint32_t wmax = crt >= (1u << 24) ? 0xFFFFFFFFu : (crt << 8) | 0xFFu;
  const float* base = a.pop_cur + (size_t)run * a.NP * a.ldx;
  const float* x1 = base + (size_t)r1 * a.ldx;
  const float* x2 = base + (size_t)r2 * a.ldx;
  const float* x3 = base + (size_t)r3 * a.ldx;
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const uint32_t jl = (uint32_t)min(4 * (lane + 64 * it), dlast);
    v1[it] = ld4(x1 + jl);
    v2[it] = ld4(x2 + jl);
    v3[it] = ld4(x3 + jl);
  }
  float acc = 0.f;
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int q = lane + 64 * it, j0 = 4 * q;
    const Words4 w = draw_block(kTagXover, (uint32_t)run, a.gen, (uint32_t)i,
                                (uint32_t)q, a.key_lo, a.key_hi);
    float4 u = xv[it];
    if (256 * (it + 1) <= a.D) {
      // every coordinate of this chunk lies inside the row
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bool tk = (w.w[c] <= wmax) || (j0 + c == jrand);
        const float mv = mutant_coord(get(v1[it], c), get(v2[it], c),
                                      get(v3[it], c), F, a.lo, a.hi);
        set(u, c, tk ? mv : get(xv[it], c));
        const float y = get(u, c) - get(ov[it], c);
        acc = fmaf(y, y, acc);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bool in = j0 + c < a.D;
        const bool tk = in && ((w.w[c] <= wmax) || (j0 + c == jrand));
        const float mv = mutant_coord(get(v1[it], c), get(v2[it], c),
                                      get(v3[it], c), F, a.lo, a.hi);
        set(u, c, tk ? mv : get(xv[it], c));
        const float y = get(u, c) - get(ov[it], c);
        acc = in ? fmaf(y, y, acc) : acc;
      }
    }
    v1[it] = u;  // the trial chunk replaces the first donor's
  }
  const float f = group_sum<64>(acc);
  const bool accept = f < fx;
  // a rejected row is rewritten only if the other buffer holds a stale copy
  if (accept || chg != 0) {
    float* nrow = a.pop_next + (size_t)g * a.ldx;
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int j0 = 4 * (lane + 64 * it);
      if (j0 < a.D) st4(nrow + j0, accept ? v1[it] : xv[it]);
    }
  }
  if (lane == 0) {
    a.fit_next[g] = accept ? f : fx;
    a.changed[g] = accept ? 1 : 0;
    if constexpr (JDE) {
      // the trial's F', CR' survive only with the trial
      a.jp_next[g] = accept ? make_float2(ctl.F, ctl.CR) : a.jp_cur[g];
    }
    if (accept) record_accept(a, run, i, f);
  }
}

namespace {

int grid_for(size_t work, int per_block) {
  size_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > (1u << 20)) b = 1u << 20;
  return (int)b;
}

template <int LPI, int ITER, bool EVAL, bool JDE>
hipError_t launch_sep_t(const GenArgs& a, hipStream_t s) {
  constexpr int IPB = 256 / LPI;
  const int blocks = (a.nrows + IPB - 1) / IPB;
  hipLaunchKernelGGL((k_sep<LPI, ITER, EVAL, JDE>), dim3(blocks), dim3(256),
                     0, s, a);
  return hipGetLastError();
}

template <int ITER, bool JDE>
hipError_t launch_sep_row_t(const GenArgs& a, hipStream_t s) {
  const int blocks = (a.nrows + 3) / 4;
  hipLaunchKernelGGL((k_sep_row<ITER, JDE>), dim3(blocks), dim3(256), 0, s,
                     a);
  return hipGetLastError();
}

template <bool EVAL, bool JDE>
hipError_t launch_sep_j(const GenArgs& a, hipStream_t s) {
  const int nq = (a.D + 3) / 4;
  if (nq <= 4) return launch_sep_t<4, 1, EVAL, JDE>(a, s);
  if (nq <= 8) return launch_sep_t<8, 1, EVAL, JDE>(a, s);
  if (nq <= 16) return launch_sep_t<16, 1, EVAL, JDE>(a, s);
  if (nq <= 32) return launch_sep_t<32, 1, EVAL, JDE>(a, s);
  if (nq <= 64) return launch_sep_t<64, 1, EVAL, JDE>(a, s);
  if constexpr (EVAL) {
    // evaluation only: the wide rows of k_sep
    if (nq <= 128) return launch_sep_t<64, 2, true, false>(a, s);
    if (nq <= 256) return launch_sep_t<64, 4, true, false>(a, s);
    if (nq <= 512) return launch_sep_t<64, 8, true, false>(a, s);
    if (nq <= 1024) return launch_sep_t<64, 16, true, false>(a, s);
  } else {
    // generations of rows over 256 coordinates: one wave per row
    if (nq <= 128) return launch_sep_row_t<2, JDE>(a, s);
    if (nq <= 256) return launch_sep_row_t<4, JDE>(a, s);
    if (nq <= 512) return launch_sep_row_t<8, JDE>(a, s);
    if (nq <= 1024) return launch_sep_row_t<16, JDE>(a, s);
  }
  return hipErrorInvalidValue;
}

template <bool EVAL>
hipError_t launch_sep_e(const GenArgs& a, hipStream_t s) {
  if (!EVAL && a.jde) return launch_sep_j<false, true>(a, s);
  return launch_sep_j<EVAL, false>(a, s);
}

template <int LPI>
hipError_t launch_resident_t(const GenArgs& a, int n_gens, float* pop_final,
                             float* fit_final, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_sep_resident<LPI>);
  const hipError_t e = set_max_dynamic_lds(fn);
  if (e != hipSuccess) return e;
  int threads = ((a.NP * LPI + 63) / 64) * 64;
  threads = std::min(std::max(threads, 64), 1024);
  hipLaunchKernelGGL((k_sep_resident<LPI>), dim3(a.runs), dim3(threads),
                     sep_resident_lds_bytes(a.NP, a.ldx, a.D), s, a, n_gens,
                     pop_final, fit_final);
  return hipGetLastError();
}

template <class P, int BM, int NT, bool EVAL, bool JDE = false,
          bool PAIR = false>
hipError_t launch_rot_t(const GenArgs& a, hipStream_t s) {
  // the paired-row form covers rows of at most 32 quads (kPairMaxDpad)
  if (PAIR && a.dpad > kPairMaxDpad) return hipErrorInvalidValue;
  const size_t lds = rot_lds_bytes<P, BM, JDE>(a.dpad);
  const hipError_t e = set_max_dynamic_lds(
      reinterpret_cast<const void*>(&k_rot<P, BM, NT, EVAL, JDE, PAIR>));
  if (e != hipSuccess) return e;
  int blocks;
  if (EVAL) {
    blocks = (a.nrows + BM - 1) / BM;
  } else {
    blocks = a.runs * ((a.NP + BM - 1) / BM);
  }
  hipLaunchKernelGGL((k_rot<P, BM, NT, EVAL, JDE, PAIR>), dim3(blocks),
                     dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <bool EVAL>
hipError_t launch_rot_e(const GenArgs& a, int prec, hipStream_t s) {
  const long long tiles = EVAL ? (a.nrows + 63) / 64
                               : (long long)a.runs * ((a.NP + 63) / 64);
  const bool narrow = rot_bf16_narrow(a.dpad, tiles, device_cus());
  const bool f32_narrow = a.dpad <= kF32NarrowMaxDpad;
  if (!EVAL && a.jde) {
    // padded width up to 128: trials built two rows per wave instruction
    if (a.dpad <= kPairMaxDpad) {
      if (prec != kPrecBF16)
        return launch_rot_t<PrecF32Narrow, 32, 512, false, true, true>(a, s);
      return narrow ? launch_rot_t<PrecBF16, 64, kRotBf16ThreadsNarrow, false,
                                   true, true>(a, s)
                    : launch_rot_t<PrecBF16, 64, kRotBf16Threads, false, true,
                                   true>(a, s);
    }
    if (prec != kPrecBF16)
      return f32_narrow
                 ? launch_rot_t<PrecF32Narrow, 32, 512, false, true>(a, s)
                 : launch_rot_t<PrecF32, 32, 512, false, true>(a, s);
    return narrow
               ? launch_rot_t<PrecBF16, 64, kRotBf16ThreadsNarrow, false,
                              true>(a, s)
               : launch_rot_t<PrecBF16, 64, kRotBf16Threads, false, true>(a,
                                                                          s);
  }
  // padded width up to 128: trials built two rows per wave instruction
  if (!EVAL && a.dpad <= kPairMaxDpad) {
    if (prec != kPrecBF16)
      return launch_rot_t<PrecF32Narrow, 32, 512, false, false, true>(a, s);
    return narrow ? launch_rot_t<PrecBF16, 64, kRotBf16ThreadsNarrow, false,
                                 false, true>(a, s)
                  : launch_rot_t<PrecBF16, 64, kRotBf16Threads, false, false,
                                 true>(a, s);
  }
  if (prec != kPrecBF16)
    return f32_narrow ? launch_rot_t<PrecF32Narrow, 32, 512, EVAL>(a, s)
                      : launch_rot_t<PrecF32, 32, 512, EVAL>(a, s);
  return narrow ? launch_rot_t<PrecBF16, 64, kRotBf16ThreadsNarrow, EVAL>(a, s)
                : launch_rot_t<PrecBF16, 64, kRotBf16Threads, EVAL>(a, s);
}

}  // namespace

// Compute units of the current device (queried once per device and kept
// in an atomic, so that handles used from several host threads do not race;
// 256 if the query fails, which only affects the choice of tile width).
int device_cus() {
  constexpr int kMaxDevices = 64;
  static std::atomic<int> known[kMaxDevices];  // 0: not queried yet
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
  if (dev < kMaxDevices) {
    n = known[dev].load(std::memory_order_relaxed);
    if (n > 0) return n;
  }
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess ||
      n <= 0)
    return 256;
  if (dev < kMaxDevices) known[dev].store(n, std::memory_order_relaxed);
  return n;
}

// LDS bytes of the rotated kernel: BF16 tiles of 64 rows, FP32 tiles of 32
// rows (independent of the number of threads).
size_t rot_lds_bytes_host(int prec, int dpad, bool jde) {
  if (prec != kPrecBF16)
    return jde ? rot_lds_bytes<PrecF32, 32, true>(dpad)
               : rot_lds_bytes<PrecF32, 32>(dpad);
  return jde ? rot_lds_bytes<PrecBF16, 64, true>(dpad)
             : rot_lds_bytes<PrecBF16, 64>(dpad);
}

bool sep_supported(int D) { return (D + 3) / 4 <= 1024; }

size_t sep_resident_lds_bytes(int NP, int ldx, int D) {
  return ((size_t)2 * NP * ldx + (size_t)2 * NP + (size_t)(D + 3) / 4 * 4) *
         sizeof(float);
}

bool sep_resident_fits(int NP, int ldx, int D) {
  return (D + 3) / 4 <= 64 &&
         sep_resident_lds_bytes(NP, ldx, D) <= kSepResidentMaxLds;
}

hipError_t launch_sep_resident(const GenArgs& a, int n_gens, float* pop_final,
                               float* fit_final, hipStream_t s) {
  const int nq = (a.D + 3) / 4;
  if (nq <= 4) return launch_resident_t<4>(a, n_gens, pop_final, fit_final, s);
  if (nq <= 8) return launch_resident_t<8>(a, n_gens, pop_final, fit_final, s);
  if (nq <= 16)
    return launch_resident_t<16>(a, n_gens, pop_final, fit_final, s);
  if (nq <= 32)
    return launch_resident_t<32>(a, n_gens, pop_final, fit_final, s);
  if (nq <= 64)
    return launch_resident_t<64>(a, n_gens, pop_final, fit_final, s);
  return hipErrorInvalidValue;
}

hipError_t set_max_dynamic_lds(const void* fn) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  // (kernel, device) pairs already set, in a fixed table (no allocation on
  // any launch path); when it is full the attribute is simply set again
  constexpr int kSlots = 512;
  static std::mutex mu;
  static const void* done_fn[kSlots];
  static int done_dev[kSlots];
  static int n_done = 0;
  std::lock_guard<std::mutex> lk(mu);
  for (int k = 0; k < n_done; ++k)
    if (done_fn[k] == fn && done_dev[k] == dev) return hipSuccess;
  hipFuncAttributes fa{};
  e = hipFuncGetAttributes(&fa, fn);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kMaxLdsBytes - (int)fa.sharedSizeBytes);
  if (e == hipSuccess && n_done < kSlots) {
    done_fn[n_done] = fn;
    done_dev[n_done] = dev;
    ++n_done;
  }
  return e;
}

hipError_t note_hip(hipError_t e, const char* file, int line) {
  if (e != hipSuccess) {
    static const bool on = std::getenv("DE_DEBUG") != nullptr;
    if (on)
      std::fprintf(stderr, "libde: %s:%d: %s (%s)\n", file, line,
                   hipGetErrorName(e), hipGetErrorString(e));
  }
  return e;
}

hipError_t launch_delay(uint32_t ns, hipStream_t s) {
  const uint64_t ticks = (std::min(ns, kMaxDelayNs) + 9) / 10;  // 100 MHz
  hipLaunchKernelGGL(k_delay, dim3(1), dim3(64), 0, s, ticks);
  return hipGetLastError();
}

hipError_t launch_generation(const GenArgs& a, int kind, int prec,
                             hipStream_t s) {
  if (kind == kObjSphere) return launch_sep_e<false>(a, s);
  return launch_rot_e<false>(a, prec, s);
}

hipError_t launch_eval(const GenArgs& a, int kind, int prec, hipStream_t s) {
  if (kind == kObjSphere) return launch_sep_e<true>(a, s);
  return launch_rot_e<true>(a, prec, s);
}

hipError_t launch_init(const GenArgs& a, hipStream_t s) {
  const size_t work = (size_t)a.nrows * ((a.D + 3) / 4);
  hipLaunchKernelGGL(k_init, dim3(grid_for(work, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_control(float2* jp, int n, float F, float CR,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_fill_control, dim3(grid_for(n, 256)), dim3(256), 0, s,
                     jp, n, F, CR);
  return hipGetLastError();
}

hipError_t launch_prep(const float* o, const float* R, int ldr, int D,
                       int dpad, int kind, int prec, float* o_pad, void* rop,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_prep_shift, dim3(grid_for(dpad, 256)), dim3(256), 0, s,
                     o, D, dpad, o_pad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || kind != kObjRotOsc) return e;
  const size_t total = (size_t)dpad * dpad;
  if (prec == kPrecBF16) {
    hipLaunchKernelGGL(k_prep_rot_bf16, dim3(grid_for(total, 256)), dim3(256),
                       0, s, R, ldr, D, dpad, reinterpret_cast<__bf16*>(rop));
  } else {
    hipLaunchKernelGGL(k_prep_rot_f32, dim3(grid_for(total, 256)), dim3(256),
                       0, s, R, ldr, D, dpad, reinterpret_cast<float*>(rop));
  }
  return hipGetLastError();
}

hipError_t launch_stats_reset(const GenArgs& a, bool reset_accepted,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_stats_reset, dim3(grid_for(a.runs, 256)), dim3(256), 0,
                     s, a, reset_accepted ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_mark_changed(const GenArgs& a, hipStream_t s) {
  const int n = a.runs * a.NP;
  hipLaunchKernelGGL(k_mark_changed, dim3(grid_for(n, 256)), dim3(256), 0, s,
                     a.changed, n);
  return hipGetLastError();
}

hipError_t launch_best_from_fit(const GenArgs& a, hipStream_t s) {
  const int bx = grid_for(a.NP, 256) > 64 ? 64 : grid_for(a.NP, 256);
  hipLaunchKernelGGL(k_best_from_fit, dim3(bx, a.runs), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_best_f64(const GenArgs& a, int kind, const float* rf32,
                           double* f64, int* idx, hipStream_t s) {
  hipLaunchKernelGGL(k_best_f64, dim3(a.runs), dim3(256), 0, s, a, kind, rf32,
                     f64, idx);
  return hipGetLastError();
}

hipError_t launch_copy_rot(const float* R, int ldr, int D, float* rf32,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_copy_rot, dim3(grid_for((size_t)D * D, 256)), dim3(256),
                     0, s, R, ldr, D, rf32);
  return hipGetLastError();
}

hipError_t launch_hit_check(const GenArgs& a, unsigned long long target_key,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_hit_check, dim3(grid_for(a.runs, 256)), dim3(256), 0,
                     s, a, target_key);
  return hipGetLastError();
}

hipError_t launch_debug_draws(const GenArgs& a, int* idx4, uint32_t* mask,
                              hipStream_t s) {
  const size_t work = (size_t)a.runs * a.NP * (size_t)((a.D + 31) / 32 + 1);
  hipLaunchKernelGGL(k_debug_draws, dim3(grid_for(work, 256)), dim3(256), 0, s,
                     a, idx4, mask);
  return hipGetLastError();
}

}  // namespace de
