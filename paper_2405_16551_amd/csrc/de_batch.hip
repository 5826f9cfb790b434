// de_batch.hip -- many independent DE/rand/1/bin runs of mixed NP, D, F and
// CR advanced together (the C ABI of include/de_batch.h).
//
// Work unit: a tile = up to BM consecutive individuals of one run.  Each
// generation, a persistent grid of workgroups walks a list of tiles; every
// tile is built, evaluated and selected exactly as one tile of the
// per-problem rotated kernel (Section 2: eq. 2 mutation with clamping,
// eq. 3 binomial crossover, greedy selection; Section 7.3.1 objective
// z = R (x - o), f = sum z^2 + sin^2(3z)), with the run's own parameters
// read from a run table.  Runs of one dimension share o and R.
//
// Tile variants:
//   k_bt_rot<BM, NT>  generic: coordinates of the tile spread over all
//                     threads (one Philox block and one float4 per item),
//                     so small D keeps every lane busy; D padded to 32; one
//                     MFMA per LDS read.
//   k_bt_wide         the per-problem BF16 tile (64 rows, 1024 threads, D
//                     padded to 128, software-pipelined MFMA loop).
// An autotuner times each variant on each dimension's runs and keeps the
// fastest; a generation is then one launch per variant in use, and chunks
// of generations are one HIP graph launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <set>
#include <vector>

#include "de.h"
#include "de_batch.h"
#include "de_device.hpp"
#include "de_internal.h"
#include "de_tile.hpp"

namespace de {

// ---------------------------------------------------------------------------
// Device tables.

struct BRun {                   // one per run
  unsigned long long pop_off;   // element offset of row 0 in either buffer
  int fit_off;                  // index of individual 0 in fit / changed
  int NP, D, ldx, inst;
  float F;
  uint32_t cr_threshold;
  int pad_;
};

struct BInst {                  // one per dimension
  const float* o;               // shift, zero-padded to dpad_w
  const __bf16* rop_g;          // R, BF16 fragment-major, dpad_g = D up to 32
  const __bf16* rop_w;          // same for dpad_w = D up to 128
  int D, dpad_g, dpad_w, pad_;
};

struct BTile {
  int run, row0;
};

struct BatchArgs {
  float* pop[2];
  float* fit[2];
  unsigned char* changed;       // [sum NP] row changed in the last step
  unsigned long long* best_key; // [nruns]
  unsigned long long* hit_gen;  // [nruns]
  unsigned long long* accepted; // [nruns]
  unsigned int* done;           // runs that have hit the target
  const BRun* runs;
  const BInst* inst;
  const BTile* tiles;
  const long long* gen_dev;     // graph replays: generation = *gen_dev + gen_add
  long long gen_add;            // direct launches: gen_dev == nullptr
  int ntiles;
  float lo, hi, target;
  uint32_t key_lo, key_hi;
};

__device__ __forceinline__ long long batch_gen(const BatchArgs& b) {
  return (b.gen_dev ? *b.gen_dev : 0ll) + b.gen_add;
}

// LDS of the generic tile kernel for padded dimension dpad (multiple of 32).
template <int BM, int NT>
__host__ __device__ constexpr size_t bt_lds_bytes(int dpad) {
  constexpr int kSlots = (NT / 64) / (BM / 32);
  return (size_t)BM * (dpad + 8) * 2        // A tile, BF16
         + (size_t)BM * 4 * sizeof(int)     // donors and j_rand
         + (size_t)kSlots * BM * sizeof(float)  // partial row sums
         + (size_t)BM * sizeof(int)         // row actions
         + (size_t)BM * (dpad / 4);         // crossover bits, 4 per byte
}

// ---------------------------------------------------------------------------
// Generic tile kernel.
//   phase 1: items (row, 4-coordinate group) over all threads, two per step
//            with their loads issued together: Philox crossover block,
//            clamped mutant, y = u - o -> BF16 A tile; crossover bits -> LDS.
//   phase 2: wave w owns row block w % (BM/32) and column blocks
//            w / (BM/32) + k * slots; per block one 32x32x16 BF16 MFMA per
//            K-step, objective summed per row in registers, then a
//            reduce-scatter over the 32 lanes of each half-wave.
//   phase 3: row totals (slots summed in fixed order) -> selection and
//            statistics; then items (row, group) write the next generation
//            (trial rows recomputed from the stored bits, stale copies of
//            rejected rows refreshed).
// Four waves per SIMD (at most 128 registers): the tiles are latency-bound,
// so more workgroups per CU in the persistent grid pay more than the
// compiler's unconstrained allocation (143 registers, three waves).
template <int BM, int NT, bool EVAL>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
void k_bt_rot(BatchArgs b) {
  constexpr int kWaves = NT / 64;
  constexpr int kMblk = BM / 32;
  constexpr int kSlots = kWaves / kMblk;
  static_assert(kWaves % kMblk == 0, "waves per row block");
  extern __shared__ __align__(16) char smem[];
  const long long gen = batch_gen(b);
  const uint32_t gen32 = (uint32_t)gen;
  const int par = (int)(gen & 1);
  const float* pc = b.pop[par];
  float* pn = b.pop[par ^ 1];
  const float* fc = b.fit[par];
  float* fn = EVAL ? b.fit[par] : b.fit[par ^ 1];
  const int tid = (int)threadIdx.x, wave = tid / 64, lane = tid % 64;

  for (int t = (int)blockIdx.x; t < b.ntiles; t += (int)gridDim.x) {
    const BTile tile = b.tiles[t];
    const BRun rn = b.runs[tile.run];
    const BInst in = b.inst[rn.inst];
    const int dpad = in.dpad_g, stride = dpad + 8, nq4 = dpad / 4;
    const int nvalid = min(BM, rn.NP - tile.row0);
    __bf16* At = reinterpret_cast<__bf16*>(smem);
    int* donors = reinterpret_cast<int*>(smem + (size_t)BM * stride * 2);
    float* fpart = reinterpret_cast<float*>(donors + BM * 4);
    int* act = reinterpret_cast<int*>(fpart + kSlots * BM);
    unsigned char* xbits = reinterpret_cast<unsigned char*>(act + BM);
    const float* base = pc + rn.pop_off;
    const uint32_t rng_run = (uint32_t)tile.run;

    if (!EVAL) {
      for (int rl = tid; rl < nvalid; rl += NT) {
        const Donors d = pick_donors(rng_run, gen32, tile.row0 + rl, rn.NP,
                                     rn.D, b.key_lo, b.key_hi);
        donors[rl * 4 + 0] = d.r1;
        donors[rl * 4 + 1] = d.r2;
        donors[rl * 4 + 2] = d.r3;
        donors[rl * 4 + 3] = d.jrand;
      }
      __syncthreads();
    }

    // ---- phase 1.  Addresses are clamped into the tile's last valid row
    // and the row's last 4-group, so the loads carry no per-lane branch.
    const int dlast = ((rn.D + 3) / 4 - 1) * 4;
    const int items = BM * nq4;
    for (int it0 = tid; it0 < items; it0 += 2 * NT) {
      int rl[2], q[2];
      float4 xv[2], ov[2], v1[2], v2[2], v3[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int it = min(it0 + h * NT, items - 1);
        rl[h] = it / nq4;
        q[h] = it - rl[h] * nq4;
        const int r = min(rl[h], nvalid - 1);
        const int jl = min(4 * q[h], dlast);
        xv[h] = ld4(base + (size_t)(tile.row0 + r) * rn.ldx + jl);
        ov[h] = ld4(in.o + jl);
        if (!EVAL) {
          v1[h] = ld4(base + (size_t)donors[r * 4 + 0] * rn.ldx + jl);
          v2[h] = ld4(base + (size_t)donors[r * 4 + 1] * rn.ldx + jl);
          v3[h] = ld4(base + (size_t)donors[r * 4 + 2] * rn.ldx + jl);
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (it0 + h * NT >= items) break;
        const int r = rl[h], j0 = 4 * q[h];
        float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
        uint32_t bits = 0;
        if (r < nvalid && j0 < rn.D) {
          float4 uu = xv[h];
          if (!EVAL) {
            const Words4 w =
                draw_block(kTagXover, rng_run, gen32,
                           (uint32_t)(tile.row0 + r), (uint32_t)q[h],
                           b.key_lo, b.key_hi);
            const int jrand = donors[r * 4 + 3];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const bool tk = (j0 + c < rn.D) &&
                              take_mutant(w.w[c], j0 + c, jrand,
                                          rn.cr_threshold);
              const float mv =
                  mutant_coord(get(v1[h], c), get(v2[h], c), get(v3[h], c),
                               rn.F, b.lo, b.hi);
              set(uu, c, tk ? mv : get(xv[h], c));
              bits |= (tk ? 1u : 0u) << c;
            }
          }
#pragma unroll
          for (int c = 0; c < 4; ++c)
            set(y, c, (j0 + c < rn.D) ? get(uu, c) - get(ov[h], c) : 0.f);
        }
        bf16x4 yb;
        yb[0] = (__bf16)y.x;
        yb[1] = (__bf16)y.y;
        yb[2] = (__bf16)y.z;
        yb[3] = (__bf16)y.w;
        *reinterpret_cast<bf16x4*>(At + (size_t)r * stride + j0) = yb;
        if (!EVAL) xbits[r * nq4 + q[h]] = (unsigned char)bits;
      }
    }
    __syncthreads();

    // ---- phase 2: Z = Y R^T, objective fused.
    {
      const int nblk = dpad / 32, kbn = dpad / 16;
      const int mb = wave % kMblk, cg = wave / kMblk;
      const __bf16* ar =
          At + (size_t)(mb * 32 + lane % 32) * stride + 8 * (lane / 32);
      const bf16x8* rop = reinterpret_cast<const bf16x8*>(in.rop_g);
      floatx16 part = {};
      for (int nb = cg; nb < nblk; nb += kSlots) {
        floatx16 c = {};
        const bf16x8* rb = rop + (size_t)nb * kbn * 64 + lane;
        // kbn is even (dpad is a multiple of 32): two K-steps per pass
        for (int k = 0; k < kbn; k += 2) {
          const bf16x8 b0 = rb[(size_t)k * 64];
          const bf16x8 b1 = rb[(size_t)(k + 1) * 64];
          const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(ar + 16 * k);
          const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(ar + 16 * k + 16);
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, c, 0, 0, 0);
        }
        osc_accumulate<true>(part, c);
      }
      // Register r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4 of the
      // row block.  Four reduce-scatter steps over lane bits 4..1 leave lane
      // l with value r = (l % 32) / 2 summed over 16 lanes; the exchange
      // with lane l ^ 1 completes the 32 columns.
      float v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = part[r];
#pragma unroll
      for (int m = 16; m >= 2; m >>= 1) {
        const bool upper = (lane & m) != 0;
#pragma unroll
        for (int k = 0; k < m / 2; ++k) {
          const float send = upper ? v[k] : v[k + m / 2];
          const float keep = upper ? v[k + m / 2] : v[k];
          v[k] = keep + __shfl_xor(send, m, 64);
        }
      }
      v[0] += __shfl_xor(v[0], 1, 64);
      if ((lane & 1) == 0) {
        const int r = (lane % 32) >> 1;
        const int row = mb * 32 + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
        fpart[cg * BM + row] = v[0];
      }
    }
    __syncthreads();

    // ---- phase 3.
    for (int rl = tid; rl < nvalid; rl += NT) {
      float f = 0.f;
#pragma unroll
      for (int sl = 0; sl < kSlots; ++sl) f += fpart[sl * BM + rl];
      const int i = tile.row0 + rl;
      const size_t g = (size_t)rn.fit_off + i;
      if (EVAL) {
        fn[g] = f;
        continue;
      }
      const float fx = fc[g];
      const bool accept = f < fx;
      const bool refresh = !accept && b.changed[g] != 0;
      fn[g] = accept ? f : fx;
      b.changed[g] = accept ? 1 : 0;
      act[rl] = accept ? 2 : (refresh ? 1 : 0);
      if (accept) {
        atomicAdd(&b.accepted[tile.run], 1ull);
        atomicMin(&b.best_key[tile.run], fit_key(f, i));
        if (f <= b.target) {
          const unsigned long long old = atomicMin(
              &b.hit_gen[tile.run], (unsigned long long)gen + 1ull);
          if (old == kNoHit) atomicAdd(b.done, 1u);
        }
      }
    }
    if (!EVAL) {
      __syncthreads();
      const int nqd = (rn.D + 3) / 4;
      for (int it = tid; it < nvalid * nqd; it += NT) {
        const int rl = it / nqd, q = it - rl * nqd;
        const int action = act[rl];
        if (action == 0) continue;
        const int i = tile.row0 + rl, j0 = 4 * q;
        const float4 xv = ld4(base + (size_t)i * rn.ldx + j0);
        float4 out = xv;
        if (action == 2) {
          const float4 a1 = ld4(base + (size_t)donors[rl * 4 + 0] * rn.ldx + j0);
          const float4 a2 = ld4(base + (size_t)donors[rl * 4 + 1] * rn.ldx + j0);
          const float4 a3 = ld4(base + (size_t)donors[rl * 4 + 2] * rn.ldx + j0);
          const uint32_t bits = xbits[rl * nq4 + q];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float mv = mutant_coord(get(a1, c), get(a2, c), get(a3, c),
                                          rn.F, b.lo, b.hi);
            set(out, c, ((bits >> c) & 1u) ? mv : get(xv, c));
          }
        }
        st4(pn + rn.pop_off + (size_t)i * rn.ldx + j0, out);
      }
    }
    __syncthreads();  // the next tile reuses the LDS
  }
}

// Wide variant: the per-problem BF16 tile with the run's own arguments, one
// workgroup per tile (its tiles are long enough that the dispatcher's order
// balances them; a tile loop here would keep lane addresses live across
// tiles and spill).  NT follows the padded width as in the per-problem
// kernel (two 512-thread workgroups per CU up to 512, else one of 1024), so
// the results equal a per-problem handle's bit for bit.
template <bool EVAL, int NT>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(NT < 1024 ? 4 : 1)))
void k_bt_wide(BatchArgs b) {
  const long long gen = batch_gen(b);
  const int par = (int)(gen & 1);
  {
    const int t = (int)blockIdx.x;
    if (t >= b.ntiles) return;
    const BTile tile = b.tiles[t];
    const BRun rn = b.runs[tile.run];
    const BInst in = b.inst[rn.inst];
    GenArgs a{};
    a.pop_cur = b.pop[par] + rn.pop_off;
    a.pop_next = b.pop[par ^ 1] + rn.pop_off;
    a.fit_cur = b.fit[par] + rn.fit_off;
    a.fit_next = (EVAL ? b.fit[par] : b.fit[par ^ 1]) + rn.fit_off;
    a.o = in.o;
    a.rop = in.rop_w;
    a.best_key = b.best_key + tile.run;
    a.hit_gen = b.hit_gen + tile.run;
    a.accepted = b.accepted + tile.run;
    a.done = b.done;
    a.changed = b.changed + rn.fit_off;
    a.runs = 1;
    a.NP = rn.NP;
    a.D = rn.D;
    a.ldx = rn.ldx;
    a.dpad = in.dpad_w;
    a.nrows = rn.NP;
    a.F = rn.F;
    a.lo = b.lo;
    a.hi = b.hi;
    a.target = b.target;
    a.cr_threshold = rn.cr_threshold;
    a.gen = (uint32_t)gen;
    a.key_lo = b.key_lo;
    a.key_hi = b.key_hi;
    a.run_base = (uint32_t)tile.run;
    rot_tile<PrecBF16, 64, NT, EVAL>(
        a, 0, tile.row0, min(64, rn.NP - tile.row0));
  }
}

// Initial population of every run (as k_init, run number = batch index).
__global__ __launch_bounds__(256) void k_bt_init(BatchArgs b, int nruns) {
  for (int r = (int)blockIdx.y; r < nruns; r += (int)gridDim.y) {
    const BRun rn = b.runs[r];
    const int nq = (rn.D + 3) / 4;
    const int total = rn.NP * nq;
    for (int t = (int)(blockIdx.x * 256 + threadIdx.x); t < total;
         t += (int)(gridDim.x * 256)) {
      const int i = t / nq, q = t - i * nq;
      const Words4 w = draw_block(kTagInit, (uint32_t)r, 0u, (uint32_t)i,
                                  (uint32_t)q, b.key_lo, b.key_hi);
      const float span = b.hi - b.lo;
      float4 v;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float u = (float)(w.w[c] >> 8) * 0x1.0p-24f;
        set(v, c, fmaf(u, span, b.lo));
      }
      float* p = b.pop[0] + rn.pop_off + (size_t)i * rn.ldx + 4 * q;
      if (4 * q + 4 <= rn.D) {
        st4(p, v);
      } else {
        for (int c = 0; 4 * q + c < rn.D; ++c) p[c] = get(v, c);
      }
    }
  }
}

// Statistics restart: no best, no hit, no acceptance, every row stale.
__global__ __launch_bounds__(256) void k_bt_reset(BatchArgs b, int nruns,
                                                  int nrows) {
  const int stride = (int)(gridDim.x * 256);
  for (int r = (int)(blockIdx.x * 256 + threadIdx.x); r < nruns; r += stride) {
    b.best_key[r] = ~0ull;
    b.hit_gen[r] = kNoHit;
    b.accepted[r] = 0ull;
  }
  for (int k = (int)(blockIdx.x * 256 + threadIdx.x); k < nrows; k += stride)
    b.changed[k] = 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) *b.done = 0u;
}

// best_key[r] = min_i key(fit[r][i], i) over the current generation.
__global__ __launch_bounds__(256) void k_bt_best(BatchArgs b, int nruns) {
  const long long gen = batch_gen(b);
  const float* fit = b.fit[gen & 1];
  for (int r = (int)blockIdx.x; r < nruns; r += (int)gridDim.x) {
    const BRun rn = b.runs[r];
    unsigned long long best = ~0ull;
    for (int i = (int)threadIdx.x; i < rn.NP; i += 256)
      best = min(best, fit_key(fit[rn.fit_off + i], i));
    for (int m = 32; m >= 1; m >>= 1) {
      const unsigned long long o =
          ((unsigned long long)__shfl_xor((unsigned)(best >> 32), m, 64)
           << 32) |
          (unsigned long long)__shfl_xor((unsigned)best, m, 64);
      best = min(best, o);
    }
    if ((threadIdx.x % 64) == 0) atomicMin(&b.best_key[r], best);
  }
}

__global__ void k_bt_set_gen(long long* gen_dev, long long gen) {
  *gen_dev = gen;
}

}  // namespace de

// ---------------------------------------------------------------------------
// Host side.

namespace {

using de::BatchArgs;
using de::BInst;
using de::BRun;
using de::BTile;

constexpr uint64_t kBatchMagic = 0x6465626174636821ull;
constexpr int kMaxGraphGens = 1024;
constexpr int kTuneRepeats = 3;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int dpad_generic(int D) { return (int)round_up((size_t)D, 32); }
int dpad_wide(int D) { return (int)round_up((size_t)D, 128); }

// Kernels of a variant: tile rows, threads, generation and evaluation form.
struct Kern {
  int bm, nt;
  const void* gen_fn;
  const void* eval_fn;
};

int variant_bm(int v) { return v == DE_BATCH_TILE32 ? 32 : 64; }

const Kern& tile_kernel(int v) {
  static const Kern kTile64 = {
      64, 256, reinterpret_cast<const void*>(&de::k_bt_rot<64, 256, false>),
      reinterpret_cast<const void*>(&de::k_bt_rot<64, 256, true>)};
  static const Kern kTile32 = {
      32, 256, reinterpret_cast<const void*>(&de::k_bt_rot<32, 256, false>),
      reinterpret_cast<const void*>(&de::k_bt_rot<32, 256, true>)};
  return v == DE_BATCH_TILE32 ? kTile32 : kTile64;
}

// The wide variant's kernel for a launch over ntiles tiles whose padded
// widths are at most dpad_max: 512 threads (two workgroups per CU) when
// two tiles fit in LDS and there are more tiles than CUs, else 1024.
const Kern& wide_kernel(int dpad_max, size_t ntiles, int cus) {
  static const Kern kNarrow = {
      64, de::kRotBf16ThreadsNarrow,
      reinterpret_cast<const void*>(
          &de::k_bt_wide<false, de::kRotBf16ThreadsNarrow>),
      reinterpret_cast<const void*>(
          &de::k_bt_wide<true, de::kRotBf16ThreadsNarrow>)};
  static const Kern kFull = {
      64, de::kRotBf16Threads,
      reinterpret_cast<const void*>(&de::k_bt_wide<false, de::kRotBf16Threads>),
      reinterpret_cast<const void*>(&de::k_bt_wide<true, de::kRotBf16Threads>)};
  return de::rot_bf16_narrow(dpad_max, (long long)ntiles, cus) ? kNarrow
                                                               : kFull;
}

size_t variant_lds(int v, int D) {
  switch (v) {
    case DE_BATCH_TILE64: return de::bt_lds_bytes<64, 256>(dpad_generic(D));
    case DE_BATCH_TILE32: return de::bt_lds_bytes<32, 256>(dpad_generic(D));
    default: return de::rot_lds_bytes<de::PrecBF16, 64>(dpad_wide(D));
  }
}

bool variant_fits(int v, int D) {
  return variant_lds(v, D) <= (size_t)de::kMaxLdsBytes;
}

// Workspace layout (byte offsets, each 256-aligned).
struct BLayout {
  size_t gen, best, hit, acc, done, changed, runs, inst, tiles, opad, rop,
      total;
  size_t max_tiles;
  std::vector<size_t> opad_at, ropg_at, ropw_at;
};

struct Sizes {
  std::vector<int64_t> pop_off, fit_off;
  std::vector<int32_t> ldx, run_inst;
  size_t pop_floats = 0, fit_floats = 0;
  BLayout L;
};

bool aligned(const void* p, size_t a) {
  return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

// Parameter checks and every size; no device access.
de_status plan_sizes(const de_batch_params* p, Sizes* out) {
  if (!p || !p->runs || !p->inst) return DE_E_INVAL;
  if (p->nruns < 1 || p->nruns >= (1 << 24)) return DE_E_INVAL;
  if (p->ninst < 1 || p->ninst > 4096) return DE_E_INVAL;
  if (!std::isfinite(p->lo) || !std::isfinite(p->hi) || !(p->lo < p->hi) ||
      !std::isfinite(p->hi - p->lo))
    return DE_E_INVAL;
  if (p->graph_gens < 1 || p->graph_gens > kMaxGraphGens) return DE_E_INVAL;
  if (std::isnan(p->target)) return DE_E_INVAL;
  if (p->gemm_prec != de::kPrecBF16) {
    return p->gemm_prec == de::kPrecF32 ? DE_E_UNSUPPORTED : DE_E_INVAL;
  }
  std::vector<int> dims(p->ninst);
  for (int k = 0; k < p->ninst; ++k) {
    const de_batch_instance& in = p->inst[k];
    if (in.D < 1 || in.ldr < in.D) return DE_E_INVAL;
    if (!in.o || !in.R || !aligned(in.o, 4) || !aligned(in.R, 4))
      return DE_E_INVAL;
    for (int j = 0; j < k; ++j)
      if (dims[j] == in.D) return DE_E_INVAL;
    dims[k] = in.D;
    if (!variant_fits(DE_BATCH_TILE64, in.D) &&
        !variant_fits(DE_BATCH_TILE32, in.D) &&
        !variant_fits(DE_BATCH_WIDE, in.D))
      return DE_E_UNSUPPORTED;
  }
  Sizes s;
  s.pop_off.resize(p->nruns);
  s.fit_off.resize(p->nruns);
  s.ldx.resize(p->nruns);
  s.run_inst.resize(p->nruns);
  size_t pop = 0, fit = 0, tiles = 0;
  for (int r = 0; r < p->nruns; ++r) {
    const de_run_spec& rs = p->runs[r];
    if (rs.NP < 4 || rs.NP > (1 << 24) || rs.D < 1) return DE_E_INVAL;
    if (!std::isfinite(rs.F) || !(rs.F > 0.f)) return DE_E_INVAL;
    if (!(rs.CR >= 0.f && rs.CR <= 1.f)) return DE_E_INVAL;
    int k = 0;
    while (k < p->ninst && dims[k] != rs.D) ++k;
    if (k == p->ninst) return DE_E_INVAL;
    s.run_inst[r] = k;
    s.ldx[r] = (int32_t)round_up((size_t)rs.D, 4);
    s.pop_off[r] = (int64_t)pop;
    s.fit_off[r] = (int64_t)fit;
    pop = round_up(pop + (size_t)rs.NP * s.ldx[r], 64);
    fit += (size_t)rs.NP;
    tiles += (size_t)(rs.NP + 31) / 32;
  }
  if (fit > (size_t)std::numeric_limits<int32_t>::max()) return DE_E_INVAL;
  s.pop_floats = pop;
  s.fit_floats = fit;
  BLayout& L = s.L;
  size_t off = 0;
  auto take = [&off](size_t bytes) {
    const size_t at = off;
    off = round_up(off + bytes, 256);
    return at;
  };
  const size_t nr = (size_t)p->nruns;
  L.gen = take(8);
  L.best = take(8 * nr);
  L.hit = take(8 * nr);
  L.acc = take(8 * nr);
  L.done = take(4);
  L.changed = take(fit);
  L.runs = take(sizeof(BRun) * nr);
  L.inst = take(sizeof(BInst) * (size_t)p->ninst);
  L.max_tiles = tiles;
  // one list per variant plus one for the tuner
  L.tiles = take(sizeof(BTile) * tiles * (DE_BATCH_NVARIANTS + 1));
  L.opad_at.resize(p->ninst);
  L.ropg_at.resize(p->ninst);
  L.ropw_at.resize(p->ninst);
  for (int k = 0; k < p->ninst; ++k) {
    const size_t dg = (size_t)dpad_generic(dims[k]);
    const size_t dw = (size_t)dpad_wide(dims[k]);
    L.opad_at[k] = take(4 * dw);
    L.ropg_at[k] = take(2 * dg * dg);
    L.ropw_at[k] = dw == dg ? L.ropg_at[k] : take(2 * dw * dw);
  }
  L.total = off;
  *out = std::move(s);
  return DE_OK;
}

de_status from_hip(hipError_t e) {
  return e == hipSuccess ? DE_OK : DE_E_DEVICE;
}
#define FROM_HIP(expr) from_hip(DE_NOTE(expr))

}  // namespace

struct de_batch {
  uint64_t magic = kBatchMagic;
  int nruns = 0, ninst = 0, graph_gens = 1;
  std::vector<de_run_spec> runs;
  std::vector<int> inst_D;
  Sizes S;
  float* pop[2] = {nullptr, nullptr};
  float* fit[2] = {nullptr, nullptr};
  char* work = nullptr;
  float lo = 0.f, hi = 0.f, target = 0.f;
  uint32_t key_lo = 0, key_hi = 0;
  int64_t gen = 0;
  std::vector<int32_t> plan;
  std::vector<float> tuned_us;
  int cus = 0;
  // one launch per variant in use
  struct Launch {
    int v, ntiles, grid;
    const Kern* k;
    size_t lds;
    const BTile* tiles;
  };
  std::vector<Launch> launches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<BatchArgs> graph_args;
};

namespace {

std::mutex g_live_mu;
std::set<const de_batch*>& live_set() {
  static std::set<const de_batch*> s;
  return s;
}

bool live(const de_batch* b) {
  if (!b) return false;
  std::lock_guard<std::mutex> lk(g_live_mu);
  return live_set().count(b) != 0 && b->magic == kBatchMagic;
}

BatchArgs base_args(const de_batch* b) {
  BatchArgs a{};
  char* w = b->work;
  const BLayout& L = b->S.L;
  a.pop[0] = b->pop[0];
  a.pop[1] = b->pop[1];
  a.fit[0] = b->fit[0];
  a.fit[1] = b->fit[1];
  a.changed = reinterpret_cast<unsigned char*>(w + L.changed);
  a.best_key = reinterpret_cast<unsigned long long*>(w + L.best);
  a.hit_gen = reinterpret_cast<unsigned long long*>(w + L.hit);
  a.accepted = reinterpret_cast<unsigned long long*>(w + L.acc);
  a.done = reinterpret_cast<unsigned int*>(w + L.done);
  a.runs = reinterpret_cast<const BRun*>(w + L.runs);
  a.inst = reinterpret_cast<const BInst*>(w + L.inst);
  a.gen_dev = nullptr;
  a.gen_add = b->gen;
  a.lo = b->lo;
  a.hi = b->hi;
  a.target = b->target;
  a.key_lo = b->key_lo;
  a.key_hi = b->key_hi;
  return a;
}

// Tiles of the runs whose instance is in `insts`, heaviest first (cost per
// tile from `tile_cost` of the instance), runs in order within a cost.
std::vector<BTile> tiles_for(const de_batch* b, const std::vector<int>& insts,
                             int bm, const std::vector<double>& tile_cost) {
  std::vector<BTile> t;
  for (int r = 0; r < b->nruns; ++r) {
    const int k = b->S.run_inst[r];
    if (std::find(insts.begin(), insts.end(), k) == insts.end()) continue;
    for (int row0 = 0; row0 < b->runs[r].NP; row0 += bm) t.push_back({r, row0});
  }
  std::stable_sort(t.begin(), t.end(), [&](const BTile& x, const BTile& y) {
    return tile_cost[b->S.run_inst[x.run]] > tile_cost[b->S.run_inst[y.run]];
  });
  return t;
}

hipError_t launch_variant(const Kern& k, bool eval, BatchArgs a, int ntiles,
                          int grid, size_t lds, const BTile* tiles,
                          hipStream_t st) {
  a.tiles = tiles;
  a.ntiles = ntiles;
  void* args[] = {&a};
  return hipLaunchKernel(eval ? k.eval_fn : k.gen_fn, dim3(grid), dim3(k.nt),
                         args, lds, st);
}

// Workgroups of a launch over ntiles tiles: the generic variants walk the
// tiles with as many workgroups as fit on the device at once; the wide
// variant takes one workgroup per tile.
int persistent_grid(const de_batch* b, int v, const Kern& k, size_t lds,
                    int ntiles) {
  if (v == DE_BATCH_WIDE) return std::max(1, ntiles);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k.gen_fn, k.nt,
                                                   lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const long long cap = (long long)per_cu * b->cus;
  return (int)std::max(1ll, std::min<long long>(cap, ntiles));
}

// Instances whose variant in vk is v, in launch groups: the wide variant
// keeps padded widths up to 512 (which may run two workgroups per CU) apart
// from wider ones; every other variant is one group.
std::vector<std::vector<int>> launch_groups(const de_batch* b,
                                            const std::vector<int>& vk,
                                            int v) {
  std::vector<int> narrow, rest;
  for (int k = 0; k < b->ninst; ++k) {
    if (vk[k] != v) continue;
    const bool small = v == DE_BATCH_WIDE &&
                       dpad_wide(b->inst_D[k]) <= de::kRotBf16NarrowMaxDpad;
    (small ? narrow : rest).push_back(k);
  }
  std::vector<std::vector<int>> g;
  if (!narrow.empty()) g.push_back(narrow);
  if (!rest.empty()) g.push_back(rest);
  return g;
}

// The kernel of a launch of variant v over instances ks and ntiles tiles.
const Kern& group_kernel(const de_batch* b, int v, const std::vector<int>& ks,
                         size_t ntiles) {
  if (v != DE_BATCH_WIDE) return tile_kernel(v);
  int dmax = 0;
  for (int k : ks) dmax = std::max(dmax, dpad_wide(b->inst_D[k]));
  return wide_kernel(dmax, ntiles, b->cus);
}

// Builds the launches of the current plan (tile lists in the workspace).
de_status build_launches(de_batch* b, hipStream_t st,
                         const std::vector<double>& tile_cost) {
  b->launches.clear();
  BTile* dev_tiles = reinterpret_cast<BTile*>(b->work + b->S.L.tiles);
  // host lists stay alive until the copies have completed
  std::vector<std::vector<BTile>> lists;
  const std::vector<int>& vk = b->plan;
  for (int v = 0; v < DE_BATCH_NVARIANTS; ++v) {
    // one launch per group (the wide variant may need two block sizes);
    // their tile lists follow each other in v's region
    size_t off = 0;
    for (const std::vector<int>& insts : launch_groups(b, vk, v)) {
      size_t lds = 0;
      for (int k : insts) lds = std::max(lds, variant_lds(v, b->inst_D[k]));
      lists.push_back(tiles_for(b, insts, variant_bm(v), tile_cost));
      const std::vector<BTile>& t = lists.back();
      if (t.empty()) continue;
      BTile* at = dev_tiles + (size_t)v * b->S.L.max_tiles + off;
      off += t.size();
      de_status rc = FROM_HIP(hipMemcpyAsync(
          at, t.data(), t.size() * sizeof(BTile), hipMemcpyHostToDevice, st));
      if (rc != DE_OK) return rc;
      de_batch::Launch l;
      l.v = v;
      l.k = &group_kernel(b, v, insts, t.size());
      l.ntiles = (int)t.size();
      l.lds = lds;
      l.grid = persistent_grid(b, v, *l.k, lds, l.ntiles);
      l.tiles = at;
      b->launches.push_back(l);
    }
  }
  return FROM_HIP(hipStreamSynchronize(st));
}

de_status destroy_graph(de_batch* b) {
  hipError_t e = hipSuccess;
  if (b->exec) e = hipGraphExecDestroy(b->exec);
  if (b->graph) {
    const hipError_t e2 = hipGraphDestroy(b->graph);
    if (e == hipSuccess) e = e2;
  }
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_args.clear();
  return FROM_HIP(e);
}

// graph_gens generations: per variant a chain of kernel nodes (variants are
// independent branches: runs never read each other's rows).
de_status build_graph(de_batch* b) {
  const int G = b->graph_gens;
  hipGraph_t g = nullptr;
  if (DE_NOTE(hipGraphCreate(&g, 0)) != hipSuccess) return DE_E_DEVICE;
  b->graph = g;
  const BatchArgs base = base_args(b);
  long long* gen_dev = reinterpret_cast<long long*>(b->work + b->S.L.gen);
  b->graph_args.assign((size_t)G * b->launches.size(), base);
  std::vector<hipGraphNode_t> prev(b->launches.size(), nullptr);
  for (int k = 0; k < G; ++k) {
    for (size_t li = 0; li < b->launches.size(); ++li) {
      const de_batch::Launch& l = b->launches[li];
      BatchArgs& a = b->graph_args[(size_t)k * b->launches.size() + li];
      a.gen_dev = gen_dev;
      a.gen_add = k;
      a.tiles = l.tiles;
      a.ntiles = l.ntiles;
      void* args[] = {&a};
      hipKernelNodeParams kp{};
      kp.func = const_cast<void*>(l.k->gen_fn);
      kp.gridDim = dim3(l.grid);
      kp.blockDim = dim3(l.k->nt);
      kp.sharedMemBytes = (unsigned)l.lds;
      kp.kernelParams = args;
      kp.extra = nullptr;
      hipGraphNode_t node = nullptr;
      if (hipGraphAddKernelNode(&node, g, prev[li] ? &prev[li] : nullptr,
                                prev[li] ? 1 : 0, &kp) != hipSuccess) {
        destroy_graph(b);
        return DE_E_DEVICE;
      }
      prev[li] = node;
    }
  }
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    destroy_graph(b);
    return DE_E_DEVICE;
  }
  return DE_OK;
}

de_status direct_generation(de_batch* b, hipStream_t st) {
  BatchArgs a = base_args(b);
  for (const de_batch::Launch& l : b->launches) {
    const de_status rc = FROM_HIP(launch_variant(*l.k, false, a, l.ntiles,
                                                 l.grid, l.lds, l.tiles, st));
    if (rc != DE_OK) return rc;
  }
  b->gen += 1;
  return DE_OK;
}

// Statistics restart and best of the current generation.
de_status reset_and_best(de_batch* b, hipStream_t st) {
  const BatchArgs a = base_args(b);
  const int nrows = (int)b->S.fit_floats;
  const int grid = (int)std::min<size_t>(
      1024, std::max<size_t>(1, (std::max<size_t>(nrows, b->nruns) + 255) / 256));
  hipLaunchKernelGGL(de::k_bt_reset, dim3(grid), dim3(256), 0, st, a,
                     b->nruns, nrows);
  de_status rc = FROM_HIP(hipGetLastError());
  if (rc != DE_OK) return rc;
  hipLaunchKernelGGL(de::k_bt_best, dim3(std::min(b->nruns, 65535)),
                     dim3(256), 0, st, a, b->nruns);
  return FROM_HIP(hipGetLastError());
}

// Times generation 0 of instance k's runs under variant v (microseconds per
// generation); the writes go to generation 1's buffers and are discarded.
de_status time_variant(de_batch* b, int k, int v, hipStream_t st, float* us) {
  const std::vector<double> flat(b->ninst, 0.0);
  const std::vector<BTile> t = tiles_for(b, {k}, variant_bm(v), flat);
  if (t.empty()) {
    *us = 0.f;
    return DE_OK;
  }
  BTile* at = reinterpret_cast<BTile*>(b->work + b->S.L.tiles) +
              (size_t)DE_BATCH_NVARIANTS * b->S.L.max_tiles;
  de_status rc = FROM_HIP(hipMemcpyAsync(at, t.data(), t.size() * sizeof(BTile),
                                         hipMemcpyHostToDevice, st));
  if (rc != DE_OK) return rc;
  const Kern& kern = group_kernel(b, v, {k}, t.size());
  const size_t lds = variant_lds(v, b->inst_D[k]);
  const int grid = persistent_grid(b, v, kern, lds, (int)t.size());
  const BatchArgs a = base_args(b);
  rc = FROM_HIP(launch_variant(kern, false, a, (int)t.size(), grid, lds, at, st));
  if (rc != DE_OK) return rc;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return DE_E_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DE_E_DEVICE;
  }
  rc = FROM_HIP(hipEventRecord(e0, st));
  for (int rep = 0; rep < kTuneRepeats && rc == DE_OK; ++rep)
    rc = FROM_HIP(launch_variant(kern, false, a, (int)t.size(), grid, lds, at, st));
  if (rc == DE_OK) rc = FROM_HIP(hipEventRecord(e1, st));
  if (rc == DE_OK) rc = FROM_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  if (rc == DE_OK) rc = FROM_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *us = ms * 1000.f / kTuneRepeats;
  return rc;
}

// f of generation 0 with TILE64 wherever it fits (input of the tuner).
de_status eval_default(de_batch* b, hipStream_t st) {
  std::vector<int> eval_v(b->ninst);
  for (int k = 0; k < b->ninst; ++k) {
    int v = DE_BATCH_TILE64;
    while (!variant_fits(v, b->inst_D[k])) ++v;
    eval_v[k] = v;
  }
  const std::vector<double> flat(b->ninst, 0.0);
  BTile* scratch = reinterpret_cast<BTile*>(b->work + b->S.L.tiles) +
                   (size_t)DE_BATCH_NVARIANTS * b->S.L.max_tiles;
  const BatchArgs a = base_args(b);
  de_status rc = DE_OK;
  for (int v = 0; v < DE_BATCH_NVARIANTS && rc == DE_OK; ++v) {
    for (const std::vector<int>& ks : launch_groups(b, eval_v, v)) {
      if (rc != DE_OK) break;
      size_t lds = 0;
      for (int k : ks) lds = std::max(lds, variant_lds(v, b->inst_D[k]));
      const std::vector<BTile> t = tiles_for(b, ks, variant_bm(v), flat);
      if (t.empty()) continue;
      const Kern& kern = group_kernel(b, v, ks, t.size());
      rc = FROM_HIP(hipMemcpyAsync(scratch, t.data(),
                                   t.size() * sizeof(BTile),
                                   hipMemcpyHostToDevice, st));
      if (rc == DE_OK)
        rc = FROM_HIP(launch_variant(kern, true, a, (int)t.size(),
                                     persistent_grid(b, v, kern, lds,
                                                     (int)t.size()),
                                     lds, scratch, st));
      // the scratch list is rewritten by the next launch: wait
      if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
    }
  }
  return rc;
}

// f of the current generation with the plan's launches.
de_status eval_with_launches(de_batch* b, hipStream_t st) {
  const BatchArgs a = base_args(b);
  for (const de_batch::Launch& l : b->launches) {
    const de_status rc = FROM_HIP(launch_variant(*l.k, true, a, l.ntiles,
                                                 l.grid, l.lds, l.tiles, st));
    if (rc != DE_OK) return rc;
  }
  return DE_OK;
}

}  // namespace

extern "C" {

DE_API de_status de_batch_layout(const de_batch_params* params,
                                 int64_t* pop_off, int32_t* ldx,
                                 int64_t* fit_off, size_t* pop_floats,
                                 size_t* fit_floats, size_t* work_bytes) {
  Sizes s;
  const de_status rc = plan_sizes(params, &s);
  if (rc != DE_OK) return rc;
  const size_t n = (size_t)params->nruns;
  if (pop_off) std::memcpy(pop_off, s.pop_off.data(), 8 * n);
  if (ldx) std::memcpy(ldx, s.ldx.data(), 4 * n);
  if (fit_off) std::memcpy(fit_off, s.fit_off.data(), 8 * n);
  if (pop_floats) *pop_floats = s.pop_floats;
  if (fit_floats) *fit_floats = s.fit_floats;
  if (work_bytes) *work_bytes = s.L.total;
  return DE_OK;
}

DE_API de_status de_batch_create(const de_batch_params* params, float* pop0,
                                 float* pop1, float* fit0, float* fit1,
                                 void* work, size_t work_bytes,
                                 const int32_t* plan, void* hip_stream,
                                 de_batch** out) {
  if (!out) return DE_E_INVAL;
  *out = nullptr;
  Sizes s;
  de_status rc = plan_sizes(params, &s);
  if (rc != DE_OK) return rc;
  const de_batch_params& p = *params;
  if (!pop0 || !pop1 || !fit0 || !fit1 || !work) return DE_E_INVAL;
  if (!aligned(pop0, 16) || !aligned(pop1, 16) || !aligned(fit0, 16) ||
      !aligned(fit1, 16) || !aligned(work, 256))
    return DE_E_INVAL;
  if (work_bytes < s.L.total) return DE_E_INVAL;
  if (plan) {
    for (int k = 0; k < p.ninst; ++k) {
      if (plan[k] < DE_BATCH_AUTO || plan[k] >= DE_BATCH_NVARIANTS)
        return DE_E_INVAL;
      if (plan[k] != DE_BATCH_AUTO && !variant_fits(plan[k], p.inst[k].D))
        return DE_E_UNSUPPORTED;
    }
  }
  de_batch* b = new (std::nothrow) de_batch();
  if (!b) return DE_E_NOMEM;
  b->nruns = p.nruns;
  b->ninst = p.ninst;
  b->graph_gens = p.graph_gens;
  b->runs.assign(p.runs, p.runs + p.nruns);
  b->inst_D.resize(p.ninst);
  for (int k = 0; k < p.ninst; ++k) b->inst_D[k] = p.inst[k].D;
  b->S = std::move(s);
  b->pop[0] = pop0;
  b->pop[1] = pop1;
  b->fit[0] = fit0;
  b->fit[1] = fit1;
  b->work = static_cast<char*>(work);
  b->lo = p.lo;
  b->hi = p.hi;
  {
    // largest float <= target, so that f <= target in float is exact
    double t = p.target;
    float f = std::isinf(t) ? (float)t
              : t >= (double)std::numeric_limits<float>::max()
                  ? std::numeric_limits<float>::max()
              : t <= -(double)std::numeric_limits<float>::max()
                  ? -std::numeric_limits<float>::infinity()
                  : (float)t;
    if (std::isfinite(f) && (double)f > t)
      f = std::nextafter(f, -std::numeric_limits<float>::infinity());
    b->target = f;
  }
  b->key_lo = (uint32_t)p.seed;
  b->key_hi = (uint32_t)(p.seed >> 32);
  b->plan.assign(p.ninst, DE_BATCH_AUTO);
  b->tuned_us.assign((size_t)p.ninst * DE_BATCH_NVARIANTS, -1.f);
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  (void)hipGetLastError();

  auto fail = [&](de_status e) {
    delete b;
    return e;
  };
  int dev = 0;
  hipDeviceProp_t prop;
  if (DE_NOTE(hipGetDevice(&dev)) != hipSuccess ||
      DE_NOTE(hipGetDeviceProperties(&prop, dev)) != hipSuccess)
    return fail(DE_E_DEVICE);
  b->cus = prop.multiProcessorCount;
  {
    // every kernel of every variant (the wide one at both block sizes)
    const Kern* ks[] = {&tile_kernel(DE_BATCH_TILE64),
                        &tile_kernel(DE_BATCH_TILE32),
                        &wide_kernel(de::kRotBf16NarrowMaxDpad, 1, 0),
                        &wide_kernel(de::kRotBf16NarrowMaxDpad + 1, 1, 0)};
    for (const Kern* k : ks)
      if (DE_NOTE(de::set_max_dynamic_lds(k->gen_fn)) != hipSuccess ||
          DE_NOTE(de::set_max_dynamic_lds(k->eval_fn)) != hipSuccess)
        return fail(DE_E_DEVICE);
  }

  // tables and instance data
  const BLayout& L = b->S.L;
  std::vector<BRun> runs(p.nruns);
  for (int r = 0; r < p.nruns; ++r) {
    BRun& x = runs[r];
    x = BRun{};
    x.pop_off = (unsigned long long)b->S.pop_off[r];
    x.fit_off = (int)b->S.fit_off[r];
    x.NP = p.runs[r].NP;
    x.D = p.runs[r].D;
    x.ldx = b->S.ldx[r];
    x.inst = b->S.run_inst[r];
    x.F = p.runs[r].F;
    x.cr_threshold = (uint32_t)std::floor((double)p.runs[r].CR * 16777216.0);
  }
  std::vector<BInst> insts(p.ninst);
  for (int k = 0; k < p.ninst; ++k) {
    const int D = p.inst[k].D;
    BInst& x = insts[k];
    x = BInst{};
    x.o = reinterpret_cast<const float*>(b->work + L.opad_at[k]);
    x.rop_g = reinterpret_cast<const __bf16*>(b->work + L.ropg_at[k]);
    x.rop_w = reinterpret_cast<const __bf16*>(b->work + L.ropw_at[k]);
    x.D = D;
    x.dpad_g = dpad_generic(D);
    x.dpad_w = dpad_wide(D);
  }
  rc = FROM_HIP(hipMemcpyAsync(b->work + L.runs, runs.data(),
                               sizeof(BRun) * runs.size(),
                               hipMemcpyHostToDevice, st));
  if (rc == DE_OK)
    rc = FROM_HIP(hipMemcpyAsync(b->work + L.inst, insts.data(),
                                 sizeof(BInst) * insts.size(),
                                 hipMemcpyHostToDevice, st));
  for (int k = 0; k < p.ninst && rc == DE_OK; ++k) {
    const de_batch_instance& in = p.inst[k];
    float* opad = reinterpret_cast<float*>(b->work + L.opad_at[k]);
    rc = FROM_HIP(de::launch_prep(in.o, in.R, in.ldr, in.D, dpad_generic(in.D),
                                  de::kObjRotOsc, de::kPrecBF16, opad,
                                  b->work + L.ropg_at[k], st));
    if (rc == DE_OK && L.ropw_at[k] != L.ropg_at[k])
      rc = FROM_HIP(de::launch_prep(in.o, in.R, in.ldr, in.D, dpad_wide(in.D),
                                    de::kObjRotOsc, de::kPrecBF16, opad,
                                    b->work + L.ropw_at[k], st));
  }
  if (rc != DE_OK) return fail(rc);

  // generation 0
  BatchArgs a = base_args(b);
  {
    const int gy = std::min(p.nruns, 65535);
    hipLaunchKernelGGL(de::k_bt_init, dim3(16, gy), dim3(256), 0, st, a,
                       p.nruns);
    rc = FROM_HIP(hipGetLastError());
  }
  if (rc != DE_OK) return fail(rc);

  // plan: given entries kept, DE_BATCH_AUTO entries tuned on generation 0
  bool tune = false;
  for (int k = 0; k < p.ninst; ++k) {
    b->plan[k] = plan ? plan[k] : DE_BATCH_AUTO;
    tune = tune || b->plan[k] == DE_BATCH_AUTO;
  }
  if (tune) {
    rc = eval_default(b, st);
    if (rc == DE_OK) rc = reset_and_best(b, st);
    for (int k = 0; k < p.ninst && rc == DE_OK; ++k) {
      if (b->plan[k] != DE_BATCH_AUTO) continue;
      float best_us = std::numeric_limits<float>::infinity();
      for (int v = 0; v < DE_BATCH_NVARIANTS && rc == DE_OK; ++v) {
        if (!variant_fits(v, p.inst[k].D)) continue;
        float us = 0.f;
        rc = time_variant(b, k, v, st, &us);
        b->tuned_us[(size_t)k * DE_BATCH_NVARIANTS + v] = us;
        if (rc == DE_OK && us < best_us) {
          best_us = us;
          b->plan[k] = v;
        }
      }
    }
    if (rc != DE_OK) return fail(rc);
  }

  // cost per tile of each instance under its variant, for tile ordering
  std::vector<double> cost(p.ninst, 1.0);
  for (int k = 0; k < p.ninst; ++k) {
    const float us = b->tuned_us[(size_t)k * DE_BATCH_NVARIANTS + b->plan[k]];
    size_t nt = 0;
    for (int r = 0; r < p.nruns; ++r)
      if (b->S.run_inst[r] == k)
        nt += (size_t)(p.runs[r].NP + variant_bm(b->plan[k]) - 1) /
              variant_bm(b->plan[k]);
    // untimed (explicit plan): padded MFMA work per tile as the estimate
    const double d = (double)(b->plan[k] == DE_BATCH_WIDE
                                  ? dpad_wide(p.inst[k].D)
                                  : dpad_generic(p.inst[k].D));
    cost[k] = us >= 0.f && nt > 0 ? (double)us / nt : d * d;
  }
  rc = build_launches(b, st, cost);
  // generation 0's fitness with the plan's own kernels (so every value of a
  // run comes from one summation order), then fresh statistics
  if (rc == DE_OK) rc = eval_with_launches(b, st);
  if (rc == DE_OK) rc = reset_and_best(b, st);
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  if (rc != DE_OK) return fail(rc);
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    live_set().insert(b);
  }
  *out = b;
  return DE_OK;
}

DE_API de_status de_batch_plan(const de_batch* batch, int32_t* plan,
                               float* us_per_gen) {
  if (!live(batch)) return DE_E_STATE;
  if (!plan) return DE_E_INVAL;
  std::memcpy(plan, batch->plan.data(), 4 * batch->plan.size());
  if (us_per_gen)
    std::memcpy(us_per_gen, batch->tuned_us.data(),
                4 * batch->tuned_us.size());
  return DE_OK;
}

DE_API de_status de_batch_generation(de_batch* batch, int64_t n_gens,
                                     void* hip_stream) {
  if (!live(batch)) return DE_E_STATE;
  if (n_gens < 0) return DE_E_INVAL;
  if (batch->gen + n_gens >= ((int64_t)1 << 32)) return DE_E_INVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  (void)hipGetLastError();
  de_status rc = DE_OK;
  const int G = batch->graph_gens;
  long long* gen_dev = reinterpret_cast<long long*>(batch->work +
                                                    batch->S.L.gen);
  while (n_gens >= G && G > 1 && rc == DE_OK) {
    if (!batch->exec) {
      rc = build_graph(batch);
      if (rc != DE_OK) break;
    }
    hipLaunchKernelGGL(de::k_bt_set_gen, dim3(1), dim3(1), 0, st, gen_dev,
                       (long long)batch->gen);
    rc = FROM_HIP(hipGetLastError());
    if (rc == DE_OK) rc = FROM_HIP(hipGraphLaunch(batch->exec, st));
    if (rc == DE_OK) {
      batch->gen += G;
      n_gens -= G;
    }
  }
  for (; n_gens > 0 && rc == DE_OK; --n_gens)
    rc = direct_generation(batch, st);
  return rc;
}

DE_API de_status de_batch_read(de_batch* batch, void* hip_stream,
                               double* best_f, int32_t* best_idx,
                               int64_t* accepted, int64_t* hit_gen) {
  if (!live(batch)) return DE_E_STATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  (void)hipGetLastError();
  const size_t n = (size_t)batch->nruns;
  std::vector<unsigned long long> key(n), acc(n), hit(n);
  const BLayout& L = batch->S.L;
  de_status rc = FROM_HIP(hipMemcpyAsync(key.data(), batch->work + L.best,
                                         8 * n, hipMemcpyDeviceToHost, st));
  if (rc == DE_OK)
    rc = FROM_HIP(hipMemcpyAsync(acc.data(), batch->work + L.acc, 8 * n,
                                 hipMemcpyDeviceToHost, st));
  if (rc == DE_OK)
    rc = FROM_HIP(hipMemcpyAsync(hit.data(), batch->work + L.hit, 8 * n,
                                 hipMemcpyDeviceToHost, st));
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  if (rc != DE_OK) return rc;
  for (size_t r = 0; r < n; ++r) {
    const uint32_t ord = (uint32_t)(key[r] >> 32);
    const uint32_t bits = (ord & 0x80000000u) ? (ord & 0x7FFFFFFFu) : ~ord;
    float f;
    std::memcpy(&f, &bits, 4);
    if (best_f) best_f[r] = (double)f;
    if (best_idx) best_idx[r] = (int32_t)(uint32_t)key[r];
    if (accepted) accepted[r] = (int64_t)acc[r];
    if (hit_gen) hit_gen[r] = hit[r] == ~0ull ? -1 : (int64_t)hit[r];
  }
  return DE_OK;
}

DE_API de_status de_batch_get_generation(const de_batch* batch, int64_t* gen) {
  if (!live(batch)) return DE_E_STATE;
  if (!gen) return DE_E_INVAL;
  *gen = batch->gen;
  return DE_OK;
}

DE_API de_status de_batch_destroy(de_batch* batch) {
  if (!live(batch)) return DE_E_STATE;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    live_set().erase(batch);
  }
  const hipError_t e = hipDeviceSynchronize();
  const de_status rc = destroy_graph(batch);
  batch->magic = 0;
  delete batch;
  if (e != hipSuccess) return DE_E_DEVICE;
  return rc;
}

}  // extern "C"
