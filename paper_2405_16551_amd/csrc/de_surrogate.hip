// de_surrogate.hip -- surrogate-assisted DE/rand/1/bin on a composition
// objective (the C ABI of include/de_surrogate.h).
//
// One generation of every run:
//   k_sur_cand     k DE/rand/1/bin candidates per target (Section 2, eqs. 2
//                  and 3; candidate c draws with individual field i | c<<24)
//   k_mlp_infer_res / k_mlp_infer
//                  the run's MLP D -> H -> H -> 1 on every candidate, BF16
//                  32x32x16 MFMA with FP32 accumulation, bias and ReLU
//                  fused; tiles of 64 candidates (the first form, for D
//                  padded to at most 128, keeps each wave's weight
//                  fragments in registers over four tiles)
//   k_sur_select   per target the lowest prediction is evaluated on the
//                  composition objective (Section 7.3.3 composition
//                  functions; the expensive step), strict selection, next
//                  generation, statistics, archive insert
// then `steps` Adam steps of every run's model (FP32):
//   k_train_fwd    minibatch rows drawn from the archive, forward pass,
//                  output error and both hidden-layer deltas, FP32 16x16x4
//                  MFMA (16 rows per workgroup)
//   k_train_grad   weight gradients as FP32 MFMA products over the
//                  minibatch (one wave per 32x32 block), bias gradients
//                  from eight partial row sums, then the Adam update per
//                  entry, which also refreshes the BF16 fragment copy used
//                  for inference and the FP32 transposed copy used by the
//                  next forward pass (k_model_prep builds both after
//                  initialisation and when the model is set)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <set>
#include <vector>

#include "de.h"
#include "de_device.hpp"
#include "de_internal.h"
#include "de_surrogate.h"
#include "de_tile.hpp"

namespace de {

struct SurArgs {
  // population (generation g -> g+1)
  const float* pop_cur;
  float* pop_next;
  const float* fit_cur;
  float* fit_next;
  int runs, NP, D, ldx, k, H, Dp, pstride;
  float F, lo, hi, xs_mul, xs_add;  // xs = x * xs_mul + xs_add
  uint32_t cr_threshold, gen, key_lo, key_hi;
  // composition
  const float* O;    // [n][D]
  const float* Rt;   // [n][D][D], Rt[c][j][i] = R[c][i][j]
  const float* bias; // [n]
  int n;
  float inv2s2;      // 1 / (2 sigma^2)
  // candidates and predictions
  float* cand;       // [runs][NP*k][ldx]
  float* pred;       // [runs][NP*k]
  int* choice;       // [runs][NP]
  int use_model;
  // model (per run, stride pstride floats)
  float* theta;
  float* m;
  float* v;
  __bf16* w1f;       // [runs][H/32][Dp/16][64][8]
  __bf16* w2f;       // [runs][H/32][H/16][64][8]
  float* w1t;        // [runs][D][H]
  float* w2t;        // [runs][H][H]
  // archive
  float* ax;         // [runs][cap][ldx]
  float* at;         // [runs][cap]
  int cap, round, filled;
  // training
  int B;
  uint32_t step, mkey_lo, mkey_hi;
  float lr, beta1, beta2, eps, c1, c2;
  float* xsb;        // [runs][B][Dp]
  float* h1b;        // [runs][B][H]
  float* h2b;
  float* d1b;
  float* d2b;
  float* eb;         // [runs][B]
  // statistics
  unsigned long long* best_key;
  unsigned long long* accepted;
};

constexpr int kEvalRows = 8;
constexpr int kEvalThreads = 128;
constexpr int kMaxComp = 64;

// ---------------------------------------------------------------------------
// Composition objective of up to kEvalRows rows (pointers in rowp), one
// workgroup of kEvalThreads threads.  Per component: y = x - O[c] into LDS
// with ||y||^2, z = R[c] y with one thread per output coordinate reading
// the transposed rotation (coalesced), g = sum z^2 + sin^2(3z); partial
// sums reduced in a fixed order.  Then the normalised weights.
__device__ void comp_eval_rows(const SurArgs& a, const float* const* rowp,
                               int nv, float* sm, float* fout) {
  const int tid = (int)threadIdx.x, lane = tid % 64, wave = tid / 64;
  constexpr int kWaves = kEvalThreads / 64;
  const int D = a.D;
  float* xs = sm;                          // [rows][D]
  float* ys = xs + kEvalRows * D;          // [rows][D]
  float* dk = ys + kEvalRows * D;          // [n][rows]
  float* gk = dk + kMaxComp * kEvalRows;   // [n][rows]
  float* red = gk + kMaxComp * kEvalRows;  // [2][rows][waves]
  for (int t = tid; t < kEvalRows * D; t += kEvalThreads) {
    const int r = t / D, j = t - r * D;
    xs[t] = r < nv ? rowp[r][j] : 0.f;
  }
  __syncthreads();
  for (int c = 0; c < a.n; ++c) {
    const float* o = a.O + (size_t)c * D;
    const float* rt = a.Rt + (size_t)c * D * D;
    float dpart[kEvalRows], gpart[kEvalRows];
#pragma unroll
    for (int r = 0; r < kEvalRows; ++r) dpart[r] = gpart[r] = 0.f;
    for (int j = tid; j < D; j += kEvalThreads) {
      const float oj = o[j];
#pragma unroll
      for (int r = 0; r < kEvalRows; ++r) {
        const float y = xs[r * D + j] - oj;
        ys[r * D + j] = y;
        dpart[r] = fmaf(y, y, dpart[r]);
      }
    }
    __syncthreads();
    for (int i = tid; i < D; i += kEvalThreads) {
      float z[kEvalRows];
#pragma unroll
      for (int r = 0; r < kEvalRows; ++r) z[r] = 0.f;
      for (int j = 0; j < D; ++j) {
        const float rv = rt[(size_t)j * D + i];
#pragma unroll
        for (int r = 0; r < kEvalRows; ++r) z[r] = fmaf(rv, ys[r * D + j], z[r]);
      }
#pragma unroll
      for (int r = 0; r < kEvalRows; ++r)
        gpart[r] += fmaf(z[r], z[r], sin_squared(3.0f * z[r]));
    }
#pragma unroll
    for (int r = 0; r < kEvalRows; ++r) {
      const float ds = group_sum<64>(dpart[r]);
      const float gs = group_sum<64>(gpart[r]);
      if (lane == 0) {
        red[(0 * kEvalRows + r) * kWaves + wave] = ds;
        red[(1 * kEvalRows + r) * kWaves + wave] = gs;
      }
    }
    __syncthreads();
    if (tid < 2 * kEvalRows) {
      float s = 0.f;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) s += red[tid * kWaves + w];
      const int q = tid / kEvalRows, r = tid % kEvalRows;
      (q == 0 ? dk : gk)[c * kEvalRows + r] = s;
    }
    __syncthreads();
  }
  if (tid < kEvalRows) {
    float dmin = INFINITY;
    for (int c = 0; c < a.n; ++c) dmin = fminf(dmin, dk[c * kEvalRows + tid]);
    float wsum = 0.f, f = 0.f;
    for (int c = 0; c < a.n; ++c) {
      const float w = expf(-(dk[c * kEvalRows + tid] - dmin) * a.inv2s2);
      wsum += w;
      f = fmaf(w, gk[c * kEvalRows + tid] + a.bias[c], f);
    }
    fout[tid] = f / wsum;
  }
  __syncthreads();
}

__host__ __device__ constexpr size_t comp_lds_floats(int D) {
  return (size_t)2 * kEvalRows * D + (size_t)2 * kMaxComp * kEvalRows +
         (size_t)2 * kEvalRows * (kEvalThreads / 64) + kEvalRows;
}

// f of rows X (row r at X + r * ldx).
__global__ __launch_bounds__(kEvalThreads) void k_comp_eval(SurArgs a,
                                                            const float* X,
                                                            int n, int ldx,
                                                            float* f) {
  extern __shared__ __align__(16) float sm[];
  __shared__ const float* rowp[kEvalRows];
  const int row0 = (int)blockIdx.x * kEvalRows;
  const int nv = min(kEvalRows, n - row0);
  if ((int)threadIdx.x < kEvalRows)
    rowp[threadIdx.x] = X + (size_t)(row0 + min((int)threadIdx.x, nv - 1)) * ldx;
  __syncthreads();
  float* fout = sm + comp_lds_floats(a.D) - kEvalRows;
  comp_eval_rows(a, rowp, nv, sm, fout);
  if ((int)threadIdx.x < nv) f[row0 + threadIdx.x] = fout[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Candidates: one wave per candidate row (i, c), or one half-wave when a
// row has at most 32 4-groups; lanes over 4-groups.
__host__ __device__ constexpr int cand_rows_per_wave(int D) {
  return (D + 3) / 4 <= 32 ? 2 : 1;
}

__global__ __launch_bounds__(256) void k_sur_cand(SurArgs a) {
  const int run = (int)blockIdx.y;
  const int wave = (int)threadIdx.x / 64;
  const int rpw = cand_rows_per_wave(a.D), lpr = 64 / rpw;
  const int lane = (int)threadIdx.x % lpr;
  const int cr = ((int)blockIdx.x * 4 + wave) * rpw + ((int)threadIdx.x % 64) / lpr;
  if (cr >= a.NP * a.k) return;  // whole row groups leave together
  const int i = cr / a.k, c = cr - i * a.k;
  const uint32_t ctr_i = (uint32_t)i | ((uint32_t)c << 24);
  const Donors d = pick_donors_ctr((uint32_t)run, a.gen, ctr_i, i, a.NP, a.D,
                                   a.key_lo, a.key_hi);
  const float* base = a.pop_cur + (size_t)run * a.NP * a.ldx;
  const float* x = base + (size_t)i * a.ldx;
  const float* x1 = base + (size_t)d.r1 * a.ldx;
  const float* x2 = base + (size_t)d.r2 * a.ldx;
  const float* x3 = base + (size_t)d.r3 * a.ldx;
  float* out = a.cand + ((size_t)run * a.NP * a.k + cr) * a.ldx;
  // predictions read 0 for a generation the model does not screen
  if (!a.use_model && lane == 0) a.pred[(size_t)run * a.NP * a.k + cr] = 0.f;
  const int nq = (a.D + 3) / 4;
  for (int q = lane; q < nq; q += lpr) {
    const int j0 = 4 * q;
    const float4 xv = ld4(x + j0), v1 = ld4(x1 + j0), v2 = ld4(x2 + j0),
                 v3 = ld4(x3 + j0);
    const Words4 w = draw_block(kTagXover, (uint32_t)run, a.gen, ctr_i,
                                (uint32_t)q, a.key_lo, a.key_hi);
    float4 u = xv;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const bool tk = (j0 + b < a.D) &&
                      take_mutant(w.w[b], j0 + b, d.jrand, a.cr_threshold);
      const float mv = mutant_coord(get(v1, b), get(v2, b), get(v3, b), a.F,
                                    a.lo, a.hi);
      set(u, b, tk ? mv : get(xv, b));
    }
    st4(out + j0, u);
  }
}

// ---------------------------------------------------------------------------
// MLP inference on MFMA: rows of X (row r at X + r * ldx) of run
// run0 + blockIdx.y, kInferRows rows per workgroup of 256 threads.
constexpr int kInferRows = 64;

__host__ __device__ constexpr size_t infer_lds_bytes(int Dp, int H) {
  return (size_t)kInferRows * (Dp + 8) * 2 + (size_t)kInferRows * (H + 8) * 2 +
         (size_t)4 * kInferRows * 4;
}

// Two 32x32 BF16 blocks (row blocks 0 and 1, same columns) over kbn
// K-steps of 16 (kbn even): A fragments from LDS at ar0 / ar1 + 16 kb, B
// fragments at wf[kb * 64], each B fragment used by both row blocks; two
// K-steps per batch, each batch's reads issued one batch ahead.
__device__ __forceinline__ void mfma_bf16_pair(const __bf16* ar0,
                                               const __bf16* ar1,
                                               const bf16x8* wf, int kbn,
                                               floatx16& c0, floatx16& c1) {
  c0 = floatx16{};
  c1 = floatx16{};
  bf16x8 a0n[2], a1n[2], bn[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    a0n[u] = *reinterpret_cast<const bf16x8*>(ar0 + 16 * u);
    a1n[u] = *reinterpret_cast<const bf16x8*>(ar1 + 16 * u);
    bn[u] = wf[(size_t)u * 64];
  }
  for (int kb = 0; kb < kbn; kb += 2) {
    bf16x8 a0[2], a1[2], b[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      a0[u] = a0n[u];
      a1[u] = a1n[u];
      b[u] = bn[u];
    }
    if (kb + 2 < kbn) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        a0n[u] = *reinterpret_cast<const bf16x8*>(ar0 + 16 * (kb + 2 + u));
        a1n[u] = *reinterpret_cast<const bf16x8*>(ar1 + 16 * (kb + 2 + u));
        bn[u] = wf[(size_t)(kb + 2 + u) * 64];
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0[u], b[u], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1[u], b[u], c1, 0, 0, 0);
    }
  }
}

// Sum over the 32 lanes of each half-wave of 16 per-lane row values
// (register r holds row 8 (r / 4) + 4 (l / 32) + r % 4 of a 32-row block):
// four reduce-scatter steps over lane bits 4..1, then lanes l, l ^ 1; lane
// l ends with row r = (l % 32) / 2 in the returned value.
__device__ __forceinline__ float rows_of_block(const floatx16& part,
                                               int lane) {
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
  return v[0] + __shfl_xor(v[0], 1, 64);
}

// MLP inference on MFMA: rows of X (row r at X + r * ldx) of run
// run0 + blockIdx.y, 64 rows per workgroup of 256 threads (4 waves, each
// two 32-column blocks per layer over both 32-row blocks).  Layer 1 writes
// relu(A W1^T + b1) to LDS in BF16; layer 2's epilogue applies relu(. + b2)
// and the output weights w3 directly, so only per-wave row sums remain.
__global__ __launch_bounds__(256) void k_mlp_infer(SurArgs a, const float* X,
                                                   size_t x_run_stride, int n,
                                                   int ldx, float* y,
                                                   size_t y_run_stride,
                                                   int run0) {
  extern __shared__ __align__(16) char smem[];
  const int run = run0 + (int)blockIdx.y;
  const int tid = (int)threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int row0 = (int)blockIdx.x * kInferRows;
  const int Dp = a.Dp, H = a.H;
  const int sa = Dp + 8, sh = H + 8;
  __bf16* A = reinterpret_cast<__bf16*>(smem);
  __bf16* H1 = A + (size_t)kInferRows * sa;
  float* ypart = reinterpret_cast<float*>(H1 + (size_t)kInferRows * sh);
  const float* Xr = X + blockIdx.y * x_run_stride;
  const float* th = a.theta + (size_t)run * a.pstride;
  const float* b1 = th + (size_t)H * a.D;
  const float* b2 = b1 + H + (size_t)H * H;
  const float* w3 = b2 + H;
  const float b3 = w3[H];
  for (int t = tid; t < kInferRows * Dp; t += 256) {
    const int r = t / Dp, dd = t - r * Dp;
    float v = 0.f;
    if (row0 + r < n && dd < a.D)
      v = fmaf(Xr[(size_t)(row0 + r) * ldx + dd], a.xs_mul, a.xs_add);
    A[r * sa + dd] = (__bf16)v;
  }
  __syncthreads();
  const int nblk = H / 32;
  const int li = lane % 32, lk = lane / 32;
  {
    const int kbn = Dp / 16;
    const bf16x8* wf = reinterpret_cast<const bf16x8*>(a.w1f) +
                       (size_t)run * nblk * kbn * 64 + lane;
    const __bf16* ar0 = A + (size_t)li * sa + 8 * lk;
    const __bf16* ar1 = ar0 + (size_t)32 * sa;
    for (int nb = wave; nb < nblk; nb += 4) {
      floatx16 c0, c1;
      mfma_bf16_pair(ar0, ar1, wf + (size_t)nb * kbn * 64, kbn, c0, c1);
      const int col = nb * 32 + li;
      const float bb = b1[col];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r / 4) + 4 * lk + (r % 4);
        H1[row * sh + col] = (__bf16)fmaxf(c0[r] + bb, 0.f);
        H1[(32 + row) * sh + col] = (__bf16)fmaxf(c1[r] + bb, 0.f);
      }
    }
  }
  __syncthreads();
  {
    const int kbn = H / 16;
    const bf16x8* wf = reinterpret_cast<const bf16x8*>(a.w2f) +
                       (size_t)run * nblk * kbn * 64 + lane;
    const __bf16* ar0 = H1 + (size_t)li * sh + 8 * lk;
    const __bf16* ar1 = ar0 + (size_t)32 * sh;
    floatx16 p0 = {}, p1 = {};
    for (int nb = wave; nb < nblk; nb += 4) {
      floatx16 c0, c1;
      mfma_bf16_pair(ar0, ar1, wf + (size_t)nb * kbn * 64, kbn, c0, c1);
      const int col = nb * 32 + li;
      const float bb = b2[col], ww = w3[col];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        p0[r] = fmaf(fmaxf(c0[r] + bb, 0.f), ww, p0[r]);
        p1[r] = fmaf(fmaxf(c1[r] + bb, 0.f), ww, p1[r]);
      }
    }
    const float s0 = rows_of_block(p0, lane);
    const float s1 = rows_of_block(p1, lane);
    if ((lane & 1) == 0) {
      const int r = li >> 1;
      const int row = 8 * (r / 4) + 4 * lk + (r % 4);
      ypart[wave * kInferRows + row] = s0;
      ypart[wave * kInferRows + 32 + row] = s1;
    }
  }
  __syncthreads();
  if (tid < kInferRows && row0 + tid < n) {
    float s = b3;
#pragma unroll
    for (int w = 0; w < 4; ++w) s += ypart[w * kInferRows + tid];
    y[blockIdx.y * y_run_stride + row0 + tid] = s;
  }
}

// rows_of_block with the lane-dependent choices as bit selects on a
// per-lane mask held in a vector register (v_bfi_b32) instead of
// per-step lane masks, which the register-resident kernel has no scalar
// registers left for.  Same exchanges and additions, same result.
__device__ __forceinline__ float bsel(uint32_t m, float a, float b) {
  const uint32_t ia = __builtin_bit_cast(uint32_t, a);
  const uint32_t ib = __builtin_bit_cast(uint32_t, b);
  return __builtin_bit_cast(float, (m & ia) | (~m & ib));  // m ? a : b
}

__device__ __forceinline__ float rows_of_block_vsel(const floatx16& part,
                                                    int lane) {
  float v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = part[r];
#pragma unroll
  for (int m = 16, sh = 4; m >= 2; m >>= 1, --sh) {
    const uint32_t up = 0u - (((uint32_t)lane >> sh) & 1u);  // all ones if set
#pragma unroll
    for (int k = 0; k < m / 2; ++k) {
      const float send = bsel(up, v[k], v[k + m / 2]);
      const float keep = bsel(up, v[k + m / 2], v[k]);
      v[k] = keep + __shfl_xor(send, m, 64);
    }
  }
  return v[0] + __shfl_xor(v[0], 1, 64);
}

// MLP inference with the weights held in registers: one workgroup of
// H / 32 waves per group of row tiles of one run; wave w keeps the BF16
// fragments of column block w of W1 (KB1 = Dp / 16 K-steps) and of W2
// (KB2 = H / 16) for the whole launch, so the K loops read only LDS.  Per
// 64-row tile: the rows go to LDS in BF16 (the next tile's rows are loaded
// into registers meanwhile), layer 1 writes relu(A W1^T + b1) to LDS,
// layer 2's epilogue applies relu(. + b2) and w3 and reduces its 32
// columns per row; the rows' totals add the waves in order, then b3.
// Same operands and per-block K order as k_mlp_infer; the row totals add
// the 32-column blocks in another order (block by block instead of two
// per wave), a difference within FP32 rounding.
constexpr int kResTiles = 4;  // 64-row tiles per workgroup

template <int KB1, int KB2>
__global__ __launch_bounds__(512) void k_mlp_infer_res(SurArgs a, const float* X,
                                                       size_t x_run_stride,
                                                       int n, int ldx, float* y,
                                                       size_t y_run_stride,
                                                       int run0) {
  constexpr int Dp = KB1 * 16, H = KB2 * 16, NW = H / 32;
  constexpr int sa = Dp + 8, sh = H + 8;
  constexpr int kStage = (kInferRows * Dp + 32 * NW * 2 - 1) / (64 * NW);
  extern __shared__ __align__(16) char smem[];
  const int run = run0 + (int)blockIdx.y;
  const int tid = (int)threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int nthr = 64 * NW;
  __bf16* A = reinterpret_cast<__bf16*>(smem);
  __bf16* H1 = A + (size_t)kInferRows * sa;
  float* ypart = reinterpret_cast<float*>(H1 + (size_t)kInferRows * sh);
  const float* Xr = X + blockIdx.y * x_run_stride;
  const float* th = a.theta + (size_t)run * a.pstride;
  const float* b1 = th + (size_t)H * a.D;
  const float* b2 = b1 + H + (size_t)H * H;
  const float* w3 = b2 + H;
  const float b3 = w3[H];
  const int li = lane % 32, lk = lane / 32;
  const int col = wave * 32 + li;
  const float b1c = b1[col], b2c = b2[col], w3c = w3[col];
  bf16x8 w1r[KB1], w2r[KB2];
  {
    const bf16x8* f1 = reinterpret_cast<const bf16x8*>(a.w1f) +
                       ((size_t)run * NW + wave) * KB1 * 64 + lane;
    const bf16x8* f2 = reinterpret_cast<const bf16x8*>(a.w2f) +
                       ((size_t)run * NW + wave) * KB2 * 64 + lane;
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb) w1r[kb] = f1[(size_t)kb * 64];
#pragma unroll
    for (int kb = 0; kb < KB2; ++kb) w2r[kb] = f2[(size_t)kb * 64];
  }
  const int tiles = (n + kInferRows - 1) / kInferRows;
  const int t0 = (int)blockIdx.x * kResTiles;
  const int t1 = min(t0 + kResTiles, tiles);
  // scaled value of element e (row e / Dp, coordinate e % Dp) of tile t
  auto xval = [&](int t, int e) {
    const int r = e / Dp, dd = e - r * Dp;
    const int row = t * kInferRows + r;
    float v = 0.f;
    if (r < kInferRows && row < n && dd < a.D)
      v = fmaf(Xr[(size_t)row * ldx + dd], a.xs_mul, a.xs_add);
    return v;
  };
  // with at most 16 elements per thread, the next tile's rows are loaded
  // into registers while the current tile is computed
  // (held as BF16 pairs: the LDS copy is BF16 anyway)
  constexpr bool kPre = kStage <= 16;
  static_assert(!kPre || kStage % 2 == 0, "staging pairs");
  constexpr int kPairs = kPre ? kStage / 2 : 1;
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  bf16x2 stage[kPairs];
  auto load_stage = [&](int t) {
#pragma unroll
    for (int u = 0; u < kPairs; ++u) {
      bf16x2 p;
      p[0] = (__bf16)xval(t, tid + (2 * u) * nthr);
      p[1] = (__bf16)xval(t, tid + (2 * u + 1) * nthr);
      stage[u] = p;
    }
  };
  if (kPre && t0 < t1) load_stage(t0);
  const __bf16* ar0 = A + (size_t)li * sa + 8 * lk;
  const __bf16* ar1 = ar0 + (size_t)32 * sa;
  const __bf16* hr0 = H1 + (size_t)li * sh + 8 * lk;
  const __bf16* hr1 = hr0 + (size_t)32 * sh;
  for (int t = t0; t < t1; ++t) {
    if constexpr (kPre) {
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int e = tid + u * nthr;
        const int r = e / Dp, dd = e - r * Dp;
        if (r < kInferRows) A[r * sa + dd] = stage[u / 2][u % 2];
      }
    } else {
      for (int e = tid; e < kInferRows * Dp; e += nthr) {
        const int r = e / Dp, dd = e - r * Dp;
        A[r * sa + dd] = (__bf16)xval(t, e);
      }
    }
    __syncthreads();  // A of tile t complete; H1 and ypart of t - 1 read
    if (kPre && t + 1 < t1) load_stage(t + 1);
    floatx16 c0 = {}, c1 = {};
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb) {
      const bf16x8 x0 = *reinterpret_cast<const bf16x8*>(ar0 + 16 * kb);
      const bf16x8 x1 = *reinterpret_cast<const bf16x8*>(ar1 + 16 * kb);
      c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, w1r[kb], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, w1r[kb], c1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r / 4) + 4 * lk + (r % 4);
      H1[row * sh + col] = (__bf16)fmaxf(c0[r] + b1c, 0.f);
      H1[(32 + row) * sh + col] = (__bf16)fmaxf(c1[r] + b1c, 0.f);
    }
    __syncthreads();  // H1 complete
    c0 = floatx16{};
    c1 = floatx16{};
#pragma unroll
    for (int kb = 0; kb < KB2; ++kb) {
      const bf16x8 h0 = *reinterpret_cast<const bf16x8*>(hr0 + 16 * kb);
      const bf16x8 h1 = *reinterpret_cast<const bf16x8*>(hr1 + 16 * kb);
      c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h0, w2r[kb], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h1, w2r[kb], c1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      c0[r] = fmaxf(c0[r] + b2c, 0.f) * w3c;
      c1[r] = fmaxf(c1[r] + b2c, 0.f) * w3c;
    }
    const float s0 = rows_of_block_vsel(c0, lane);
    const float s1 = rows_of_block_vsel(c1, lane);
    if ((lane & 1) == 0) {
      const int r = li >> 1;
      const int row = 8 * (r / 4) + 4 * lk + (r % 4);
      ypart[wave * kInferRows + row] = s0;
      ypart[wave * kInferRows + 32 + row] = s1;
    }
    __syncthreads();  // ypart complete
    const int row = t * kInferRows + tid;
    if (tid < kInferRows && row < n) {
      float s = b3;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += ypart[w * kInferRows + tid];
      y[blockIdx.y * y_run_stride + row] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Choice, true evaluation, selection, next generation, archive insert:
// kEvalRows targets per workgroup.
__global__ __launch_bounds__(kEvalThreads) void k_sur_select(SurArgs a) {
  extern __shared__ __align__(16) float sm[];
  __shared__ const float* rowp[kEvalRows];
  __shared__ int acc_s[kEvalRows];
  const int run = (int)blockIdx.y;
  const int i0 = (int)blockIdx.x * kEvalRows;
  const int nv = min(kEvalRows, a.NP - i0);
  const int tid = (int)threadIdx.x;
  if (tid < kEvalRows) {
    const int i = i0 + min(tid, nv - 1);
    const size_t t = (size_t)run * a.NP + i;
    int best = 0;
    if (a.use_model) {
      float bp = a.pred[t * a.k];
      for (int c = 1; c < a.k; ++c) {
        const float p = a.pred[t * a.k + c];
        if (p < bp) {
          bp = p;
          best = c;
        }
      }
    }
    rowp[tid] = a.cand + (t * a.k + best) * a.ldx;
    if (tid < nv) a.choice[t] = best;
  }
  __syncthreads();
  float* fout = sm + comp_lds_floats(a.D) - kEvalRows;
  comp_eval_rows(a, rowp, nv, sm, fout);
  if (tid < nv) {
    const int i = i0 + tid;
    const size_t t = (size_t)run * a.NP + i;
    const float fu = fout[tid], fx = a.fit_cur[t];
    const bool accept = fu < fx;
    a.fit_next[t] = accept ? fu : fx;
    acc_s[tid] = accept ? 1 : 0;
    if (accept) {
      atomicAdd(&a.accepted[run], 1ull);
      atomicMin(&a.best_key[run], fit_key(fu, i));
    }
    const int pos = (int)(((long long)a.round * a.NP + i) % a.cap);
    a.at[(size_t)run * a.cap + pos] = log10f(fu + 1e-8f);
  }
  __syncthreads();
  const int nq = (a.D + 3) / 4;
  for (int t2 = tid; t2 < nv * nq; t2 += kEvalThreads) {
    const int r = t2 / nq, q = t2 - r * nq;
    const int i = i0 + r;
    const size_t t = (size_t)run * a.NP + i;
    const float4 u = ld4(rowp[r] + 4 * q);
    const float4 xv = ld4(a.pop_cur + t * a.ldx + 4 * q);
    st4(a.pop_next + t * a.ldx + 4 * q, acc_s[r] ? u : xv);
    const int pos = (int)(((long long)a.round * a.NP + i) % a.cap);
    st4(a.ax + ((size_t)run * a.cap + pos) * a.ldx + 4 * q, u);
  }
}

// Generation 0 into the archive (its first fill): rows and their targets.
__global__ __launch_bounds__(256) void k_archive_init(SurArgs a) {
  const int nq = (a.D + 3) / 4;
  const size_t total = (size_t)a.runs * a.NP * nq;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (size_t)gridDim.x * 256) {
    const size_t row = t / nq;
    const int q = (int)(t - row * nq);
    const int run = (int)(row / a.NP), i = (int)(row - (size_t)run * a.NP);
    const int pos = i % a.cap;
    st4(a.ax + ((size_t)run * a.cap + pos) * a.ldx + 4 * q,
        ld4(a.pop_cur + row * a.ldx + 4 * q));
    if (q == 0) a.at[(size_t)run * a.cap + pos] = log10f(a.fit_cur[row] + 1e-8f);
  }
}

// ---------------------------------------------------------------------------
// Model: initial weights (He-uniform from Philox tag 6, biases zero), BF16
// fragment and FP32 transposed copies, training.
__global__ __launch_bounds__(256) void k_model_init(SurArgs a, int P) {
  const size_t total = (size_t)a.runs * a.pstride;
  const int H = a.H, D = a.D;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (size_t)gridDim.x * 256) {
    const int run = (int)(t / a.pstride), p = (int)(t - (size_t)run * a.pstride);
    float bound = 0.f;
    if (p < H * D) bound = sqrtf(6.0f / D);
    else if (p >= H * D + H && p < H * D + H + H * H) bound = sqrtf(6.0f / H);
    else if (p >= H * D + H + H * H + H && p < H * D + H + H * H + 2 * H)
      bound = sqrtf(3.0f / H);
    float val = 0.f;
    if (bound > 0.f && p < P) {
      const Words4 w = draw_block(kTagModel, (uint32_t)run, 0u, 0u,
                                  (uint32_t)(p >> 2), a.mkey_lo, a.mkey_hi);
      const int sl = p & 3;
      const uint32_t word = sl == 0 ? w.w[0] : sl == 1 ? w.w[1]
                            : sl == 2 ? w.w[2] : w.w[3];
      const float u = (float)(word >> 8) * 0x1.0p-24f;
      val = bound * fmaf(2.0f, u, -1.0f);
    }
    a.theta[t] = val;
    a.m[t] = 0.f;
    a.v[t] = 0.f;
  }
}

// Position of element (n, k) of a weight matrix with K padded columns in
// the BF16 MFMA B-operand layout: block n / 32, K-step k / 16, lane, slot.
__device__ __forceinline__ size_t frag_index(int n, int k, int K) {
  const size_t nb = n / 32, kb = k / 16;
  const int ln = (n % 32) + 32 * ((k % 16) / 8);
  return ((nb * (K / 16) + kb) * 64 + ln) * 8 + (k % 8);
}

__global__ __launch_bounds__(256) void k_model_prep(SurArgs a) {
  const int H = a.H, D = a.D, Dp = a.Dp;
  const size_t per = (size_t)H * Dp + (size_t)H * H;
  const size_t total = (size_t)a.runs * per;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (size_t)gridDim.x * 256) {
    const int run = (int)(t / per);
    size_t e = t - (size_t)run * per;
    const float* th = a.theta + (size_t)run * a.pstride;
    int n, k, K;
    __bf16* dst;
    float v;
    if (e < (size_t)H * Dp) {
      n = (int)(e / Dp);
      k = (int)(e - (size_t)n * Dp);
      K = Dp;
      v = k < D ? th[(size_t)n * D + k] : 0.f;
      dst = a.w1f + (size_t)run * H * Dp;
      if (k < D) a.w1t[((size_t)run * D + k) * H + n] = v;
    } else {
      e -= (size_t)H * Dp;
      n = (int)(e / H);
      k = (int)(e - (size_t)n * H);
      K = H;
      v = th[(size_t)H * D + H + (size_t)n * H + k];
      dst = a.w2f + (size_t)run * H * H;
      a.w2t[((size_t)run * H + k) * H + n] = v;
    }
    dst[frag_index(n, k, K)] = (__bf16)v;
  }
}

// Training on FP32 MFMA.  The gradient's products use 32x32x2 blocks (lane
// l supplies A(l % 32, 2 kb + l / 32) and B(2 kb + l / 32, l % 32);
// register r of lane l holds C(8 (r / 4) + 4 (l / 32) + r % 4, l % 32));
// the forward pass takes the minibatch in blocks of kTrainRows = 16 rows
// with 16x16x4 blocks (lane l supplies A(l % 16, 4 s + l / 16) and
// B(4 s + l / 16, l % 16) for K-step s; register r of lane l holds
// C(4 (l / 16) + r, l % 16)), so that a minibatch of 128 rows of 30 runs
// already spreads over 240 workgroups.
constexpr int kTrainRows = 16;
typedef float floatx4 __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr size_t train_lds_floats(int Dp, int H) {
  return (size_t)kTrainRows * (Dp + 1) + (size_t)3 * kTrainRows * (H + 1) +
         2 * kTrainRows;
}

__device__ __forceinline__ int c_row(int r, int lane) {
  return 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
}

// One 32x32 block C = A B over K (a multiple of 16): the lane's A values
// at ap[2 kb * astep], its B values at bp[2 kb * bstep] (rows k >= kvalid
// of B read as zero).  K-steps go in batches of eight whose loads are
// issued one batch ahead of the MFMAs that use them.
__device__ __forceinline__ floatx16 mfma_block(const float* ap, int astep,
                                               const float* bp, int bstep,
                                               int K, int kvalid, int lk) {
  floatx16 c = {};
  float an[8], bn[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    an[u] = ap[(size_t)2 * u * astep];
    bn[u] = 2 * u + lk < kvalid ? bp[(size_t)2 * u * bstep] : 0.f;
  }
  for (int kb = 0; kb < K / 2; kb += 8) {
    float ac[8], bc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      ac[u] = an[u];
      bc[u] = bn[u];
    }
    if (kb + 8 < K / 2) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k2 = 2 * (kb + 8 + u);
        an[u] = ap[(size_t)k2 * astep];
        bn[u] = k2 + lk < kvalid ? bp[(size_t)k2 * bstep] : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[u], bc[u], c, 0, 0, 0);
  }
  return c;
}

// Two 16x16 blocks of C = A B over K (a multiple of 32), columns boff0 and
// boff1 of B, sharing the A reads: the lane's A value of K-step s at
// ap[4 s + lq] (lq = l / 16), B(k, n) at bb[k * bstep + boff] (rows
// k >= kvalid read as zero); `two` = 0 leaves c1 untouched.  KS = K / 4 when
// K is compile-time: the B values of the first 32 K-steps are requested
// before the first MFMA and each later one 32 steps ahead of its use.
// Otherwise K-steps go in batches of eight, issued one batch ahead.
template <int KS>
__device__ __forceinline__ void mfma16_pair(const float* ap, const float* bb,
                                            int boff0, int boff1, int bstep,
                                            int K, int kvalid, int lq,
                                            bool two, floatx4& c0,
                                            floatx4& c1) {
  auto load_b = [&](int st, int boff) {
    const int k = 4 * st + lq;
    return k < kvalid ? bb[(size_t)k * bstep + boff] : 0.f;
  };
  c0 = floatx4{0.f, 0.f, 0.f, 0.f};
  c1 = c0;
  if constexpr (KS > 0) {
    static_assert(KS % 8 == 0, "K-steps in groups of eight");
    constexpr int P = KS < 32 ? KS : 32;  // K-steps in flight
    float b0[KS], b1[KS];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      b0[u] = load_b(u, boff0);
      b1[u] = two ? load_b(u, boff1) : 0.f;
    }
#pragma unroll
    for (int u0 = 0; u0 < KS; u0 += 8) {
      float av[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) av[u] = ap[4 * (u0 + u) + lq];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], b0[u0 + u], c0, 0,
                                                  0, 0);
        if (two)
          c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], b1[u0 + u], c1, 0,
                                                    0, 0);
      }
#pragma unroll
      for (int u = u0; u < u0 + 8; ++u) {
        if (u + P < KS) {
          b0[u + P] = load_b(u + P, boff0);
          b1[u + P] = two ? load_b(u + P, boff1) : 0.f;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    float a_n[8], b0n[8], b1n[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a_n[u] = ap[4 * u + lq];
      b0n[u] = load_b(u, boff0);
      b1n[u] = two ? load_b(u, boff1) : 0.f;
    }
    for (int s0 = 0; s0 < K / 4; s0 += 8) {
      float ac[8], b0c[8], b1c[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        ac[u] = a_n[u];
        b0c[u] = b0n[u];
        b1c[u] = b1n[u];
      }
      if (s0 + 8 < K / 4) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a_n[u] = ap[4 * (s0 + 8 + u) + lq];
          b0n[u] = load_b(s0 + 8 + u, boff0);
          b1n[u] = two ? load_b(s0 + 8 + u, boff1) : 0.f;
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[u], b0c[u], c0, 0, 0, 0);
        if (two)
          c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[u], b1c[u], c1, 0, 0,
                                                    0);
      }
    }
  }
}

// Forward pass of 16 minibatch rows per workgroup (8 waves; wave w owns the
// 16-column blocks w, w + 8, ... of each product, two at a time), output
// error e = 2 (y - t) / B, delta2 = [h2 > 0] e w3 and delta1 =
// [h1 > 0] (delta2 W2); what the gradient needs goes to the scratch
// arrays.  Odd LDS row strides keep the A reads conflict-free.
// KS1 = Dp / 4 and KS2 = H / 4 when the sizes are compile-time, else 0.
template <int KS1, int KS2>
__global__ __launch_bounds__(512) void k_train_fwd(SurArgs a) {
  extern __shared__ __align__(16) float sm[];
  const int run = (int)blockIdx.y;
  const int tid = (int)threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int li = lane % 16, lq = lane / 16;
  const int H = KS2 > 0 ? 4 * KS2 : a.H, D = a.D;
  const int Dp = KS1 > 0 ? 4 * KS1 : a.Dp;
  const int b0 = (int)blockIdx.x * kTrainRows;
  const int sx = Dp + 1, sh = H + 1;
  float* XS = sm;                       // [16][sx]
  float* H1 = XS + kTrainRows * sx;     // [16][sh]
  float* H2 = H1 + kTrainRows * sh;
  float* D2 = H2 + kTrainRows * sh;
  float* E = D2 + kTrainRows * sh;      // [16]
  int* src = reinterpret_cast<int*>(E + kTrainRows);
  const float* th = a.theta + (size_t)run * a.pstride;
  const float* b1 = th + (size_t)H * D;
  const float* W2 = b1 + H;
  const float* b2 = W2 + (size_t)H * H;
  const float* w3 = b2 + H;
  const float b3 = w3[H];
  const float* w1t = a.w1t + (size_t)run * D * H;
  const float* w2t = a.w2t + (size_t)run * H * H;
  const size_t rb = (size_t)run * a.B + b0;
  if (tid < kTrainRows) {
    const Words4 w = draw_block(kTagTrain, (uint32_t)run, a.step,
                                (uint32_t)(b0 + tid), 0u, a.mkey_lo,
                                a.mkey_hi);
    src[tid] = uniform_below(w.w[0], (uint32_t)a.filled);
  }
  __syncthreads();
  for (int t = tid; t < kTrainRows * Dp; t += 512) {
    const int r = t / Dp, dd = t - r * Dp;
    const float v =
        dd < D ? fmaf(a.ax[((size_t)run * a.cap + src[r]) * a.ldx + dd],
                      a.xs_mul, a.xs_add)
               : 0.f;
    XS[r * sx + dd] = v;
    a.xsb[(rb + r) * Dp + dd] = v;
  }
  __syncthreads();
  const int nblk = H / 16;
  // the lane's C values: rows 4 lq + r, column li of each block
  for (int nb = wave; nb < nblk; nb += 16) {  // layer 1: B(k, n) = W1[n][k]
    const bool two = nb + 8 < nblk;
    floatx4 c[2];
    mfma16_pair<KS1>(XS + li * sx, w1t, nb * 16 + li, (nb + 8) * 16 + li, H,
                     Dp, D, lq, two, c[0], c[1]);
    for (int q = 0; q < (two ? 2 : 1); ++q) {
      const int n = (nb + 8 * q) * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * lq + r;
        const float v = fmaxf(c[q][r] + b1[n], 0.f);
        H1[row * sh + n] = v;
        a.h1b[(rb + row) * H + n] = v;
      }
    }
  }
  __syncthreads();
  for (int nb = wave; nb < nblk; nb += 16) {  // layer 2: B(k, n) = W2[n][k]
    const bool two = nb + 8 < nblk;
    floatx4 c[2];
    mfma16_pair<KS2>(H1 + li * sh, w2t, nb * 16 + li, (nb + 8) * 16 + li, H,
                     H, H, lq, two, c[0], c[1]);
    for (int q = 0; q < (two ? 2 : 1); ++q) {
      const int n = (nb + 8 * q) * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * lq + r;
        const float v = fmaxf(c[q][r] + b2[n], 0.f);
        H2[row * sh + n] = v;
        a.h2b[(rb + row) * H + n] = v;
      }
    }
  }
  __syncthreads();
  {
    // y of row r from 32 partial sums (i = part mod 32), then a butterfly
    const int r = tid / 32, part = tid % 32;
    float y = 0.f;
    for (int i = part; i < H; i += 32) y = fmaf(w3[i], H2[r * sh + i], y);
    y += __shfl_xor(y, 1, 64);
    y += __shfl_xor(y, 2, 64);
    y += __shfl_xor(y, 4, 64);
    y += __shfl_xor(y, 8, 64);
    y += __shfl_xor(y, 16, 64);
    if (part == 0) {
      const float e =
          2.0f * (y + b3 - a.at[(size_t)run * a.cap + src[r]]) / (float)a.B;
      E[r] = e;
      a.eb[rb + r] = e;
    }
  }
  __syncthreads();
  for (int t = tid; t < kTrainRows * H; t += 512) {
    const int r = t / H, i = t - r * H;
    const float dv = H2[r * sh + i] > 0.f ? E[r] * w3[i] : 0.f;
    D2[r * sh + i] = dv;
    a.d2b[(rb + r) * H + i] = dv;
  }
  __syncthreads();
  for (int nb = wave; nb < nblk; nb += 16) {  // delta1: B(k = i, n = j) = W2[i][j]
    const bool two = nb + 8 < nblk;
    floatx4 c[2];
    mfma16_pair<KS2>(D2 + li * sh, W2, nb * 16 + li, (nb + 8) * 16 + li, H,
                     H, H, lq, two, c[0], c[1]);
    for (int q = 0; q < (two ? 2 : 1); ++q) {
      const int n = (nb + 8 * q) * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * lq + r;
        a.d1b[(rb + row) * H + n] = H1[row * sh + n] > 0.f ? c[q][r] : 0.f;
      }
    }
  }
}

// One Adam step of a parameter from its moments m, v and value th with
// gradient g: new moments in mv, vv, new value returned.
__device__ __forceinline__ float adam_math(const SurArgs& a, float m, float v,
                                           float th, float g, float& mv,
                                           float& vv) {
  mv = fmaf(a.beta1, m, (1.0f - a.beta1) * g);
  vv = fmaf(a.beta2, v, (1.0f - a.beta2) * g * g);
  return th - a.lr * (mv / a.c1) / (sqrtf(vv / a.c2) + a.eps);
}

__device__ __forceinline__ float adam_update(const SurArgs& a, size_t at,
                                             float g) {
  float mv, vv;
  const float t = adam_math(a, a.m[at], a.v[at], a.theta[at], g, mv, vv);
  a.m[at] = mv;
  a.v[at] = vv;
  a.theta[at] = t;
  return t;
}

// Weight-matrix gradients as products over the minibatch, one wave per
// 32x32 block (W1: delta1^T xs, W2: delta2^T h1), then Adam on each entry.
__device__ void grad_vec(const SurArgs& a, int run, int t);

// The weight-gradient block product with the minibatch extent known at
// compile time (KS K-steps of two rows, every row valid): both operands come
// from memory, and the values of K-step u + P are requested when the MFMAs
// of K-steps u .. u + 7 have been issued, so the chain waits for about one
// round trip per P steps instead of one per batch of eight.  Same products
// and order as mfma_block.
template <int KS>
__device__ __forceinline__ floatx16 mfma_block_mm(const float* ap, int astep,
                                                  const float* bp,
                                                  int bstep) {
  static_assert(KS % 8 == 0, "K-steps in groups of eight");
  constexpr int P = KS < 32 ? KS : 32;  // K-steps in flight
  float av[KS], bv[KS];
#pragma unroll
  for (int u = 0; u < P; ++u) {
    av[u] = ap[(size_t)2 * u * astep];
    bv[u] = bp[(size_t)2 * u * bstep];
  }
  floatx16 c = {};
#pragma unroll
  for (int u0 = 0; u0 < KS; u0 += 8) {
#pragma unroll
    for (int u = u0; u < u0 + 8; ++u)
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], bv[u], c, 0, 0, 0);
#pragma unroll
    for (int u = u0; u < u0 + 8; ++u) {
      if (u + P < KS) {
        av[u + P] = ap[(size_t)2 * (u + P) * astep];
        bv[u + P] = bp[(size_t)2 * (u + P) * bstep];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  return c;
}

// Workgroups 0 .. ceil(blocks / 4) - 1: one wave per 32x32 weight block;
// the rest: the vector parameters.  Every updated weight is also written to
// the BF16 inference copy and the FP32 transposed copy.  KS = B / 2 when the
// minibatch size is compile-time (the deep-prefetch product), else 0.
template <int KS>
__global__ __launch_bounds__(256) void k_train_grad(SurArgs a) {
  __shared__ float tblk[4][32][33];  // one 32x32 block per wave (+1 column)
  const int run = (int)blockIdx.y;
  const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
  const int li = lane % 32, lk = lane / 32;
  const int H = a.H, D = a.D, Dp = a.Dp, B = a.B;
  const int nbh = H / 32, nbd = Dp / 32;
  const int nb1 = nbh * nbd, nb2 = nbh * nbh;
  const int mat_wgs = (nb1 + nb2 + 3) / 4;
  if ((int)blockIdx.x >= mat_wgs) {
    grad_vec(a, run, ((int)blockIdx.x - mat_wgs) * 256 + (int)threadIdx.x);
    return;
  }
  const int blk = (int)blockIdx.x * 4 + wave;
  if (blk >= nb1 + nb2) return;  // whole waves; no barrier in this kernel
  const bool w1 = blk < nb1;
  const int q = w1 ? blk : blk - nb1;
  const int ib = w1 ? q / nbd : q / nbh;
  const int jb = w1 ? q - ib * nbd : q - ib * nbh;
  const float* dl = (w1 ? a.d1b : a.d2b) + (size_t)run * B * H;
  const int ldh = w1 ? Dp : H;
  const float* hv = w1 ? a.xsb + (size_t)run * B * Dp : a.h1b + (size_t)run * B * H;
  const int i = ib * 32 + li, j = jb * 32 + li;
  // A(i, b) = delta[b][i], B(b, j) = input[b][j]; B is a multiple of 32
  floatx16 c;
  if constexpr (KS > 0)
    c = mfma_block_mm<KS>(dl + (size_t)lk * H + i, H,
                          hv + (size_t)lk * ldh + j, ldh);
  else
    c = mfma_block(dl + (size_t)lk * H + i, H, hv + (size_t)lk * ldh + j, ldh,
                   B, B, lk);
  // Adam on the lane's 16 entries: the entries are distinct, so every m, v
  // and theta is read before any is written and the reads share one wait
  const size_t base = (size_t)run * a.pstride;
  const int jj = jb * 32 + li;
  const bool valid = !w1 || jj < D;
  float mo[16], vo[16], to[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int ii = ib * 32 + c_row(r, lane);
    const size_t at = w1 ? base + (size_t)ii * D + jj
                         : base + (size_t)H * D + H + (size_t)ii * H + jj;
    if (valid) {
      mo[r] = a.m[at];
      vo[r] = a.v[at];
      to[r] = a.theta[at];
    }
  }
  // the block's new weights (0 in W1's padding columns) go through LDS so
  // that the transposed copy is written in rows of 32 and the BF16
  // fragment copy in 16-byte pieces
  float(*tb)[33] = tblk[wave];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int rr = c_row(r, lane);
    float t = 0.f;
    if (valid) {
      const int ii = ib * 32 + rr;
      const size_t at = w1 ? base + (size_t)ii * D + jj
                           : base + (size_t)H * D + H + (size_t)ii * H + jj;
      float mv, vv;
      t = adam_math(a, mo[r], vo[r], to[r], c[r], mv, vv);
      a.m[at] = mv;
      a.v[at] = vv;
      a.theta[at] = t;
    }
    tb[rr][li] = t;
  }
  __builtin_amdgcn_wave_barrier();
  // transposed copy: row jj of wT holds column jj of the block (32 floats)
  float* wt = w1 ? a.w1t + (size_t)run * D * H : a.w2t + (size_t)run * H * H;
  const int nrow_t = w1 ? D : H;
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int jl = 2 * s2 + lk, jr = jb * 32 + jl;
    if (jr < nrow_t) wt[(size_t)jr * H + ib * 32 + li] = tb[li][jl];
  }
  // BF16 fragments: K-steps 2 jb and 2 jb + 1 of block row ib, 1 KB each;
  // lane l holds the eight consecutive k of one row there
  const int K = w1 ? Dp : H;
  __bf16* wf = w1 ? a.w1f + (size_t)run * H * Dp : a.w2f + (size_t)run * H * H;
#pragma unroll
  for (int kbl = 0; kbl < 2; ++kbl) {
    const int k0 = kbl * 16 + lk * 8;
    bf16x8 v;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (__bf16)tb[li][k0 + q];
    *reinterpret_cast<bf16x8*>(wf + frag_index(ib * 32 + li, jb * 32 + k0, K)) =
        v;
  }
}

// Bias and output-layer gradients (3H + 1 per run, t indexes them), summed
// over the minibatch rows, then Adam.  Eight partial sums over rows
// b = u mod 8, each in increasing b, added in order at the end; the rows'
// values are read 32 at a time so that the reads share one wait.
__device__ void grad_vec(const SurArgs& a, int run, int t) {
  const int H = a.H, D = a.D, B = a.B;
  if (t > 3 * H) return;
  const float* d1 = a.d1b + (size_t)run * B * H;
  const float* d2 = a.d2b + (size_t)run * B * H;
  const float* h2 = a.h2b + (size_t)run * B * H;
  const float* e = a.eb + (size_t)run * B;
  // row b contributes col[b * stride] (w3: times e[b])
  const float* col;
  int stride = H;
  bool times_e = false;
  size_t p;
  if (t < H) {  // b1
    col = d1 + t;
    p = (size_t)H * D + t;
  } else if (t < 2 * H) {  // b2
    col = d2 + (t - H);
    p = (size_t)H * D + H + (size_t)H * H + (t - H);
  } else if (t < 3 * H) {  // w3
    col = h2 + (t - 2 * H);
    times_e = true;
    p = (size_t)H * D + H + (size_t)H * H + H + (t - 2 * H);
  } else {  // b3
    col = e;
    stride = 1;
    p = (size_t)H * D + H + (size_t)H * H + 2 * H;
  }
  float gp[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  constexpr int kChunk = 32;  // B is a multiple of 32
  for (int b0 = 0; b0 < B; b0 += kChunk) {
    float v[kChunk], w[kChunk];
#pragma unroll
    for (int q = 0; q < kChunk; ++q) {
      v[q] = col[(size_t)(b0 + q) * stride];
      w[q] = times_e ? e[b0 + q] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kChunk; ++q)
      gp[q % 8] = times_e ? fmaf(w[q], v[q], gp[q % 8]) : gp[q % 8] + v[q];
  }
  float g = 0.f;
#pragma unroll
  for (int u = 0; u < 8; ++u) g += gp[u];
  adam_update(a, (size_t)run * a.pstride + p, g);
}

__global__ __launch_bounds__(256) void k_sur_reset(SurArgs a) {
  for (int r = (int)(blockIdx.x * 256 + threadIdx.x); r < a.runs;
       r += (int)(gridDim.x * 256)) {
    a.best_key[r] = ~0ull;
    a.accepted[r] = 0ull;
  }
}

__global__ __launch_bounds__(256) void k_sur_best(SurArgs a) {
  const int run = (int)blockIdx.x;
  unsigned long long best = ~0ull;
  for (int i = (int)threadIdx.x; i < a.NP; i += 256)
    best = min(best, fit_key(a.fit_cur[(size_t)run * a.NP + i], i));
  for (int m = 32; m >= 1; m >>= 1) {
    const unsigned long long o =
        ((unsigned long long)__shfl_xor((unsigned)(best >> 32), m, 64) << 32) |
        (unsigned long long)__shfl_xor((unsigned)best, m, 64);
    best = min(best, o);
  }
  if ((threadIdx.x % 64) == 0) atomicMin(&a.best_key[run], best);
}

// Transposed rotations Rt[c][j][i] = R[c][i][j] and shifts.
__global__ __launch_bounds__(256) void k_comp_prep(const float* O,
                                                   const float* R, int ldr,
                                                   int n, int D, float* Op,
                                                   float* Rt) {
  const size_t per = (size_t)D * D;
  const size_t total = (size_t)n * per;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (size_t)gridDim.x * 256) {
    const int c = (int)(t / per);
    const size_t e = t - (size_t)c * per;
    const int j = (int)(e / D), i = (int)(e - (size_t)j * D);
    Rt[t] = R[((size_t)c * D + i) * ldr + j];
    if (j == 0) Op[(size_t)c * D + i] = O[(size_t)c * D + i];
  }
}

}  // namespace de

// ---------------------------------------------------------------------------
// Host side.

namespace {

using de::SurArgs;

constexpr uint64_t kSurMagic = 0x6465737572726721ull;

size_t rup(size_t v, size_t m) { return (v + m - 1) / m * m; }

int64_t model_size(int D, int H) {
  return (int64_t)H * D + H + (int64_t)H * H + H + H + 1;
}

struct SLayout {
  size_t best, acc, O, Rt, bias, cand, pred, choice, theta, m, v, w1f, w2f,
      w1t, w2t, ax, at, xsb, h1b, h2b, d1b, d2b, eb, total;
  int pstride, Dp;
};

de_status check(const de_params* p, const de_composition* c,
                const de_surrogate_params* s) {
  if (!p || !c || !s) return DE_E_INVAL;
  if (p->runs < 1 || p->runs > 65535 || p->NP < 4 || p->D < 1)
    return DE_E_INVAL;
  if ((int64_t)p->runs * p->NP * 16 > std::numeric_limits<int32_t>::max())
    return DE_E_INVAL;
  if (!std::isfinite(p->F) || !(p->F > 0.f)) return DE_E_INVAL;
  if (!(p->CR >= 0.f && p->CR <= 1.f)) return DE_E_INVAL;
  if (!std::isfinite(p->lo) || !std::isfinite(p->hi) || !(p->lo < p->hi) ||
      !std::isfinite(p->hi - p->lo))
    return DE_E_INVAL;
  if (c->n < 1 || c->n > de::kMaxComp || c->reserved != 0) return DE_E_INVAL;
  if (c->ldr < p->D || !c->O || !c->R || !c->bias) return DE_E_INVAL;
  if (!std::isfinite(c->sigma) || !(c->sigma > 0.f)) return DE_E_INVAL;
  for (int k = 0; k < c->n; ++k)
    if (!std::isfinite(c->bias[k])) return DE_E_INVAL;
  if (s->k < 1 || s->k > 16) return DE_E_INVAL;
  if (s->hidden < 32 || s->hidden > 256 || s->hidden % 32) return DE_E_INVAL;
  if (s->batch < 32 || s->batch > 1024 || s->batch % 32) return DE_E_INVAL;
  if (s->archive < s->batch || s->archive < p->NP) return DE_E_INVAL;
  if ((int64_t)s->archive * p->runs > std::numeric_limits<int32_t>::max())
    return DE_E_INVAL;
  if (s->steps < 0 || s->warmup_gens < 0) return DE_E_INVAL;
  if (!std::isfinite(s->lr) || !(s->lr > 0.f)) return DE_E_INVAL;
  if (!(s->beta1 >= 0.f && s->beta1 < 1.f) || !(s->beta2 >= 0.f && s->beta2 < 1.f))
    return DE_E_INVAL;
  if (!std::isfinite(s->eps) || !(s->eps > 0.f)) return DE_E_INVAL;
  // LDS: composition evaluation and model inference
  if (de::comp_lds_floats(p->D) * 4 > (size_t)de::kMaxLdsBytes ||
      de::infer_lds_bytes((int)rup(p->D, 32), s->hidden) >
          (size_t)de::kMaxLdsBytes ||
      de::train_lds_floats((int)rup(p->D, 32), s->hidden) * 4 >
          (size_t)de::kMaxLdsBytes)
    return DE_E_UNSUPPORTED;
  return DE_OK;
}

SLayout layout(const de_params& p, const de_composition& c,
               const de_surrogate_params& s, int ldx) {
  SLayout L{};
  size_t off = 0;
  auto take = [&off](size_t bytes) {
    const size_t at = off;
    off = rup(off + bytes, 256);
    return at;
  };
  const size_t R = (size_t)p.runs, NP = (size_t)p.NP, D = (size_t)p.D;
  const size_t H = (size_t)s.hidden, k = (size_t)s.k, B = (size_t)s.batch;
  L.Dp = (int)rup(D, 32);
  L.pstride = (int)rup((size_t)model_size(p.D, s.hidden), 64);
  L.best = take(8 * R);
  L.acc = take(8 * R);
  L.O = take(4 * (size_t)c.n * D);
  L.Rt = take(4 * (size_t)c.n * D * D);
  L.bias = take(4 * (size_t)c.n);
  L.cand = take(4 * R * NP * k * ldx);
  L.pred = take(4 * R * NP * k);
  L.choice = take(4 * R * NP);
  L.theta = take(4 * R * L.pstride);
  L.m = take(4 * R * L.pstride);
  L.v = take(4 * R * L.pstride);
  L.w1f = take(2 * R * H * L.Dp);
  L.w2f = take(2 * R * H * H);
  L.w1t = take(4 * R * D * H);
  L.w2t = take(4 * R * H * H);
  L.ax = take(4 * R * (size_t)s.archive * ldx);
  L.at = take(4 * R * (size_t)s.archive);
  L.xsb = take(4 * R * B * L.Dp);
  L.h1b = take(4 * R * B * H);
  L.h2b = take(4 * R * B * H);
  L.d1b = take(4 * R * B * H);
  L.d2b = take(4 * R * B * H);
  L.eb = take(4 * R * B);
  L.total = off;
  return L;
}

de_status from_hip(hipError_t e) {
  return e == hipSuccess ? DE_OK : DE_E_DEVICE;
}
#define FROM_HIP(expr) from_hip(DE_NOTE(expr))

int grid_for(size_t work, int per) {
  size_t b = (work + per - 1) / per;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

}  // namespace

struct de_sur {
  uint64_t magic = kSurMagic;
  de_params p{};
  de_surrogate_params sp{};
  int n = 0, ldx = 0;
  float sigma = 0.f;
  float* pop[2] = {nullptr, nullptr};
  float* fit[2] = {nullptr, nullptr};
  char* work = nullptr;
  SLayout L{};
  int64_t gen = 0;
  int64_t step = 0;  // Adam steps taken
  int64_t rounds = 1;  // archive insert rounds done (generation 0 is one)
  int last_use_model = 0;
};

namespace {

std::mutex g_mu;
std::set<const de_sur*>& live_set() {
  static std::set<const de_sur*> s;
  return s;
}

bool live(const de_sur* s) {
  if (!s) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  return live_set().count(s) != 0 && s->magic == kSurMagic;
}

SurArgs args_of(const de_sur* s) {
  SurArgs a{};
  char* w = s->work;
  const SLayout& L = s->L;
  const int b = (int)(s->gen & 1);
  a.pop_cur = s->pop[b];
  a.pop_next = s->pop[b ^ 1];
  a.fit_cur = s->fit[b];
  a.fit_next = s->fit[b ^ 1];
  a.runs = s->p.runs;
  a.NP = s->p.NP;
  a.D = s->p.D;
  a.ldx = s->ldx;
  a.k = s->sp.k;
  a.H = s->sp.hidden;
  a.Dp = L.Dp;
  a.pstride = L.pstride;
  a.F = s->p.F;
  a.lo = s->p.lo;
  a.hi = s->p.hi;
  a.xs_mul = 2.0f / (s->p.hi - s->p.lo);
  a.xs_add = -(s->p.lo + s->p.hi) / (s->p.hi - s->p.lo);
  a.cr_threshold = (uint32_t)std::floor((double)s->p.CR * 16777216.0);
  a.gen = (uint32_t)s->gen;
  a.key_lo = (uint32_t)s->p.seed;
  a.key_hi = (uint32_t)(s->p.seed >> 32);
  a.O = reinterpret_cast<const float*>(w + L.O);
  a.Rt = reinterpret_cast<const float*>(w + L.Rt);
  a.bias = reinterpret_cast<const float*>(w + L.bias);
  a.n = s->n;
  a.inv2s2 = (float)(1.0 / (2.0 * (double)s->sigma * s->sigma));
  a.cand = reinterpret_cast<float*>(w + L.cand);
  a.pred = reinterpret_cast<float*>(w + L.pred);
  a.choice = reinterpret_cast<int*>(w + L.choice);
  a.theta = reinterpret_cast<float*>(w + L.theta);
  a.m = reinterpret_cast<float*>(w + L.m);
  a.v = reinterpret_cast<float*>(w + L.v);
  a.w1f = reinterpret_cast<__bf16*>(w + L.w1f);
  a.w2f = reinterpret_cast<__bf16*>(w + L.w2f);
  a.w1t = reinterpret_cast<float*>(w + L.w1t);
  a.w2t = reinterpret_cast<float*>(w + L.w2t);
  a.ax = reinterpret_cast<float*>(w + L.ax);
  a.at = reinterpret_cast<float*>(w + L.at);
  a.cap = s->sp.archive;
  a.round = (int)s->rounds;
  a.filled = (int)std::min<int64_t>(s->sp.archive, s->rounds * s->p.NP);
  a.B = s->sp.batch;
  a.step = (uint32_t)s->step;
  a.mkey_lo = (uint32_t)s->sp.model_seed;
  a.mkey_hi = (uint32_t)(s->sp.model_seed >> 32);
  a.lr = s->sp.lr;
  a.beta1 = s->sp.beta1;
  a.beta2 = s->sp.beta2;
  a.eps = s->sp.eps;
  a.xsb = reinterpret_cast<float*>(w + L.xsb);
  a.h1b = reinterpret_cast<float*>(w + L.h1b);
  a.h2b = reinterpret_cast<float*>(w + L.h2b);
  a.d1b = reinterpret_cast<float*>(w + L.d1b);
  a.d2b = reinterpret_cast<float*>(w + L.d2b);
  a.eb = reinterpret_cast<float*>(w + L.eb);
  a.best_key = reinterpret_cast<unsigned long long*>(w + L.best);
  a.accepted = reinterpret_cast<unsigned long long*>(w + L.acc);
  return a;
}

de_status set_lds_attributes() {
  const void* fns[] = {reinterpret_cast<const void*>(&de::k_comp_eval),
                       reinterpret_cast<const void*>(&de::k_sur_select),
                       reinterpret_cast<const void*>(&de::k_mlp_infer),
                       reinterpret_cast<const void*>(&de::k_train_fwd<0, 0>),
                       reinterpret_cast<const void*>(&de::k_train_fwd<32, 64>)};
  for (const void* f : fns) {
    const de_status rc = FROM_HIP(de::set_max_dynamic_lds(f));
    if (rc != DE_OK) return rc;
  }
  return DE_OK;
}

// Inference of n rows per run for nruns runs from run0 (X and y strided by
// run): the register-resident kernel for padded widths up to 128 and
// H in {32, 64, 128, 256}, else the general one.
using InferRes = void (*)(SurArgs, const float*, size_t, int, int, float*,
                          size_t, int);

template <int KB1>
InferRes infer_res_for_h(int H) {
  switch (H) {
    case 32: return &de::k_mlp_infer_res<KB1, 2>;
    case 64: return &de::k_mlp_infer_res<KB1, 4>;
    case 128: return &de::k_mlp_infer_res<KB1, 8>;
    case 256: return &de::k_mlp_infer_res<KB1, 16>;
    default: return nullptr;
  }
}

InferRes infer_res_kernel(int Dp, int H) {
  switch (Dp) {
    case 32: return infer_res_for_h<2>(H);
    case 64: return infer_res_for_h<4>(H);
    case 96: return infer_res_for_h<6>(H);
    case 128: return infer_res_for_h<8>(H);
    default: return nullptr;
  }
}

de_status launch_infer(const SurArgs& a, const float* X, size_t x_stride,
                       int n, int ldx, float* y, size_t y_stride, int run0,
                       int nruns, hipStream_t st) {
  if (const InferRes fn = infer_res_kernel(a.Dp, a.H)) {
    const int tiles = (n + de::kInferRows - 1) / de::kInferRows;
    const size_t lds = (size_t)de::kInferRows * (a.Dp + 8) * 2 +
                       (size_t)de::kInferRows * (a.H + 8) * 2 +
                       (size_t)(a.H / 32) * de::kInferRows * 4;
    hipLaunchKernelGGL(fn,
                       dim3((tiles + de::kResTiles - 1) / de::kResTiles, nruns),
                       dim3(64 * (a.H / 32)), lds, st, a, X, x_stride, n, ldx,
                       y, y_stride, run0);
  } else {
    hipLaunchKernelGGL(de::k_mlp_infer,
                       dim3((n + de::kInferRows - 1) / de::kInferRows, nruns),
                       dim3(256), de::infer_lds_bytes(a.Dp, a.H), st, a, X,
                       x_stride, n, ldx, y, y_stride, run0);
  }
  return FROM_HIP(hipGetLastError());
}

de_status prep_model(de_sur* s, hipStream_t st) {
  const SurArgs a = args_of(s);
  const size_t work = (size_t)a.runs *
                      ((size_t)a.H * a.Dp + (size_t)a.H * a.H);
  hipLaunchKernelGGL(de::k_model_prep, dim3(grid_for(work, 256)), dim3(256), 0,
                     st, a);
  return FROM_HIP(hipGetLastError());
}

de_status train_steps(de_sur* s, int n, hipStream_t st) {
  for (int k = 0; k < n; ++k) {
    s->step += 1;
    SurArgs a = args_of(s);
    a.c1 = (float)(1.0 - std::pow((double)s->sp.beta1, (double)s->step));
    a.c2 = (float)(1.0 - std::pow((double)s->sp.beta2, (double)s->step));
    const size_t lds = de::train_lds_floats(a.Dp, a.H) * 4;
    // D padded to 128 and H = 256 (the configured model): the form with
    // every B value requested at once
    if (a.Dp == 128 && a.H == 256)
      hipLaunchKernelGGL((de::k_train_fwd<32, 64>),
                         dim3(a.B / de::kTrainRows, a.runs), dim3(512), lds,
                         st, a);
    else
      hipLaunchKernelGGL((de::k_train_fwd<0, 0>),
                         dim3(a.B / de::kTrainRows, a.runs), dim3(512), lds,
                         st, a);
    de_status rc = FROM_HIP(hipGetLastError());
    if (rc != DE_OK) return rc;
    const int nblocks = (a.H / 32) * (a.Dp / 32) + (a.H / 32) * (a.H / 32);
    const int wgs = (nblocks + 3) / 4 + (3 * a.H + 1 + 255) / 256;
    // minibatches of 128 and 256: the deep-prefetch product
    if (a.B == 256)
      hipLaunchKernelGGL((de::k_train_grad<128>), dim3(wgs, a.runs),
                         dim3(256), 0, st, a);
    else if (a.B == 128)
      hipLaunchKernelGGL((de::k_train_grad<64>), dim3(wgs, a.runs),
                         dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((de::k_train_grad<0>), dim3(wgs, a.runs), dim3(256),
                         0, st, a);
    rc = FROM_HIP(hipGetLastError());
    if (rc != DE_OK) return rc;
  }
  return DE_OK;
}

de_status comp_eval(const de_sur* s, const float* X, int n, int ldx, float* f,
                    hipStream_t st) {
  if (n == 0) return DE_OK;
  const SurArgs a = args_of(s);
  const size_t lds = de::comp_lds_floats(a.D) * 4;
  hipLaunchKernelGGL(de::k_comp_eval,
                     dim3((n + de::kEvalRows - 1) / de::kEvalRows),
                     dim3(de::kEvalThreads), lds, st, a, X, n, ldx, f);
  return FROM_HIP(hipGetLastError());
}

de_status one_generation(de_sur* s, hipStream_t st) {
  SurArgs a = args_of(s);
  a.use_model = (s->sp.k > 1 && s->gen >= s->sp.warmup_gens) ? 1 : 0;
  s->last_use_model = a.use_model;
  const int per_wg = 4 * de::cand_rows_per_wave(a.D);
  hipLaunchKernelGGL(de::k_sur_cand,
                     dim3((a.NP * a.k + per_wg - 1) / per_wg, a.runs),
                     dim3(256), 0, st, a);
  de_status rc = FROM_HIP(hipGetLastError());
  if (rc != DE_OK) return rc;
  if (a.use_model) {
    const int rows = a.NP * a.k;
    rc = launch_infer(a, a.cand, (size_t)rows * a.ldx, rows, a.ldx, a.pred,
                      (size_t)rows, 0, a.runs, st);
    if (rc != DE_OK) return rc;
  }
  hipLaunchKernelGGL(de::k_sur_select,
                     dim3((a.NP + de::kEvalRows - 1) / de::kEvalRows, a.runs),
                     dim3(de::kEvalThreads), de::comp_lds_floats(a.D) * 4, st,
                     a);
  rc = FROM_HIP(hipGetLastError());
  if (rc != DE_OK) return rc;
  s->gen += 1;
  s->rounds += 1;
  return train_steps(s, s->sp.steps, st);
}

}  // namespace

extern "C" {

DE_API int64_t de_sur_model_size(int32_t D, int32_t hidden) {
  if (D < 1 || hidden < 1) return 0;
  return model_size(D, hidden);
}

DE_API de_status de_sur_workspace_bytes(const de_params* params,
                                        const de_composition* comp,
                                        const de_surrogate_params* sp,
                                        size_t* bytes) {
  if (!bytes) return DE_E_INVAL;
  const de_status rc = check(params, comp, sp);
  if (rc != DE_OK) return rc;
  // the caller's ldx is not known here: rows are sized for D rounded to 4
  *bytes = layout(*params, *comp, *sp, (int)rup(params->D, 4)).total;
  return DE_OK;
}

DE_API de_status de_sur_init(const de_params* params,
                             const de_composition* comp,
                             const de_surrogate_params* sp,
                             const de_buffers* buffers, void* hip_stream,
                             de_sur** out) {
  if (!out || !buffers) return DE_E_INVAL;
  *out = nullptr;
  de_status rc = check(params, comp, sp);
  if (rc != DE_OK) return rc;
  const de_params& p = *params;
  if (buffers->reserved != 0) return DE_E_INVAL;
  if (buffers->ldx != (int32_t)rup(p.D, 4)) return DE_E_INVAL;
  for (int b = 0; b < 2; ++b) {
    if (!buffers->pop[b] || !buffers->fit[b]) return DE_E_INVAL;
    if (reinterpret_cast<uintptr_t>(buffers->pop[b]) % 16 ||
        reinterpret_cast<uintptr_t>(buffers->fit[b]) % 4)
      return DE_E_INVAL;
  }
  if (buffers->pop[0] == buffers->pop[1] || buffers->fit[0] == buffers->fit[1])
    return DE_E_INVAL;
  const SLayout L = layout(p, *comp, *sp, buffers->ldx);
  if (!buffers->work || reinterpret_cast<uintptr_t>(buffers->work) % 256 ||
      buffers->work_bytes < L.total)
    return DE_E_INVAL;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  rc = set_lds_attributes();
  if (rc != DE_OK) return rc;
  de_sur* s = new (std::nothrow) de_sur();
  if (!s) return DE_E_NOMEM;
  s->p = p;
  s->sp = *sp;
  s->n = comp->n;
  s->sigma = comp->sigma;
  s->ldx = buffers->ldx;
  for (int b = 0; b < 2; ++b) {
    s->pop[b] = buffers->pop[b];
    s->fit[b] = buffers->fit[b];
  }
  s->work = static_cast<char*>(buffers->work);
  s->L = L;
  auto fail = [&](de_status e) {
    delete s;
    return e;
  };
  SurArgs a = args_of(s);
  // composition data
  hipLaunchKernelGGL(de::k_comp_prep,
                     dim3(grid_for((size_t)comp->n * p.D * p.D, 256)),
                     dim3(256), 0, st, comp->O, comp->R, comp->ldr, comp->n,
                     p.D, const_cast<float*>(a.O), const_cast<float*>(a.Rt));
  rc = FROM_HIP(hipGetLastError());
  if (rc == DE_OK)
    rc = FROM_HIP(hipMemcpyAsync(const_cast<float*>(a.bias), comp->bias,
                                 4 * (size_t)comp->n, hipMemcpyHostToDevice,
                                 st));
  // generation 0 (the per-problem initialisation kernel, same draws)
  if (rc == DE_OK) {
    de::GenArgs g{};
    g.pop_next = s->pop[0];
    g.runs = p.runs;
    g.NP = p.NP;
    g.D = p.D;
    g.ldx = s->ldx;
    g.nrows = p.runs * p.NP;
    g.lo = p.lo;
    g.hi = p.hi;
    g.key_lo = (uint32_t)p.seed;
    g.key_hi = (uint32_t)(p.seed >> 32);
    rc = FROM_HIP(de::launch_init(g, st));
  }
  if (rc == DE_OK)
    rc = comp_eval(s, s->pop[0], p.runs * p.NP, s->ldx, s->fit[0], st);
  if (rc == DE_OK) {
    hipLaunchKernelGGL(de::k_archive_init,
                       dim3(grid_for((size_t)p.runs * p.NP * ((p.D + 3) / 4),
                                     256)),
                       dim3(256), 0, st, a);
    rc = FROM_HIP(hipGetLastError());
  }
  if (rc == DE_OK) {
    hipLaunchKernelGGL(de::k_sur_reset, dim3(grid_for(p.runs, 256)),
                       dim3(256), 0, st, a);
    rc = FROM_HIP(hipGetLastError());
  }
  if (rc == DE_OK) {
    hipLaunchKernelGGL(de::k_sur_best, dim3(p.runs), dim3(256), 0, st, a);
    rc = FROM_HIP(hipGetLastError());
  }
  if (rc == DE_OK) {
    const int P = (int)model_size(p.D, sp->hidden);
    hipLaunchKernelGGL(de::k_model_init,
                       dim3(grid_for((size_t)p.runs * L.pstride, 256)),
                       dim3(256), 0, st, a, P);
    rc = FROM_HIP(hipGetLastError());
  }
  if (rc == DE_OK) rc = prep_model(s, st);
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  if (rc != DE_OK) return fail(rc);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    live_set().insert(s);
  }
  *out = s;
  return DE_OK;
}

DE_API de_status de_sur_generation(de_sur* s, int32_t n_gens,
                                   void* hip_stream) {
  if (!live(s)) return DE_E_STATE;
  if (n_gens < 0) return DE_E_INVAL;
  if (s->gen + n_gens >= ((int64_t)1 << 32)) return DE_E_INVAL;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  for (int g = 0; g < n_gens; ++g) {
    const de_status rc = one_generation(s, st);
    if (rc != DE_OK) return rc;
  }
  return DE_OK;
}

DE_API de_status de_sur_read(de_sur* s, void* hip_stream, double* best_f,
                             int32_t* best_idx, int64_t* accepted) {
  if (!live(s)) return DE_E_STATE;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const size_t n = (size_t)s->p.runs;
  std::vector<unsigned long long> key(n), acc(n);
  de_status rc = FROM_HIP(hipMemcpyAsync(key.data(), s->work + s->L.best,
                                         8 * n, hipMemcpyDeviceToHost, st));
  if (rc == DE_OK)
    rc = FROM_HIP(hipMemcpyAsync(acc.data(), s->work + s->L.acc, 8 * n,
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
  }
  return DE_OK;
}

DE_API de_status de_sur_get_generation(const de_sur* s, int64_t* gen) {
  if (!live(s)) return DE_E_STATE;
  if (!gen) return DE_E_INVAL;
  *gen = s->gen;
  return DE_OK;
}

DE_API de_status de_sur_eval(de_sur* s, const float* x_dev, int32_t n,
                             int32_t ldx, float* f_dev, void* hip_stream) {
  if (!live(s)) return DE_E_STATE;
  if (n < 0 || (n > 0 && (!x_dev || !f_dev)) || ldx < s->p.D || ldx % 4)
    return DE_E_INVAL;
  (void)hipGetLastError();
  return comp_eval(s, x_dev, n, ldx, f_dev,
                   reinterpret_cast<hipStream_t>(hip_stream));
}

DE_API de_status de_sur_predict(de_sur* s, int32_t run, const float* x_dev,
                                int32_t n, int32_t ldx, float* y_dev,
                                void* hip_stream) {
  if (!live(s)) return DE_E_STATE;
  if (run < 0 || run >= s->p.runs || n < 0 || ldx < s->p.D ||
      (n > 0 && (!x_dev || !y_dev)))
    return DE_E_INVAL;
  if (n == 0) return DE_OK;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const SurArgs a = args_of(s);
  return launch_infer(a, x_dev, 0, n, ldx, y_dev, 0, run, 1, st);
}

DE_API de_status de_sur_get_model(de_sur* s, void* hip_stream, float* theta,
                                  float* m, float* v, int64_t* step) {
  if (!live(s)) return DE_E_STATE;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const size_t P = (size_t)model_size(s->p.D, s->sp.hidden);
  float* dst[3] = {theta, m, v};
  const size_t src[3] = {s->L.theta, s->L.m, s->L.v};
  de_status rc = DE_OK;
  for (int q = 0; q < 3 && rc == DE_OK; ++q) {
    if (!dst[q]) continue;
    for (int r = 0; r < s->p.runs && rc == DE_OK; ++r)
      rc = FROM_HIP(hipMemcpyAsync(
          dst[q] + (size_t)r * P,
          s->work + src[q] + 4 * (size_t)r * s->L.pstride, 4 * P,
          hipMemcpyDeviceToHost, st));
  }
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  if (rc == DE_OK && step) *step = s->step;
  return rc;
}

DE_API de_status de_sur_set_model(de_sur* s, void* hip_stream,
                                  const float* theta, const float* m,
                                  const float* v, int64_t step) {
  if (!live(s)) return DE_E_STATE;
  if (!theta || !m || !v || step < 0 || step >= ((int64_t)1 << 32))
    return DE_E_INVAL;
  const size_t P = (size_t)model_size(s->p.D, s->sp.hidden);
  const size_t n = P * s->p.runs;
  for (size_t t = 0; t < n; ++t)
    if (!std::isfinite(theta[t]) || !std::isfinite(m[t]) ||
        !std::isfinite(v[t]) || v[t] < 0.f)
      return DE_E_INVAL;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const float* srcs[3] = {theta, m, v};
  const size_t dst[3] = {s->L.theta, s->L.m, s->L.v};
  de_status rc = DE_OK;
  for (int q = 0; q < 3 && rc == DE_OK; ++q)
    for (int r = 0; r < s->p.runs && rc == DE_OK; ++r)
      rc = FROM_HIP(hipMemcpyAsync(
          s->work + dst[q] + 4 * (size_t)r * s->L.pstride,
          srcs[q] + (size_t)r * P, 4 * P, hipMemcpyHostToDevice, st));
  if (rc == DE_OK) rc = prep_model(s, st);
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  if (rc == DE_OK) s->step = step;
  return rc;
}

DE_API de_status de_sur_train(de_sur* s, int32_t n_steps, void* hip_stream) {
  if (!live(s)) return DE_E_STATE;
  if (n_steps < 0) return DE_E_INVAL;
  (void)hipGetLastError();
  return train_steps(s, n_steps, reinterpret_cast<hipStream_t>(hip_stream));
}

DE_API de_status de_sur_get_archive(de_sur* s, void* hip_stream, float* X,
                                    float* T, int64_t* filled) {
  if (!live(s)) return DE_E_STATE;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const size_t cap = (size_t)s->sp.archive, R = (size_t)s->p.runs;
  de_status rc = DE_OK;
  if (X)
    rc = FROM_HIP(hipMemcpy2DAsync(X, 4 * (size_t)s->p.D, s->work + s->L.ax,
                                   4 * (size_t)s->ldx, 4 * (size_t)s->p.D,
                                   R * cap, hipMemcpyDeviceToHost, st));
  if (rc == DE_OK && T)
    rc = FROM_HIP(hipMemcpyAsync(T, s->work + s->L.at, 4 * R * cap,
                                 hipMemcpyDeviceToHost, st));
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  if (rc == DE_OK && filled)
    for (size_t r = 0; r < R; ++r)
      filled[r] = std::min<int64_t>(s->sp.archive, s->rounds * s->p.NP);
  return rc;
}

DE_API de_status de_sur_last(de_sur* s, void* hip_stream, float* cand,
                             float* pred, int32_t* choice) {
  if (!live(s)) return DE_E_STATE;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const size_t R = (size_t)s->p.runs, NP = (size_t)s->p.NP,
               k = (size_t)s->sp.k;
  de_status rc = DE_OK;
  if (cand)
    rc = FROM_HIP(hipMemcpy2DAsync(cand, 4 * (size_t)s->p.D,
                                   s->work + s->L.cand, 4 * (size_t)s->ldx,
                                   4 * (size_t)s->p.D, R * NP * k,
                                   hipMemcpyDeviceToHost, st));
  if (rc == DE_OK && pred)
    rc = FROM_HIP(hipMemcpyAsync(pred, s->work + s->L.pred, 4 * R * NP * k,
                                 hipMemcpyDeviceToHost, st));
  if (rc == DE_OK && choice)
    rc = FROM_HIP(hipMemcpyAsync(choice, s->work + s->L.choice, 4 * R * NP,
                                 hipMemcpyDeviceToHost, st));
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  return rc;
}

DE_API de_status de_sur_destroy(de_sur* s) {
  if (!live(s)) return DE_E_STATE;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    live_set().erase(s);
  }
  s->magic = 0;
  delete s;
  return DE_OK;
}

}  // extern "C"
