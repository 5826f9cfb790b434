/*
 * de_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, scalar FP64 reference of DE/rand/1/bin as defined in
 * Janssen, Pullan & Liew, "GPU Based Differential Evolution: New Insights and
 * Comparative Study" (arXiv 2405.16551), Section 2 (eqs. 2 and 3 and the
 * selection rule stated with them), with the benchmark transform of
 * Section 7.3.1 (shift y = x - o, rotation z = M y, search box [-100, 100]).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file.  It shares no code with the GPU library: the Philox
 * generator, the index sampler and every piece of arithmetic below are
 * written here independently.
 *
 * Readings of points the paper leaves open (each one is listed in the design
 * notes of the repository):
 *   - random numbers come from Philox4x32-10 (Salmon, Moraes, Dror & Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11), one stream per
 *     (tag, run, generation, individual, dimension group);
 *   - rand_j of eq. 3 lives on the 24-bit lattice {k * 2^-24}; the test
 *     rand_j <= CR is done exactly in integers;
 *   - the three mutually exclusive donors of eq. 2 come from a
 *     rejection-free "skip" map over uniform integers;
 *   - a mutant coordinate outside the box is clamped back onto it;
 *   - selection keeps the target on ties (strict "better") and on NaN;
 *   - generations are synchronous: every donor comes from generation g.
 *
 * Precision: every floating-point step is FP64 (the paper fixes none).
 * Summation runs in index order j = 0 .. D-1.
 *
 * Parity unpinned: the jDE constants (Brest et al.'s; the paper prints
 * none) and the surrogate's network and training configuration (not in
 * the paper).  Every other function is pinned by the tests against the
 * mathematics or an independent implementation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11): a 4x32-bit counter, a 2x32-bit key,
 * ten rounds of two 32x32->64 multiplies, key bumped by the Weyl constants
 * (golden ratio and sqrt(3)-1, as 32-bit fractions) between rounds.        */
#define OR_PHILOX_M0 0xD2511F53u
#define OR_PHILOX_M1 0xCD9E8D57u
#define OR_PHILOX_W0 0x9E3779B9u
#define OR_PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += OR_PHILOX_W0;
      k1 += OR_PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)OR_PHILOX_M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)OR_PHILOX_M1 * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Batch form for the tests: n counters/keys laid out [n][4] and [n][2]. */
void oracle_philox_batch(const uint32_t* ctr, const uint32_t* key,
                         uint32_t* out, int64_t n) {
  for (int64_t t = 0; t < n; ++t)
    oracle_philox4x32_10(ctr + 4 * t, key + 2 * t, out + 4 * t);
}

enum { OR_TAG_INIT = 1, OR_TAG_IDX = 2, OR_TAG_XOVER = 3, OR_TAG_JDE = 4 };

/* The four words drawn for (tag, run, gen, individual i, group q).
 * key = the 64-bit seed split into two words; counter = (q, i, gen,
 * tag << 24 | run).                                                       */
static void or_draw(uint64_t seed, int tag, uint32_t run, uint32_t gen,
                    uint32_t i, uint32_t q, uint32_t w[4]) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {q, i, gen, ((uint32_t)tag << 24) | run};
  oracle_philox4x32_10(ctr, key, w);
}

/* Uniform integer in [0, n): the high word of w * n (multiply-shift). */
uint32_t oracle_uniform_index(uint32_t w, uint32_t n) {
  return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

/* ---------------------------------------------------------------------- */
/* Mutually exclusive donors for eq. 2: r1, r2, r3 all distinct and all
 * different from the target i.  a, b, c are uniform in [0, NP-1),
 * [0, NP-2), [0, NP-3).  Each value is mapped onto the integers of [0, NP)
 * that are not yet taken by stepping over the taken ones in ascending
 * order, which is a bijection between the (a, b, c) box and the ordered
 * triples of distinct indices other than i.                               */
static int or_skip(int v, const int* taken, int ntaken) {
  /* taken[] must be sorted ascending */
  for (int t = 0; t < ntaken; ++t)
    if (v >= taken[t]) ++v;
  return v;
}

static void or_sort(int* a, int n) {
  for (int s = 1; s < n; ++s)
    for (int t = s; t > 0 && a[t - 1] > a[t]; --t) {
      int tmp = a[t]; a[t] = a[t - 1]; a[t - 1] = tmp;
    }
}

void oracle_skip_triple(int i, int a, int b, int c, int32_t out[3]) {
  int taken[3];
  taken[0] = i;
  int r1 = or_skip(a, taken, 1);
  taken[1] = r1;
  or_sort(taken, 2);
  int r2 = or_skip(b, taken, 2);
  taken[2] = r2;
  or_sort(taken, 3);
  int r3 = or_skip(c, taken, 3);
  out[0] = r1; out[1] = r2; out[2] = r3;
}

/* r1, r2, r3 and j_rand of individual i in generation gen (eqs. 2, 3). */
void oracle_draw_indices(uint64_t seed, int run, int64_t gen, int i, int NP,
                         int D, int32_t out[4]) {
  uint32_t w[4];
  or_draw(seed, OR_TAG_IDX, (uint32_t)run, (uint32_t)gen, (uint32_t)i, 0u, w);
  int a = (int)oracle_uniform_index(w[0], (uint32_t)(NP - 1));
  int b = (int)oracle_uniform_index(w[1], (uint32_t)(NP - 2));
  int c = (int)oracle_uniform_index(w[2], (uint32_t)(NP - 3));
  oracle_skip_triple(i, a, b, c, out);
  out[3] = (int32_t)oracle_uniform_index(w[3], (uint32_t)D);
}

/* Threshold for "rand_j <= CR" on the 24-bit lattice rand_j = k * 2^-24:
 * k * 2^-24 <= CR  <=>  k <= floor(CR * 2^24).  CR * 2^24 is exact.      */
static uint32_t or_cr_threshold(double CR) {
  return (uint32_t)floor(CR * 16777216.0);
}

/* Does the trial take the mutant's coordinate j (eq. 3)? */
int oracle_take_mutant(uint64_t seed, int run, int64_t gen, int i, int j,
                       int jrand, double CR) {
  if (j == jrand) return 1;
  uint32_t w[4];
  or_draw(seed, OR_TAG_XOVER, (uint32_t)run, (uint32_t)gen, (uint32_t)i,
          (uint32_t)(j >> 2), w);
  uint32_t k = w[j & 3] >> 8;
  return k <= or_cr_threshold(CR);
}

/* ---------------------------------------------------------------------- */
/* Objectives of Section 7.3.1: y = x - o; sphere f = sum y_j^2; rotated
 * oscillating f = sum_i z_i^2 + sin^2(3 z_i) with z = R y, R row-major
 * [D][D] (z_i = sum_j R[i][j] y_j).                                        */
enum { OR_OBJ_SPHERE = 0, OR_OBJ_ROT_OSC = 1 };

double oracle_objective(int kind, int D, const double* x, const double* o,
                        const double* R) {
  if (kind == OR_OBJ_SPHERE) {
    double f = 0.0;
    for (int j = 0; j < D; ++j) {
      double y = x[j] - o[j];
      f += y * y;
    }
    return f;
  }
  double f = 0.0;
  for (int r = 0; r < D; ++r) {
    double z = 0.0;
    for (int j = 0; j < D; ++j) z += R[(size_t)r * D + j] * (x[j] - o[j]);
    double s = sin(3.0 * z);
    f += z * z + s * s;
  }
  return f;
}

void oracle_objective_batch(int kind, int D, int64_t n, const double* x,
                            const double* o, const double* R, double* f,
                            int nthreads) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int64_t t = 0; t < n; ++t)
    f[t] = oracle_objective(kind, D, x + t * D, o, R);
  (void)nthreads;
}

/* ---------------------------------------------------------------------- */
/* Population initialisation (Section 2): x_ij uniform in the box,
 * x_ij = lo + u (hi - lo) with u = k * 2^-24 from the INIT stream, then
 * every individual is evaluated.  pop is [runs][NP][D]; run r of the array
 * uses run number run0 + r in the draw counter.                            */
void oracle_init(int runs, int run0, int NP, int D, double lo, double hi,
                 uint64_t seed, double* pop) {
  for (int r = 0; r < runs; ++r)
    for (int i = 0; i < NP; ++i)
      for (int j = 0; j < D; ++j) {
        uint32_t w[4];
        or_draw(seed, OR_TAG_INIT, (uint32_t)(run0 + r), 0u, (uint32_t)i,
                (uint32_t)(j >> 2), w);
        double u = (double)(w[j & 3] >> 8) * (1.0 / 16777216.0);
        pop[((size_t)r * NP + i) * D + j] = lo + u * (hi - lo);
      }
}

/* ---------------------------------------------------------------------- */
/* One synchronous generation g -> g+1 of DE/rand/1/bin.
 *   mutation   (eq. 2): v = x_r1 + F (x_r2 - x_r3), then clamped to [lo, hi]
 *   crossover  (eq. 3): u_j = v_j if rand_j <= CR or j = j_rand, else x_ij
 *   selection  (Sec. 2): u replaces x iff f(u) < f(x)
 * pop/fit hold generation g; pop_next/fit_next receive g+1.  Optional
 * outputs (NULL to skip): trial [runs][NP][D], ftrial [runs][NP],
 * accept [runs][NP], draws [runs][NP][4].  Run r of the arrays uses run
 * number run0 + r in the draw counters (runs of a larger batch).           */
void oracle_generation(int runs, int run0, int NP, int D, double F, double CR,
                       double lo, double hi, uint64_t seed, int64_t gen, int kind,
                       const double* o, const double* R, const double* pop,
                       const double* fit, double* pop_next, double* fit_next,
                       double* trial, double* ftrial, int32_t* accept,
                       int32_t* draws, int nthreads) {
  int64_t total = (int64_t)runs * NP;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int64_t t = 0; t < total; ++t) {
    int r = (int)(t / NP), i = (int)(t % NP);
    const double* P = pop + (size_t)r * NP * D;
    int32_t d[4];
    oracle_draw_indices(seed, run0 + r, gen, i, NP, D, d);
    const double* x = P + (size_t)i * D;
    const double* x1 = P + (size_t)d[0] * D;
    const double* x2 = P + (size_t)d[1] * D;
    const double* x3 = P + (size_t)d[2] * D;
    double* u = (double*)malloc(sizeof(double) * (size_t)D);
    for (int j = 0; j < D; ++j) {
      if (oracle_take_mutant(seed, run0 + r, gen, i, j, d[3], CR)) {
        double v = x1[j] + F * (x2[j] - x3[j]);
        if (v < lo) v = lo;
        if (v > hi) v = hi;
        u[j] = v;
      } else {
        u[j] = x[j];
      }
    }
    double fu = oracle_objective(kind, D, u, o, R);
    double fx = fit[t];
    int acc = fu < fx;
    double* xn = pop_next + (size_t)t * D;
    memcpy(xn, acc ? u : x, sizeof(double) * (size_t)D);
    fit_next[t] = acc ? fu : fx;
    if (trial) memcpy(trial + (size_t)t * D, u, sizeof(double) * (size_t)D);
    if (ftrial) ftrial[t] = fu;
    if (accept) accept[t] = acc;
    if (draws) memcpy(draws + 4 * t, d, sizeof(d));
    free(u);
  }
  (void)nthreads;
}

/* ---------------------------------------------------------------------- */
/* jDE: control parameters adapted per individual (listed among the DE
 * variants of Section 2; the GPU code cujDE of Section 8.2).  The rule and
 * its constants are those of Brest, Greiner, Boskovic, Mernik & Zumer,
 * "Self-adapting control parameters in differential evolution" (IEEE TEVC
 * 2006), not of the paper: the constants are parity unpinned against the
 * paper (the tests pin only the rule's structure).  Before building its
 * trial, individual i draws
 * four uniforms u1..u4 (one Philox block, tag 4, group 0) and takes
 *     F'  = F_lo + u1 * F_span   if u2 < tau_F,   else F_i
 *     CR' = u3                   if u4 < tau_CR,  else CR_i
 * The trial uses F' and CR' in eqs. 2 and 3; when it replaces the target,
 * F' and CR' replace F_i and CR_i, otherwise they are dropped.
 * Readings: u = (w >> 8) * 2^-24 as in eq. 3; "u < tau" is decided as
 * (w >> 8) < floor(tau * 2^24); control values are FP32 numbers: F' is
 * F_lo + u1 F_span (computed exactly in FP64: u1 and F_span are 24-bit
 * values and F_lo a float, so the sum needs fewer than 53 bits) rounded
 * once to FP32, CR' = u3 is exact.  F and CR arrays are [runs][NP]; Fp/CRp
 * (nullable) receive the F' and CR' each trial used.                      */
static float or_round_float(double v) { return (float)v; }

void oracle_jde_generation(int runs, int run0, int NP, int D, double F_lo,
                           double F_span, double tau_F, double tau_CR,
                           double lo, double hi, uint64_t seed, int64_t gen,
                           int kind, const double* o, const double* R,
                           const double* pop, const double* fit,
                           const double* F, const double* CR,
                           double* pop_next, double* fit_next,
                           double* F_next, double* CR_next, double* trial,
                           double* ftrial, int32_t* accept, double* Fp,
                           double* CRp, int nthreads) {
  const uint32_t tF = (uint32_t)floor(tau_F * 16777216.0);
  const uint32_t tCR = (uint32_t)floor(tau_CR * 16777216.0);
  int64_t total = (int64_t)runs * NP;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int64_t t = 0; t < total; ++t) {
    int r = (int)(t / NP), i = (int)(t % NP);
    const double* P = pop + (size_t)r * NP * D;
    uint32_t w[4];
    or_draw(seed, OR_TAG_JDE, (uint32_t)(run0 + r), (uint32_t)gen,
            (uint32_t)i, 0u, w);
    double Fi = F[t], CRi = CR[t];
    if ((w[1] >> 8) < tF)
      Fi = (double)or_round_float(F_lo + (double)(w[0] >> 8) *
                                             (1.0 / 16777216.0) * F_span);
    if ((w[3] >> 8) < tCR) CRi = (double)(w[2] >> 8) * (1.0 / 16777216.0);
    int32_t d[4];
    oracle_draw_indices(seed, run0 + r, gen, i, NP, D, d);
    const double* x = P + (size_t)i * D;
    const double* x1 = P + (size_t)d[0] * D;
    const double* x2 = P + (size_t)d[1] * D;
    const double* x3 = P + (size_t)d[2] * D;
    double* u = (double*)malloc(sizeof(double) * (size_t)D);
    for (int j = 0; j < D; ++j) {
      if (oracle_take_mutant(seed, run0 + r, gen, i, j, d[3], CRi)) {
        double v = x1[j] + Fi * (x2[j] - x3[j]);
        if (v < lo) v = lo;
        if (v > hi) v = hi;
        u[j] = v;
      } else {
        u[j] = x[j];
      }
    }
    double fu = oracle_objective(kind, D, u, o, R);
    double fx = fit[t];
    int acc = fu < fx;
    memcpy(pop_next + (size_t)t * D, acc ? u : x, sizeof(double) * (size_t)D);
    fit_next[t] = acc ? fu : fx;
    F_next[t] = acc ? Fi : F[t];
    CR_next[t] = acc ? CRi : CR[t];
    if (trial) memcpy(trial + (size_t)t * D, u, sizeof(double) * (size_t)D);
    if (ftrial) ftrial[t] = fu;
    if (accept) accept[t] = acc;
    if (Fp) Fp[t] = Fi;
    if (CRp) CRp[t] = CRi;
    free(u);
  }
  (void)nthreads;
}

/* ---------------------------------------------------------------------- */
/* A whole run (Section 2 loop; Section 7.3.4 bookkeeping): initialise,
 * evaluate, then G generations.  Records per run the best value after each
 * generation (best_trace [runs][G+1], entry 0 = after initialisation), the
 * first generation whose best is <= target (hit_gen [runs], -1 if never),
 * and the number of accepted trials (accepted [runs]).  pop_out/fit_out
 * (nullable) receive the final population.                                */
int oracle_run(int runs, int NP, int D, double F, double CR, double lo,
               double hi, uint64_t seed, int kind, const double* o,
               const double* R, int64_t G, double target, double* best_trace,
               int64_t* hit_gen, int64_t* accepted, double* pop_out,
               double* fit_out, int nthreads) {
  size_t n = (size_t)runs * NP;
  double* pa = (double*)malloc(sizeof(double) * n * D);
  double* pb = (double*)malloc(sizeof(double) * n * D);
  double* fa = (double*)malloc(sizeof(double) * n);
  double* fb = (double*)malloc(sizeof(double) * n);
  int32_t* acc = (int32_t*)malloc(sizeof(int32_t) * n);
  if (!pa || !pb || !fa || !fb || !acc) {
    free(pa); free(pb); free(fa); free(fb); free(acc);
    return 1;
  }
  oracle_init(runs, 0, NP, D, lo, hi, seed, pa);
  oracle_objective_batch(kind, D, (int64_t)n, pa, o, R, fa, nthreads);
  for (int r = 0; r < runs; ++r) {
    hit_gen[r] = -1;
    accepted[r] = 0;
  }
  for (int64_t g = 0; g <= G; ++g) {
    if (g > 0) {
      oracle_generation(runs, 0, NP, D, F, CR, lo, hi, seed, g - 1, kind, o, R,
                        pa, fa, pb, fb, NULL, NULL, acc, NULL, nthreads);
      double* t = pa; pa = pb; pb = t;
      t = fa; fa = fb; fb = t;
      for (size_t k = 0; k < n; ++k) accepted[k / NP] += acc[k];
    }
    for (int r = 0; r < runs; ++r) {
      double best = fa[(size_t)r * NP];
      for (int i = 1; i < NP; ++i)
        if (fa[(size_t)r * NP + i] < best) best = fa[(size_t)r * NP + i];
      if (best_trace) best_trace[(size_t)r * (G + 1) + g] = best;
      if (hit_gen[r] < 0 && best <= target) hit_gen[r] = g;
    }
  }
  if (pop_out) memcpy(pop_out, pa, sizeof(double) * n * D);
  if (fit_out) memcpy(fit_out, fa, sizeof(double) * n);
  free(pa); free(pb); free(fa); free(fb); free(acc);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Composition objective (Section 7.3.3, composition functions):
 *     f(x) = sum_k omega_k (g_k(x) + bias_k),  omega_k = w_k / sum_j w_j,
 * g_k the rotated oscillating function with shift O[k] and rotation R[k]
 * (D x D row-major, k-th block of R).  Weights, as in the surrogate
 * benchmark configuration: w_k = exp(-d_k / (2 sigma^2)) with
 * d_k = ||x - O[k]||^2 (the paper's 1/sqrt(d_k) factor and the D in the
 * exponent are dropped: the former is singular at x = O[k]).  Every exponent
 * is shifted by min_k d_k, which cancels in the normalisation and keeps the
 * largest weight at 1 (no underflow of all weights far from every O[k]).   */
double oracle_composition(int D, int n, const double* x, const double* O,
                          const double* R, const double* bias, double sigma) {
  double d[64], g[64];
  double dmin = INFINITY;
  for (int k = 0; k < n; ++k) {
    double dk = 0.0;
    for (int j = 0; j < D; ++j) {
      double y = x[j] - O[(size_t)k * D + j];
      dk += y * y;
    }
    d[k] = dk;
    if (dk < dmin) dmin = dk;
    g[k] = oracle_objective(OR_OBJ_ROT_OSC, D, x, O + (size_t)k * D,
                            R + (size_t)k * D * D);
  }
  double wsum = 0.0, f = 0.0;
  for (int k = 0; k < n; ++k) {
    double w = exp(-(d[k] - dmin) / (2.0 * sigma * sigma));
    wsum += w;
    f += w * (g[k] + bias[k]);
  }
  return f / wsum;
}

void oracle_composition_batch(int D, int n, int64_t rows, const double* X,
                              const double* O, const double* R,
                              const double* bias, double sigma, double* f,
                              int nthreads) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int64_t t = 0; t < rows; ++t)
    f[t] = oracle_composition(D, n, X + t * D, O, R, bias, sigma);
  (void)nthreads;
}

/* ---------------------------------------------------------------------- */
/* Surrogate MLP D -> H -> H -> 1 with ReLU (the online-trained fitness
 * model of the surrogate-assisted variant).  Parameters packed as
 *     theta = [W1 (H x D) | b1 (H) | W2 (H x H) | b2 (H) | w3 (H) | b3],
 * W row-major (a = W h).  Input scaled to [-1, 1]:
 * xs_j = (2 x_j - (lo + hi)) / (hi - lo).                                  */
static int64_t or_mlp_size(int D, int H) {
  return (int64_t)H * D + H + (int64_t)H * H + H + H + 1;
}

int64_t oracle_mlp_size(int D, int H) { return or_mlp_size(D, H); }

/* One row: fills h1, h2 (after ReLU) and a1, a2 (before) when non-NULL. */
static double or_mlp_row(int D, int H, const double* th, double lo, double hi,
                         const double* x, double* xs, double* a1, double* h1,
                         double* a2, double* h2) {
  const double* W1 = th;
  const double* b1 = W1 + (size_t)H * D;
  const double* W2 = b1 + H;
  const double* b2 = W2 + (size_t)H * H;
  const double* w3 = b2 + H;
  const double b3 = w3[H];
  for (int j = 0; j < D; ++j) xs[j] = (2.0 * x[j] - (lo + hi)) / (hi - lo);
  for (int i = 0; i < H; ++i) {
    double a = b1[i];
    for (int j = 0; j < D; ++j) a += W1[(size_t)i * D + j] * xs[j];
    a1[i] = a;
    h1[i] = a > 0.0 ? a : 0.0;
  }
  for (int i = 0; i < H; ++i) {
    double a = b2[i];
    for (int j = 0; j < H; ++j) a += W2[(size_t)i * H + j] * h1[j];
    a2[i] = a;
    h2[i] = a > 0.0 ? a : 0.0;
  }
  double y = b3;
  for (int i = 0; i < H; ++i) y += w3[i] * h2[i];
  return y;
}

void oracle_mlp_forward(int D, int H, const double* theta, double lo,
                        double hi, int64_t rows, const double* X, double* y) {
  double* buf = (double*)malloc(sizeof(double) * (size_t)(D + 4 * H));
  for (int64_t t = 0; t < rows; ++t)
    y[t] = or_mlp_row(D, H, theta, lo, hi, X + t * D, buf, buf + D,
                      buf + D + H, buf + D + 2 * H, buf + D + 3 * H);
  free(buf);
}

/* Gradient of the mean squared error L = (1/B) sum_b (y_b - t_b)^2 with
 * respect to theta (same packing), by backpropagation; returns L.         */
double oracle_mlp_grad(int D, int H, const double* theta, double lo,
                       double hi, int B, const double* X, const double* T,
                       double* grad) {
  const int64_t P = or_mlp_size(D, H);
  memset(grad, 0, sizeof(double) * (size_t)P);
  const double* W2 = theta + (size_t)H * D + H;
  const double* w3 = W2 + (size_t)H * H + H;
  double* gW1 = grad;
  double* gb1 = gW1 + (size_t)H * D;
  double* gW2 = gb1 + H;
  double* gb2 = gW2 + (size_t)H * H;
  double* gw3 = gb2 + H;
  double* gb3 = gw3 + H;
  double* buf = (double*)malloc(sizeof(double) * (size_t)(D + 6 * H));
  double* xs = buf;
  double* a1 = xs + D;
  double* h1 = a1 + H;
  double* a2 = h1 + H;
  double* h2 = a2 + H;
  double* d2 = h2 + H;
  double* d1 = d2 + H;
  double loss = 0.0;
  for (int b = 0; b < B; ++b) {
    double y = or_mlp_row(D, H, theta, lo, hi, X + (size_t)b * D, xs, a1, h1,
                          a2, h2);
    double r = y - T[b];
    loss += r * r;
    double e = 2.0 * r / B;
    *gb3 += e;
    for (int i = 0; i < H; ++i) {
      gw3[i] += e * h2[i];
      d2[i] = a2[i] > 0.0 ? e * w3[i] : 0.0;
      gb2[i] += d2[i];
      for (int j = 0; j < H; ++j) gW2[(size_t)i * H + j] += d2[i] * h1[j];
    }
    for (int j = 0; j < H; ++j) {
      double s = 0.0;
      for (int i = 0; i < H; ++i) s += W2[(size_t)i * H + j] * d2[i];
      d1[j] = a1[j] > 0.0 ? s : 0.0;
      gb1[j] += d1[j];
      for (int k = 0; k < D; ++k) gW1[(size_t)j * D + k] += d1[j] * xs[k];
    }
  }
  free(buf);
  return loss / B;
}

/* One Adam step (Kingma & Ba, 2015) on the minibatch (X, T): step counter
 * t >= 1, moments m, v updated in place, bias-corrected update
 * theta -= lr * mhat / (sqrt(vhat) + eps).  Returns the loss before it.   */
double oracle_mlp_adam_step(int D, int H, double* theta, double* m,
                            double* v, int64_t t, double lr, double beta1,
                            double beta2, double eps, double lo, double hi,
                            int B, const double* X, const double* T) {
  const int64_t P = or_mlp_size(D, H);
  double* g = (double*)malloc(sizeof(double) * (size_t)P);
  double loss = oracle_mlp_grad(D, H, theta, lo, hi, B, X, T, g);
  const double c1 = 1.0 - pow(beta1, (double)t);
  const double c2 = 1.0 - pow(beta2, (double)t);
  for (int64_t p = 0; p < P; ++p) {
    m[p] = beta1 * m[p] + (1.0 - beta1) * g[p];
    v[p] = beta2 * v[p] + (1.0 - beta2) * g[p] * g[p];
    theta[p] -= lr * (m[p] / c1) / (sqrt(v[p] / c2) + eps);
  }
  free(g);
  return loss;
}

/* ---------------------------------------------------------------------- */
/* Surrogate-assisted generation: every target i builds k DE/rand/1/bin
 * trials (candidate c draws with individual field i | c << 24 of the
 * counter, so candidate 0 is the plain trial), the surrogate (theta of the
 * run) predicts each candidate's scaled fitness, the candidate with the
 * lowest prediction (lowest c on ties; c = 0 when use_model is 0) is the
 * only one evaluated on the composition objective, and selection is the
 * usual strict comparison.  Outputs as oracle_generation, plus (nullable)
 * cand [runs][NP][k][D], pred [runs][NP][k] and choice [runs][NP].        */
static void or_draw_indices_ctr(uint64_t seed, uint32_t run, int64_t gen,
                                uint32_t ctr_i, int i, int NP, int D,
                                int32_t out[4]) {
  uint32_t w[4];
  or_draw(seed, OR_TAG_IDX, run, (uint32_t)gen, ctr_i, 0u, w);
  int a = (int)oracle_uniform_index(w[0], (uint32_t)(NP - 1));
  int b = (int)oracle_uniform_index(w[1], (uint32_t)(NP - 2));
  int c = (int)oracle_uniform_index(w[2], (uint32_t)(NP - 3));
  oracle_skip_triple(i, a, b, c, out);
  out[3] = (int32_t)oracle_uniform_index(w[3], (uint32_t)D);
}

static int or_take_ctr(uint64_t seed, uint32_t run, int64_t gen,
                       uint32_t ctr_i, int j, int jrand, double CR) {
  if (j == jrand) return 1;
  uint32_t w[4];
  or_draw(seed, OR_TAG_XOVER, run, (uint32_t)gen, ctr_i, (uint32_t)(j >> 2),
          w);
  return (w[j & 3] >> 8) <= or_cr_threshold(CR);
}

void oracle_sur_generation(int runs, int run0, int NP, int D, int k, double F,
                           double CR, double lo, double hi, uint64_t seed,
                           int64_t gen, int use_model, int H,
                           const double* theta, int n, const double* O,
                           const double* R, const double* bias, double sigma,
                           const double* pop, const double* fit,
                           double* pop_next, double* fit_next, double* cand,
                           double* pred, int32_t* choice, double* ftrial,
                           int32_t* accept, int nthreads) {
  const int64_t P = or_mlp_size(D, H);
  int64_t total = (int64_t)runs * NP;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int64_t t = 0; t < total; ++t) {
    int r = (int)(t / NP), i = (int)(t % NP);
    const double* Pp = pop + (size_t)r * NP * D;
    const double* x = Pp + (size_t)i * D;
    double* u = (double*)malloc(sizeof(double) * (size_t)k * D);
    double* buf = (double*)malloc(sizeof(double) * (size_t)(D + 4 * H));
    int best_c = 0;
    double best_p = INFINITY;
    for (int c = 0; c < k; ++c) {
      const uint32_t ci = (uint32_t)i | ((uint32_t)c << 24);
      int32_t d[4];
      or_draw_indices_ctr(seed, (uint32_t)(run0 + r), gen, ci, i, NP, D, d);
      double* uc = u + (size_t)c * D;
      for (int j = 0; j < D; ++j) {
        if (or_take_ctr(seed, (uint32_t)(run0 + r), gen, ci, j, d[3], CR)) {
          double v = Pp[(size_t)d[0] * D + j] +
                     F * (Pp[(size_t)d[1] * D + j] - Pp[(size_t)d[2] * D + j]);
          if (v < lo) v = lo;
          if (v > hi) v = hi;
          uc[j] = v;
        } else {
          uc[j] = x[j];
        }
      }
      double p = 0.0;
      if (use_model)
        p = or_mlp_row(D, H, theta + (size_t)r * P, lo, hi, uc, buf, buf + D,
                       buf + D + H, buf + D + 2 * H, buf + D + 3 * H);
      if (pred) pred[t * k + c] = p;
      if (cand) memcpy(cand + ((size_t)t * k + c) * D, uc, sizeof(double) * D);
      if (use_model && p < best_p) {
        best_p = p;
        best_c = c;
      }
    }
    const double* uc = u + (size_t)best_c * D;
    double fu = oracle_composition(D, n, uc, O, R, bias, sigma);
    double fx = fit[t];
    int acc = fu < fx;
    memcpy(pop_next + (size_t)t * D, acc ? uc : x, sizeof(double) * D);
    fit_next[t] = acc ? fu : fx;
    if (choice) choice[t] = best_c;
    if (ftrial) ftrial[t] = fu;
    if (accept) accept[t] = acc;
    free(u);
    free(buf);
  }
  (void)nthreads;
}

/* Threads the OpenMP runtime would give a parallel region (1 without it). */
int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
