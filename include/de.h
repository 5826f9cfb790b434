/*
 * de.h -- C ABI of the MI355X (gfx950) DE/rand/1/bin library (libde.so).
 *
 * The library runs differential evolution, DE/rand/1/bin, entirely on one
 * GPU, following Section 2 of Janssen, Pullan & Liew, "GPU Based
 * Differential Evolution: New Insights and Comparative Study" (arXiv
 * 2405.16551): random initialisation in the search box, DE/rand/1 mutation
 * (eq. 2), binomial crossover (eq. 3) and greedy one-to-one selection, over
 * `runs` independent populations of NP individuals with D parameters each.
 * Objectives follow the benchmark transform of Section 7.3.1: minimise
 * f(x) over the box, with y = x - o (shift) and z = R y (rotation).
 *
 * Conventions shared by every entry point:
 *   - Every call returns de_status (DE_OK = 0) unless stated otherwise.
 *   - Device pointers are plain HIP device addresses.  They are owned by the
 *     caller; the library never allocates, frees or retains device memory
 *     beyond the lifetime the caller gives it.  The only library-owned object
 *     is the opaque host-side de_state handle.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  Launches
 *     are asynchronous on that stream.  Argument checks are synchronous and
 *     happen before any launch: an invalid call leaves the device untouched.
 *   - Asynchronous device faults surface at the next synchronising call
 *     (de_best, de_evolve, de_read_stats) as DE_E_DEVICE.
 *   - A handle is not thread-safe; distinct handles are independent.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit
 * seed, counter = (q, i, gen, tag << 24 | run).  Every draw is therefore a
 * pure function of (seed, run, generation, individual, dimension), so
 * results do not depend on launch shape, on how generations are split
 * across calls, or on checkpoint/restart.
 */
#ifndef DE_MI355X_DE_H_
#define DE_MI355X_DE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DE_ABI_VERSION 1

#if defined(DE_BUILDING_LIBRARY)
#define DE_API __attribute__((visibility("default")))
#else
#define DE_API
#endif

typedef enum de_status {
  DE_OK = 0,
  DE_E_INVAL = 1,       /* an argument is out of range or inconsistent     */
  DE_E_NOMEM = 2,       /* host allocation of the handle failed            */
  DE_E_DEVICE = 3,      /* a HIP call or a kernel failed                   */
  DE_E_STATE = 4,       /* NULL / destroyed handle, or wrong call order    */
  DE_E_UNSUPPORTED = 5  /* valid, but beyond what the library implements  */
} de_status;

/* Objective kinds (Section 7.3.1 transform; minimisation, optimum f = 0 at
 * x = o).
 *   DE_OBJ_SPHERE : f(x) = sum_j (x_j - o_j)^2                (separable)
 *   DE_OBJ_ROT_OSC: z = R (x - o);  f(x) = sum_i z_i^2 + sin^2(3 z_i)     */
typedef enum de_obj_kind { DE_OBJ_SPHERE = 0, DE_OBJ_ROT_OSC = 1 } de_obj_kind;

/* Arithmetic of the rotation product z = R y (DE_OBJ_ROT_OSC only).
 *   DE_GEMM_FP32: FP32 operands, FP32 accumulation (MFMA f32).
 *   DE_GEMM_BF16: y and R rounded to BF16 (nearest-even), FP32 accumulation
 *                 (MFMA bf16).  Everything else stays FP32.                */
typedef enum de_gemm_prec { DE_GEMM_FP32 = 0, DE_GEMM_BF16 = 1 } de_gemm_prec;

/* DE control parameters (Section 2).
 *   runs  >= 1 independent populations, evolved side by side; they share the
 *         objective and seed and differ in the counter's run field (< 2^24).
 *   NP    >= 4 individuals per population (eq. 2 needs three donors that
 *         differ from each other and from the target).
 *   D     >= 1 parameters per individual.
 *   F     differential weight of eq. 2, finite and > 0.
 *   CR    crossover rate of eq. 3, in [0, 1]; rand_j is drawn on the 24-bit
 *         lattice k * 2^-24 and compared exactly.
 *   lo,hi finite search box, lo < hi; initial values are uniform in
 *         [lo, hi) and mutant coordinates are clamped to [lo, hi].
 *   seed  64-bit Philox key.                                                */
typedef struct de_params {
  int32_t runs;
  int32_t NP;
  int32_t D;
  float F;
  float CR;
  float lo;
  float hi;
  uint64_t seed;
} de_params;

/* The objective.  `o` is a device array of D floats.  For DE_OBJ_ROT_OSC,
 * `R` is a device array of D rows of `ldr` floats, row-major, z_i = sum_j
 * R[i*ldr + j] y_j, ldr >= D; the library reads R (and converts it to the
 * GEMM operand layout inside the workspace) during de_init_population only,
 * stream-ordered, so R may be released once that work has run.  `o` is
 * likewise copied into the workspace during de_init_population.  For
 * DE_OBJ_SPHERE, R is ignored (may be NULL) and gemm_prec is ignored.       */
typedef struct de_objective {
  int32_t kind;       /* de_obj_kind  */
  int32_t gemm_prec;  /* de_gemm_prec */
  int32_t ldr;
  int32_t reserved;   /* must be 0    */
  const float* o;
  const float* R;
} de_objective;

/* Caller-owned device buffers.
 *   pop[0], pop[1]: two populations, each runs * NP rows of ldx floats
 *                   (row (r, i) starts at element (r * NP + i) * ldx).
 *                   ldx >= D, ldx % 4 == 0, both pointers 16-byte aligned.
 *                   Generation g lives in pop[g & 1] (ping-pong).
 *   fit[0], fit[1]: runs * NP floats each, the objective of the matching row.
 *                   Between calls the library owns the contents of both
 *                   population buffers: a step may leave a row of the
 *                   buffer it writes untouched when that buffer already
 *                   holds the row's new value, so callers change populations
 *                   only through de_load_population.
 *   work          : scratch of at least de_workspace_bytes() bytes,
 *                   256-byte aligned; holds per-run statistics and, for
 *                   rotated objectives, R in the GEMM operand layout.  Its
 *                   contents must be preserved between calls on a handle.   */
typedef struct de_buffers {
  float* pop[2];
  float* fit[2];
  int32_t ldx;
  int32_t reserved;   /* must be 0 */
  void* work;
  size_t work_bytes;
} de_buffers;

typedef struct de_state de_state; /* opaque; owned by the library */

/* Library ABI version (DE_ABI_VERSION of the build).  Never fails. */
DE_API int32_t de_abi_version(void);

/* Static description of a status code.  Never returns NULL. */
DE_API const char* de_strerror(de_status status);

/* Bytes of device workspace needed for (params, objective).  Pure host
 * computation.  DE_E_INVAL on bad arguments, DE_E_UNSUPPORTED for sizes the
 * library's kernels do not cover.                                         */
DE_API de_status de_workspace_bytes(const de_params* params,
                             const de_objective* objective, size_t* bytes);

/* Create a handle and generation 0 (Section 2, population initialisation):
 * x_ij = lo + u (hi - lo), u uniform on the 24-bit lattice of [0, 1), into
 * pop[0]; then evaluate every individual into fit[0]; reset the statistics
 * (best, first-hit generation, accepted counts).  On success *out is a new
 * handle at generation 0.  Asynchronous on hip_stream.                     */
DE_API de_status de_init_population(const de_params* params,
                             const de_objective* objective,
                             const de_buffers* buffers, void* hip_stream,
                             de_state** out);

/* Advance n_gens >= 0 generations (Section 2 loop; eq. 2 mutation with
 * clamping, eq. 3 crossover, greedy selection: the trial replaces the target
 * iff f(trial) < f(target), so ties and NaN keep the target).  Synchronous
 * generations: every donor comes from generation g.  Asynchronous.
 * Calls of at least 16 generations on rotated problems with two or more
 * runs and at least one 64-row tile per compute unit run as two run groups
 * on two streams that such handles create at initialisation (ordered after,
 * and waited for by, hip_stream through events; released by de_destroy),
 * the second group offset by half the time per generation measured on an
 * earlier call, so that one group's trial build overlaps the other's
 * rotation product.  The results are identical to one launch per
 * generation; the environment variable DE_STAGGER=0 turns the split off,
 * and so does a hip_stream that is being captured into a graph.          */
DE_API de_status de_generation(de_state* state, int32_t n_gens, void* hip_stream);

/* Run until every run's best value is <= target or max_gens further
 * generations have run (Section 7.3.4: budget or error threshold).  The
 * generations are queued in chunks of check_every (>= 1); behind each
 * chunk the device's count of runs at the target is copied to pinned host
 * memory (the solution-found flag of Section 8, copied asynchronously), and
 * the next chunk is queued before the host reads the previous chunk's
 * count, so the device does not wait on the host between chunks.  The call
 * therefore stops at most one chunk after the chunk in which the last run
 * reached the target: with h the generation at which every run had hit,
 * gens_done <= h + 2 * check_every - 1 (counted from the call's start), and
 * no generation is run when every run is at the target already.  The
 * first-hit generation is recorded on the device and is exact whatever
 * check_every is.  *gens_done receives the number of generations run by
 * this call; hit_gen (nullable, runs entries) receives per run the first
 * generation at which the best was <= target, or -1.  The handle keeps two
 * pinned host words and two events for the polling from its first
 * de_evolve call until de_destroy.  Synchronises hip_stream.               */
DE_API de_status de_evolve(de_state* state, int64_t max_gens, double target,
                    int32_t check_every, void* hip_stream, int64_t* gens_done,
                    int64_t* hit_gen);

/* Best individual of one run in the current generation: lowest f, ties to
 * the lowest index.  x_host (nullable, D floats), f_host, idx_host
 * (nullable) are host pointers.  Synchronises hip_stream.                  */
DE_API de_status de_best(de_state* state, int32_t run, void* hip_stream,
                  float* x_host, double* f_host, int32_t* idx_host);

/* jDE: DE/rand/1/bin whose F and CR are adapted per individual (listed
 * among the DE variants of Section 2; the GPU code cujDE compared in
 * Section 8.2).  The rule is that of Brest, Greiner, Boskovic, Mernik and
 * Zumer (IEEE TEVC 2006): before building its trial, individual i takes
 *     F' = F_lo + u1 F_span   with probability tau_F,   else its F,
 *     CR' = u3                with probability tau_CR,  else its CR,
 * with u on the 2^-24 lattice from Philox (tag 4, group 0 of (i, gen)); the
 * trial uses F' and CR' in eqs. 2 and 3, and they replace the individual's
 * values only if the trial replaces it.  Brest et al. use F_lo = 0.1,
 * F_span = 0.9, tau_F = tau_CR = 0.1, and F = 0.5, CR = 0.9 at the start.
 * Checks: F_lo >= 0, F_span > 0 (finite), tau in [0, 1].                   */
typedef struct de_jde {
  float F_lo;
  float F_span;
  float tau_F;
  float tau_CR;
} de_jde;

/* As de_init_population, with jDE adaptation for every later generation;
 * params->F and params->CR are every individual's starting values.  Same
 * workspace size (the per-individual values are always reserved).        */
DE_API de_status de_init_population_jde(const de_params* params,
                                        const de_objective* objective,
                                        const de_jde* jde,
                                        const de_buffers* buffers,
                                        void* hip_stream, de_state** out);

/* jDE handles only (DE_E_STATE otherwise): copy the current generation's
 * per-individual F and CR (runs * NP floats each, host arrays, individual
 * (r, i) at r * NP + i) out of, or into, the workspace.  de_set_control
 * checks F > 0 finite and CR in [0, 1] (DE_E_INVAL) and is the way to
 * restore them with de_load_population (which keeps the current values).
 * Both synchronise hip_stream.                                             */
DE_API de_status de_get_control(de_state* state, void* hip_stream, float* F,
                                float* CR);
DE_API de_status de_set_control(de_state* state, void* hip_stream,
                                const float* F, const float* CR);

/* FP64 re-evaluation of every run's current best individual (the row the
 * FP32 best key points at): y = x - o and, for DE_OBJ_ROT_OSC, z = R y with R
 * as the FP32 matrix given at initialisation, are formed in FP64 and f is
 * summed in FP64 (Section 7.3.1 objective; Section 7.3.4 records the minimum
 * error).  This states the error of the FP32/BF16 arithmetic of the
 * generation step against exact arithmetic on the same vector.  f_host
 * receives runs doubles; idx_host (nullable) runs indices.  Synchronises
 * hip_stream.                                                              */
DE_API de_status de_best_f64(de_state* state, void* hip_stream, double* f_host,
                             int32_t* idx_host);

/* Current generation number of the handle (host-side counter). */
DE_API de_status de_get_generation(const de_state* state, int64_t* gen);

/* Per-run statistics, host pointers, each nullable, runs entries:
 * accepted = trials accepted since initialisation; best_f = current best
 * value.  Synchronises hip_stream.                                         */
DE_API de_status de_read_stats(de_state* state, void* hip_stream, int64_t* accepted,
                        double* best_f);

/* Declare that the caller has written generation `gen` into pop[gen & 1]
 * (for example, restoring a checkpoint).  The library re-evaluates every
 * row into fit[gen & 1] and resets best and first-hit statistics; the next
 * de_generation continues from `gen` with the same draws an uninterrupted
 * run would use, so a restart reproduces the uninterrupted run bit for bit.
 * 0 <= gen < 2^32.  Asynchronous.                                          */
DE_API de_status de_load_population(de_state* state, int64_t gen, void* hip_stream);

/* Objective values of n rows of ldx floats at x_dev into f_dev (device),
 * through the same kernels and precision as the generation step.
 * ldx >= D, ldx % 4 == 0, x_dev 16-byte aligned.  Asynchronous.           */
DE_API de_status de_eval(de_state* state, const float* x_dev, int32_t n, int32_t ldx,
                  float* f_dev, void* hip_stream);

/* Test support: the draws generation `gen` would use, written to device
 * arrays idx4_dev [runs][NP][4] = (r1, r2, r3, j_rand) (eqs. 2, 3) and
 * mask_dev [runs][NP][ceil(D/32)] (bit j%32 of word j/32 set iff trial
 * coordinate j comes from the mutant, j_rand included).  Either may be NULL.
 * Asynchronous.                                                            */
DE_API de_status de_debug_draws(const de_state* state, int64_t gen, int32_t* idx4_dev,
                         uint32_t* mask_dev, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * generation gen -> gen + 1 of all runs, as de_generation computes it on a
 * handle at generation gen, without a handle or a workspace.
 *   pop_cur, fit_cur : generation gen (runs * NP rows of ldx floats, runs * NP
 *                      values), device, read only;
 *   pop_next, fit_next: generation gen + 1, device, written (every row);
 *   ldx >= D, ldx % 4 == 0, row buffers 16-byte aligned, the two populations
 *   distinct; 0 <= gen < 2^32 - 1.  params and objective as for
 *   de_init_population (plain DE; o and R are read during the call).
 * The results equal those of de_generation on a handle holding the same
 * generation, bit for bit.  The library's own scratch (per-run statistics,
 * row flags, the padded shift and R in the product's operand layout) lives
 * in a fixed device array of 8 MiB inside the library, one per GPU, kept
 * until the process ends; the call allocates nothing and rewrites every
 * part of that array it uses with kernels (no memset), so it may be
 * captured into a graph.  Bytes used: sections of 8 runs (three of them),
 * 4, runs * NP, 4 dpad and, for DE_OBJ_ROT_OSC, dpad^2 * (2 BF16 | 4 FP32),
 * each rounded up to a multiple of 256, with dpad = D rounded up to 128;
 * beyond 8 MiB the call returns DE_E_UNSUPPORTED before any device work
 * (16 runs of NP 1024 at D = 1000 take 2.0 MiB with the BF16 product,
 * 4.0 MiB with FP32).  Statistics are not
 * reported.  Calls on one GPU share the array: calls that overlap in time
 * on one GPU (other streams, other host threads) race and must not be
 * issued.  Asynchronous on hip_stream.                                     */
DE_API de_status de_generation_noalloc(const de_params* params,
                                       const de_objective* objective,
                                       int64_t gen, const float* pop_cur,
                                       const float* fit_cur, float* pop_next,
                                       float* fit_next, int32_t ldx,
                                       void* hip_stream);

/* Release the handle (host memory only).  NULL is accepted. */
DE_API de_status de_destroy(de_state* state);

#ifdef __cplusplus
}
#endif

#endif /* DE_MI355X_DE_H_ */
