/*
 * de_batch.h -- many independent DE runs of mixed size on one GPU
 * (libde.so, same library and conventions as de.h).
 *
 * A batch holds nruns independent DE/rand/1/bin runs (Section 2 of arXiv
 * 2405.16551), each with its own population size NP, dimension D, F and CR,
 * on the rotated oscillating objective of Section 7.3.1 with one shift o and
 * rotation R per dimension ("instance").  Runs never exchange individuals:
 * they are the sub-populations of the multi-population model of Section
 * 5.4, without migration.  All runs advance together.  One generation of
 * every run is one persistent launch per tile variant in use, and a chunk
 * of graph_gens generations is one HIP graph launch.  This is the
 * consolidated-kernel, automatically configured, concurrent-kernel design
 * of the improved GPU DE reviewed in Section 6.1, carried to mixed-size
 * sub-populations as Section 9 proposes.  The tile variant of each instance
 * is chosen by an autotuner that times every candidate on the batch itself
 * (or fixed by the caller).
 *
 * Conventions are those of de.h: every call returns de_status; device
 * memory is caller-owned; launches are asynchronous on hip_stream; argument
 * checks are synchronous and precede any launch; a handle is not
 * thread-safe.
 *
 * Draws: run r of a batch uses run number r in the Philox counter
 * (q, i, gen, tag << 24 | r) keyed by the seed, so its generation g draws
 * exactly what run r of a de.h handle with the same seed, NP, D, F and CR
 * draws.  Results are a pure function of (params, instances, seed,
 * generation, plan): the plan fixes the FP32 summation order of the
 * objective, and nothing else depends on it.
 */
#ifndef DE_MI355X_DE_BATCH_H_
#define DE_MI355X_DE_BATCH_H_

#include "de.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One run: NP >= 4 (eq. 2 needs three donors distinct from the target),
 * D >= 1 and equal to the D of exactly one instance, F finite and > 0
 * (eq. 2), CR in [0, 1] (eq. 3).                                          */
typedef struct de_run_spec {
  int32_t NP;
  int32_t D;
  float F;
  float CR;
} de_run_spec;

/* Shift and rotation of one dimension (Section 7.3.1): device arrays o [D]
 * and R [D][ldr] (row-major, z_i = sum_j R[i*ldr + j] (x_j - o_j)),
 * ldr >= D, 4-byte aligned.  Read during de_batch_create only (converted
 * into the workspace); they may be released once that call returns.      */
typedef struct de_batch_instance {
  int32_t D;
  int32_t ldr;
  const float* o;
  const float* R;
} de_batch_instance;

/* Batch description.
 *   nruns      1 .. 2^24 - 1 runs; runs[] (host) describes each.
 *   ninst      >= 1 instances with distinct D; inst[] (host).
 *   lo, hi     search box shared by every run (finite, lo < hi).
 *   seed       64-bit Philox key.
 *   gemm_prec  arithmetic of z = R y: DE_GEMM_BF16 (BF16 operands, FP32
 *              accumulation).  DE_GEMM_FP32 returns DE_E_UNSUPPORTED.
 *   graph_gens generations per graph launch, 1 .. 1024 (1: direct launches
 *              only).
 *   target     hit_gen records the first generation whose best <= target. */
typedef struct de_batch_params {
  int32_t nruns;
  int32_t ninst;
  const de_run_spec* runs;
  const de_batch_instance* inst;
  float lo;
  float hi;
  uint64_t seed;
  int32_t gemm_prec;
  int32_t graph_gens;
  double target;
} de_batch_params;

/* Tile variants (values of a plan entry).
 *   DE_BATCH_AUTO   : let the autotuner choose (de_batch_create only).
 *   DE_BATCH_TILE64 : 64 trial rows per tile, 256 threads; D padded to a
 *                     multiple of 32; one MFMA K-step per LDS read.
 *   DE_BATCH_TILE32 : 32 rows per tile, 256 threads, same padding.
 *   DE_BATCH_WIDE   : 64 rows per tile, 1024 threads, D padded to a multiple
 *                     of 128, software-pipelined MFMA loop (the kernel of
 *                     de.h's BF16 path).                                    */
enum {
  DE_BATCH_AUTO = -1,
  DE_BATCH_TILE64 = 0,
  DE_BATCH_TILE32 = 1,
  DE_BATCH_WIDE = 2,
  DE_BATCH_NVARIANTS = 3
};

/* Memory layout of a batch (host-only computation, no device access).
 * Population buffer b (two of them, ping-pong: generation g in buffer
 * g & 1) holds row i of run r at element pop_off[r] + i * ldx[r]; ldx[r] is
 * D rounded up to a multiple of 4 and pop_off[r] a multiple of 64.  Fitness
 * buffer b holds f of that row at element fit_off[r] + i.  Outputs:
 * pop_off, ldx, fit_off ([nruns], each nullable); pop_floats and
 * fit_floats (floats per population / fitness buffer) and work_bytes
 * (workspace bytes), each nullable.  DE_E_INVAL / DE_E_UNSUPPORTED as for
 * de_batch_create's parameter checks.                                      */
DE_API de_status de_batch_layout(const de_batch_params* params,
                                 int64_t* pop_off, int32_t* ldx,
                                 int64_t* fit_off, size_t* pop_floats,
                                 size_t* fit_floats, size_t* work_bytes);

typedef struct de_batch de_batch; /* opaque; owned by the library */

/* Creates a batch at generation 0: initialises every run (uniform in the
 * box, as de_init_population), evaluates it, converts the instances and
 * fixes the plan.  pop0/pop1 (pop_floats each) and fit0/fit1 (fit_floats
 * each) are caller-owned device buffers, 16-byte aligned; `work` is a
 * caller-owned device workspace of at least work_bytes bytes, 256-byte
 * aligned, preserved between calls.  The library owns the contents of all
 * five between calls (as in de.h); callers read populations through the
 * layout above.
 * plan: host [ninst] tile variant per instance, DE_BATCH_AUTO entries tuned;
 * NULL tunes every instance.  Tuning times each candidate variant on the
 * instance's own runs (a few repeats of generation 0, whose result is
 * discarded).  A variant an instance cannot use (LDS) is DE_E_UNSUPPORTED
 * when requested explicitly.  Synchronises hip_stream.                     */
DE_API de_status de_batch_create(const de_batch_params* params, float* pop0,
                                 float* pop1, float* fit0, float* fit1,
                                 void* work, size_t work_bytes,
                                 const int32_t* plan, void* hip_stream,
                                 de_batch** out);

/* The plan in use: plan [ninst] variants; us_per_gen (nullable,
 * [ninst * DE_BATCH_NVARIANTS]) the tuner's time per generation of each
 * instance's runs alone under each variant, in microseconds, or -1 where
 * not timed.                                                               */
DE_API de_status de_batch_plan(const de_batch* batch, int32_t* plan,
                               float* us_per_gen);

/* Advances every run by n_gens >= 0 generations (asynchronous).  Whole
 * chunks of graph_gens generations run as one HIP graph launch (the graph
 * is built on first use); the remainder as direct launches.  Both give
 * identical results.                                                       */
DE_API de_status de_batch_generation(de_batch* batch, int64_t n_gens,
                                     void* hip_stream);

/* Per-run results, each output [nruns] and nullable: best_f / best_idx the
 * lowest f of the current generation and its lowest index; accepted the
 * trials accepted since creation; hit_gen the first generation whose best
 * was <= target (-1 if none yet).  Synchronises hip_stream.               */
DE_API de_status de_batch_read(de_batch* batch, void* hip_stream,
                               double* best_f, int32_t* best_idx,
                               int64_t* accepted, int64_t* hit_gen);

/* Current generation number of the batch. */
DE_API de_status de_batch_get_generation(const de_batch* batch, int64_t* gen);

/* Releases the handle and its graph (no device memory is freed: all of it
 * is the caller's).  Synchronises the device first.                        */
DE_API de_status de_batch_destroy(de_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* DE_MI355X_DE_BATCH_H_ */
