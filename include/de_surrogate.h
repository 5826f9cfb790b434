/*
 * de_surrogate.h -- surrogate-assisted DE/rand/1/bin on a composition
 * objective (libde.so, same library and conventions as de.h).
 *
 * The objective is a composition function (Section 7.3.3 of arXiv
 * 2405.16551): n rotated oscillating components g_k with shifts O[k] and
 * rotations R[k], biases bias[k] and normalised weights,
 *     f(x) = sum_k omega_k (g_k(x) + bias_k),
 *     omega_k = w_k / sum_j w_j,  w_k = exp(-||x - O[k]||^2 / (2 sigma^2)),
 *     g_k(x) = sum_i z_i^2 + sin^2(3 z_i),  z = R[k] (x - O[k]).
 * (The paper's weight also carries 1/sqrt(||x - O[k]||^2), singular at
 * x = O[k], and D in the exponent; both are dropped.  Exponents are shifted
 * by the smallest ||x - O[k]||^2, which cancels in the normalisation.)
 * Its evaluation is the expensive step the paper's Section 6 singles out.
 *
 * Each generation, every target i of every run builds k DE/rand/1/bin
 * trials (Section 2; candidate c draws with counter individual field
 * i | c << 24, so candidate 0 is the plain trial), a per-run MLP surrogate
 * D -> H -> H -> 1 (ReLU) predicts each candidate's scaled fitness on MFMA
 * in BF16 (FP32 accumulation), and only the candidate with the lowest
 * prediction (lowest c on ties) is evaluated on f; selection is the usual
 * strict comparison with the target.  Every evaluated point enters a
 * per-run ring-buffer archive with target t = log10(f + 1e-8); after each
 * generation the model takes `steps` Adam steps (FP32) on minibatches
 * drawn uniformly from the archive (Philox tag 5).  During the first
 * warmup_gens generations (and when k = 1) the model is not consulted and
 * candidate 0 is evaluated.  Model weights start He-uniform from Philox
 * (tag 6, keyed by model_seed), biases and Adam moments at zero.
 *
 * Model parameters of a run, packed (FP32):
 *     theta = [W1 (H x D) | b1 (H) | W2 (H x H) | b2 (H) | w3 (H) | b3],
 * input scaled to [-1, 1]: xs = (2 x - (lo + hi)) / (hi - lo).
 */
#ifndef DE_MI355X_DE_SURROGATE_H_
#define DE_MI355X_DE_SURROGATE_H_

#include "de.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Composition objective: n in 1..64 components of dimension D (must equal
 * de_params.D); O device [n][D], R device [n][D][ldr] (row-major,
 * z_i = sum_j R[k][i][j] y_j), bias host [n], sigma finite > 0.  Read
 * during de_sur_init only (converted into the workspace).                 */
typedef struct de_composition {
  int32_t n;
  int32_t ldr;
  float sigma;
  int32_t reserved;  /* must be 0 */
  const float* O;
  const float* R;
  const float* bias;
} de_composition;

/* Surrogate settings.
 *   k           candidates per target, 1..16
 *   hidden      H, a multiple of 32 in 32..256
 *   archive     archive rows per run, >= max(batch, NP)
 *   batch       minibatch rows, a multiple of 32 in 32..1024
 *   steps       Adam steps per generation, >= 0
 *   warmup_gens generations before the model screens candidates, >= 0
 *   lr, beta1, beta2, eps   Adam (finite; lr > 0, betas in [0, 1), eps > 0)
 *   model_seed  key of the initial weights                                */
typedef struct de_surrogate_params {
  int32_t k;
  int32_t hidden;
  int32_t archive;
  int32_t batch;
  int32_t steps;
  int32_t warmup_gens;
  float lr;
  float beta1;
  float beta2;
  float eps;
  uint64_t model_seed;
} de_surrogate_params;

typedef struct de_sur de_sur; /* opaque; owned by the library */

/* Parameters per run of the packed model (H*D + H*H + 3H + 1). */
DE_API int64_t de_sur_model_size(int32_t D, int32_t hidden);

/* Workspace bytes for (params, composition, settings).  Checks as
 * de_sur_init (DE_E_INVAL / DE_E_UNSUPPORTED).                             */
DE_API de_status de_sur_workspace_bytes(const de_params* params,
                                        const de_composition* comp,
                                        const de_surrogate_params* sp,
                                        size_t* bytes);

/* Creates a handle at generation 0: initialises every run's population
 * (as de_init_population, same draws), evaluates it on f, fills the
 * archive with it, initialises the models.  buffers as in de.h (pop/fit
 * ping-pong, workspace of de_sur_workspace_bytes bytes, 256-aligned,
 * preserved between calls), with ldx equal to D rounded up to a multiple
 * of 4.  params->F and params->CR are used by every candidate; runs is at
 * most 65535.                                                              */
DE_API de_status de_sur_init(const de_params* params,
                             const de_composition* comp,
                             const de_surrogate_params* sp,
                             const de_buffers* buffers, void* hip_stream,
                             de_sur** out);

/* n_gens >= 0 generations, each followed by the model's training steps. */
DE_API de_status de_sur_generation(de_sur* s, int32_t n_gens,
                                   void* hip_stream);

/* Per run (each [runs], nullable): lowest f of the current population and
 * its lowest index; trials accepted since creation.  Synchronises.        */
DE_API de_status de_sur_read(de_sur* s, void* hip_stream, double* best_f,
                             int32_t* best_idx, int64_t* accepted);

DE_API de_status de_sur_get_generation(const de_sur* s, int64_t* gen);

/* f of n rows x_dev (device, row r at x_dev + r * ldx, ldx >= D, ldx % 4
 * == 0, 16-byte aligned) into f_dev (device [n]).  Asynchronous.         */
DE_API de_status de_sur_eval(de_sur* s, const float* x_dev, int32_t n,
                             int32_t ldx, float* f_dev, void* hip_stream);

/* The surrogate of run `run` (BF16 inference kernel) on n rows: y_dev
 * (device [n]) receives the predicted scaled fitness.  Asynchronous.     */
DE_API de_status de_sur_predict(de_sur* s, int32_t run, const float* x_dev,
                                int32_t n, int32_t ldx, float* y_dev,
                                void* hip_stream);

/* Model state, host arrays of runs * model_size floats each (run r at
 * r * model_size): parameters, Adam first and second moments, and the
 * Adam step counter (steps taken).  Set checks finiteness and v >= 0.
 * Both synchronise.                                                        */
DE_API de_status de_sur_get_model(de_sur* s, void* hip_stream, float* theta,
                                  float* m, float* v, int64_t* step);
DE_API de_status de_sur_set_model(de_sur* s, void* hip_stream,
                                  const float* theta, const float* m,
                                  const float* v, int64_t step);

/* n_steps Adam steps on the archive without a generation. */
DE_API de_status de_sur_train(de_sur* s, int32_t n_steps, void* hip_stream);

/* Archive, host arrays: X [runs][archive][D], T [runs][archive], and the
 * number of filled rows per run (nullable outputs).  Synchronises.        */
DE_API de_status de_sur_get_archive(de_sur* s, void* hip_stream, float* X,
                                    float* T, int64_t* filled);

/* The last generation's candidates [runs][NP][k][D], predictions
 * [runs][NP][k] (0 when the model was not consulted) and choices
 * [runs][NP], host arrays, each nullable.  Synchronises.                  */
DE_API de_status de_sur_last(de_sur* s, void* hip_stream, float* cand,
                             float* pred, int32_t* choice);

DE_API de_status de_sur_destroy(de_sur* s);

#ifdef __cplusplus
}
#endif

#endif /* DE_MI355X_DE_SURROGATE_H_ */
