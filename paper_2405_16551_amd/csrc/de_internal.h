// de_internal.h -- launch interface between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace de {

enum { kObjSphere = 0, kObjRotOsc = 1 };
enum { kPrecF32 = 0, kPrecBF16 = 1 };

constexpr int kMaxLdsBytes = 160 * 1024;  // gfx950 LDS per workgroup

// Everything one generation launch needs, passed by value.
struct GenArgs {
  const float* pop_cur;   // generation g rows (EVAL: rows to evaluate)
  float* pop_next;        // generation g+1 rows (init: generation 0)
  const float* fit_cur;   // f of generation g
  float* fit_next;        // f of generation g+1 (EVAL: output values)
  const float* o;         // shift, zero-padded to dpad
  const void* rop;        // R in the MFMA B-operand layout (rotated only)
  unsigned long long* best_key;  // [runs] ordered (f, index) keys
  unsigned long long* hit_gen;   // [runs] first generation with best <= target
  unsigned long long* accepted;  // [runs] accepted trials
  unsigned int* done;            // runs that have hit the target
  unsigned char* changed;        // [runs*NP] row changed in the last step
  int runs, NP, D, ldx, dpad, nrows;
  float F, lo, hi, target;
  uint32_t cr_threshold, gen, key_lo, key_hi;
  uint32_t run_base;  // rotated kernels: draw-counter run = run_base + run
  // jDE (jde != 0): per-individual (F, CR) of generation g and g+1, and the
  // adaptation constants (tau as floor(tau 2^24))
  int jde;
  const float2* jp_cur;
  float2* jp_next;
  float jF_lo, jF_span;
  uint32_t jtau_F, jtau_CR;
};

// A HIP call's status, reported on stderr with its source location when the
// environment variable DE_DEBUG is set and the call failed.
hipError_t note_hip(hipError_t e, const char* file, int line);
#define DE_NOTE(expr) ::de::note_hip((expr), __FILE__, __LINE__)

// Allows kernel fn the dynamic LDS that its static LDS leaves free of the
// CU's 160 KB, on the current device (once per kernel and device).
hipError_t set_max_dynamic_lds(const void* fn);

size_t rot_lds_bytes_host(int prec, int dpad, bool jde = false);
bool sep_supported(int D);

// Resident form of the separable step (one workgroup per run, population in
// LDS for several generations): for rows of at most 256 coordinates whose
// two buffers fit in kSepResidentMaxLds bytes.
constexpr size_t kSepResidentMaxLds = 64 * 1024;
size_t sep_resident_lds_bytes(int NP, int ldx, int D);
bool sep_resident_fits(int NP, int ldx, int D);
hipError_t launch_sep_resident(const GenArgs& a, int n_gens, float* pop_final,
                               float* fit_final, hipStream_t s);

hipError_t launch_generation(const GenArgs& a, int kind, int prec,
                             hipStream_t s);
hipError_t launch_eval(const GenArgs& a, int kind, int prec, hipStream_t s);
hipError_t launch_init(const GenArgs& a, hipStream_t s);
hipError_t launch_fill_control(float2* jp, int n, float F, float CR,
                               hipStream_t s);
hipError_t launch_prep(const float* o, const float* R, int ldr, int D,
                       int dpad, int kind, int prec, float* o_pad, void* rop,
                       hipStream_t s);
hipError_t launch_stats_reset(const GenArgs& a, bool reset_accepted,
                              hipStream_t s);
hipError_t launch_best_from_fit(const GenArgs& a, hipStream_t s);
hipError_t launch_mark_changed(const GenArgs& a, hipStream_t s);
hipError_t launch_best_f64(const GenArgs& a, int kind, const float* rf32,
                           double* f64, int* idx, hipStream_t s);
hipError_t launch_copy_rot(const float* R, int ldr, int D, float* rf32,
                           hipStream_t s);
hipError_t launch_hit_check(const GenArgs& a, unsigned long long target_key,
                            hipStream_t s);
hipError_t launch_debug_draws(const GenArgs& a, int* idx4, uint32_t* mask,
                              hipStream_t s);

// One wave that waits `ns` nanoseconds (at most kMaxDelayNs) on the GPU's
// constant 100 MHz clock, then ends: a stream-ordered start offset.
constexpr uint32_t kMaxDelayNs = 1000000;
hipError_t launch_delay(uint32_t ns, hipStream_t s);

// Compute units of the current device.
int device_cus();

}  // namespace de
