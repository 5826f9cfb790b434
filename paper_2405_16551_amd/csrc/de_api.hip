// de_api.hip -- host runtime behind the C ABI of include/de.h.
//
// Validation (synchronous, before any launch), workspace layout, the
// generation counter and ping-pong parity, the host side of the
// early-stopping loop, and error mapping.  All device work is launched
// through de_internal.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <unordered_set>
#include <vector>

#include "de.h"
#include "de_internal.h"

// Scratch of de_generation_noalloc: a fixed array in the library's device
// code, one copy on every GPU the library runs on, held until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy (in
// host code the name stands for a host-side shadow): it uses the device
// address that hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

using de::GenArgs;

constexpr uint64_t kMagic = 0x4445'6d69'3335'3578ull;
constexpr int64_t kGenLimit = int64_t(1) << 32;  // counter field is 32-bit

struct Layout {
  size_t best, hit, acc, done, changed, opad, rop, rf32, f64, idx, jp[2],
      total;
};

size_t round_up(size_t v, size_t m) { return (v + m - 1) / m * m; }

// D padded for the MFMA tiling: 128 keeps the BF16 K loop a multiple of
// eight K-steps of 16.
int dpad_for(int D) { return (int)round_up((size_t)D, 128); }

// handle: the workspace of a handle; otherwise only what one generation
// step uses (statistics, changed flags, padded shift, R operand layout), the
// scratch of de_generation_noalloc.
Layout layout_for(const de_params& p, int kind, int prec, bool handle = true) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up(bytes, 256);
    return o;
  };
  const int dpad = dpad_for(p.D);
  L.best = take(8 * (size_t)p.runs);
  L.hit = take(8 * (size_t)p.runs);
  L.acc = take(8 * (size_t)p.runs);
  L.done = take(4);
  L.changed = take((size_t)p.runs * p.NP);
  L.opad = take(4 * (size_t)dpad);
  L.rop = 0;
  L.rf32 = 0;
  if (kind == de::kObjRotOsc)
    L.rop = take((size_t)dpad * dpad * (prec == de::kPrecBF16 ? 2 : 4));
  if (!handle) {
    L.total = off;
    return L;
  }
  if (kind == de::kObjRotOsc) L.rf32 = take((size_t)p.D * p.D * 4);
  L.f64 = take(8 * (size_t)p.runs);
  L.idx = take(4 * (size_t)p.runs);
  // jDE control values (F, CR) per individual, generation g and g+1
  L.jp[0] = take(8 * (size_t)p.runs * p.NP);
  L.jp[1] = take(8 * (size_t)p.runs * p.NP);
  L.total = off;
  return L;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices];  // per device, set on first use

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
hipError_t static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

}  // namespace

struct de_state {
  uint64_t magic;
  de_params p;
  int kind, prec, dpad, ldx;
  float* pop[2];
  float* fit[2];
  char* work;
  Layout L;
  int64_t gen;
  uint32_t cr_threshold;
  float target;  // -inf outside de_evolve: no hit bookkeeping
  hipStream_t last_stream;
  // jDE (de_init_population_jde): adaptation constants
  int jde;
  float jF_lo, jF_span;
  uint32_t jtau_F, jtau_CR;
  // de_evolve's overlapped polling: two pinned host slots for the device's
  // done counter and the events that mark their copies; created on the
  // first de_evolve call, released by de_destroy
  unsigned int* poll_slot;
  hipEvent_t poll_ev[2];
  // staggered run groups (see run_staggered): two streams and their events,
  // created on first use, released by de_destroy; the last measured time
  // per generation (0: none yet) and the generations timed by t0..t1 whose
  // result has not been read (0: none)
  hipStream_t grp[2];
  hipEvent_t grp_fork, grp_join[2], grp_t0, grp_t1;
  int64_t grp_timed;
  float gen_us;
  bool grp_failed;
};

namespace {

std::mutex g_live_mu;
std::unordered_set<const de_state*> g_live;

bool live(const de_state* s) {
  if (!s) return false;
  std::lock_guard<std::mutex> lk(g_live_mu);
  return g_live.count(s) != 0 && s->magic == kMagic;
}

bool aligned(const void* p, size_t a) {
  return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

de_status check_problem(const de_params* p, const de_objective* o) {
  if (!p || !o) return DE_E_INVAL;
  if (p->runs < 1 || p->runs >= (1 << 24)) return DE_E_INVAL;
  if (p->NP < 4 || p->D < 1) return DE_E_INVAL;
  if ((int64_t)p->runs * p->NP > std::numeric_limits<int32_t>::max())
    return DE_E_INVAL;
  if (!std::isfinite(p->F) || !(p->F > 0.f)) return DE_E_INVAL;
  if (!(p->CR >= 0.f && p->CR <= 1.f)) return DE_E_INVAL;
  if (!std::isfinite(p->lo) || !std::isfinite(p->hi) || !(p->lo < p->hi) ||
      !std::isfinite(p->hi - p->lo))
    return DE_E_INVAL;
  if (o->reserved != 0) return DE_E_INVAL;
  if (o->kind != de::kObjSphere && o->kind != de::kObjRotOsc)
    return DE_E_INVAL;
  if (!o->o || !aligned(o->o, 4)) return DE_E_INVAL;
  if (o->kind == de::kObjRotOsc) {
    if (o->gemm_prec != de::kPrecF32 && o->gemm_prec != de::kPrecBF16)
      return DE_E_INVAL;
    if (!o->R || !aligned(o->R, 4) || o->ldr < p->D) return DE_E_INVAL;
    const int dpad = dpad_for(p->D);
    if (de::rot_lds_bytes_host(o->gemm_prec, dpad) > (size_t)de::kMaxLdsBytes)
      return DE_E_UNSUPPORTED;
  } else {
    if (!de::sep_supported(p->D)) return DE_E_UNSUPPORTED;
  }
  return DE_OK;
}

de_status check_rows(const void* x, int32_t n_rows_hint, int32_t ldx, int D) {
  (void)n_rows_hint;
  if (!x || !aligned(x, 16)) return DE_E_INVAL;
  if (ldx < D || ldx % 4 != 0) return DE_E_INVAL;
  return DE_OK;
}

de_status from_hip(hipError_t e) { return e == hipSuccess ? DE_OK : DE_E_DEVICE; }
#define FROM_HIP(expr) from_hip(DE_NOTE(expr))

GenArgs base_args(const de_state* s) {
  GenArgs a{};
  a.o = reinterpret_cast<const float*>(s->work + s->L.opad);
  a.rop = s->L.rop ? s->work + s->L.rop : nullptr;
  a.best_key = reinterpret_cast<unsigned long long*>(s->work + s->L.best);
  a.hit_gen = reinterpret_cast<unsigned long long*>(s->work + s->L.hit);
  a.accepted = reinterpret_cast<unsigned long long*>(s->work + s->L.acc);
  a.done = reinterpret_cast<unsigned int*>(s->work + s->L.done);
  a.changed = reinterpret_cast<unsigned char*>(s->work + s->L.changed);
  a.runs = s->p.runs;
  a.NP = s->p.NP;
  a.D = s->p.D;
  a.ldx = s->ldx;
  a.dpad = s->dpad;
  a.nrows = s->p.runs * s->p.NP;
  a.F = s->p.F;
  a.lo = s->p.lo;
  a.hi = s->p.hi;
  a.target = s->target;
  a.cr_threshold = s->cr_threshold;
  a.gen = (uint32_t)s->gen;
  a.key_lo = (uint32_t)s->p.seed;
  a.key_hi = (uint32_t)(s->p.seed >> 32);
  a.jde = s->jde;
  a.jp_cur = reinterpret_cast<const float2*>(s->work + s->L.jp[s->gen & 1]);
  a.jp_next = reinterpret_cast<float2*>(s->work + s->L.jp[(s->gen + 1) & 1]);
  a.jF_lo = s->jF_lo;
  a.jF_span = s->jF_span;
  a.jtau_F = s->jtau_F;
  a.jtau_CR = s->jtau_CR;
  return a;
}

// f of pop[gen & 1] into fit[gen & 1], then statistics restart.
de_status eval_current_and_reset(de_state* s, hipStream_t st) {
  GenArgs a = base_args(s);
  const int b = (int)(s->gen & 1);
  a.pop_cur = s->pop[b];
  a.fit_next = s->fit[b];
  de_status rc = FROM_HIP(de::launch_eval(a, s->kind, s->prec, st));
  if (rc != DE_OK) return rc;
  rc = FROM_HIP(de::launch_stats_reset(a, true, st));
  if (rc != DE_OK) return rc;
  // the other buffer's rows are unknown: the next step rewrites every row
  rc = FROM_HIP(de::launch_mark_changed(a, st));
  if (rc != DE_OK) return rc;
  a.fit_cur = s->fit[b];
  return FROM_HIP(de::launch_best_from_fit(a, st));
}

// Largest float <= t (so that f <= t in float equals f <= t exactly).
float float_at_or_below(double t) {
  if (std::isinf(t)) return (float)t;
  if (t >= (double)std::numeric_limits<float>::max())
    return std::numeric_limits<float>::max();
  if (t <= -(double)std::numeric_limits<float>::max())
    return -std::numeric_limits<float>::infinity();
  float f = (float)t;
  if ((double)f > t) f = std::nextafter(f, -std::numeric_limits<float>::infinity());
  return f;
}

unsigned long long key_of(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  const uint32_t ord = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return (unsigned long long)ord << 32;
}

float f_of_key(unsigned long long key) {
  const uint32_t ord = (uint32_t)(key >> 32);
  const uint32_t b = (ord & 0x80000000u) ? (ord & 0x7FFFFFFFu) : ~ord;
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}

// Generations per launch of the resident separable form.
constexpr int64_t kResidentChunk = 1024;

// Staggered run groups, for rotated-objective problems that fill the GPU
// (at least as many tiles as compute units) with two or more runs.  Every
// CU of one launch goes through the same phases at the same time: the
// trial build (Philox draws, gathers of population rows from HBM), then
// the rotation product (MFMA, R fragments from L2), then selection.  Here
// the runs are split into two halves, each launched on a stream of its
// own, and the second half starts about half a generation after the first
// (a delay kernel of half the last measured time per generation), so one
// half builds trials while the other multiplies: HBM, L2 and the matrix
// cores are busy together and the chip's power is spread over the
// generation.  Each run's kernel arguments and draws are those of the
// single launch (pointers and the draw counter's run offset by the group's
// first run), so the results are identical.  DE_STAGGER=0 in the
// environment turns this off.
bool stagger_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("DE_STAGGER");
    return !(e && e[0] == '0');
  }();
  return on;
}

// Fewest generations per call that take the split: the second group's
// offset leaves half a generation of it after the first group's last
// kernel, so short calls keep one launch per generation.
constexpr int64_t kStaggerMinGens = 16;

// Problems that take the split: rotated objective, two or more runs, at
// least one 64-row tile per compute unit.  Their handles create the two
// streams at initialisation.
bool stagger_shape(const de_state* s) {
  if (s->kind != de::kObjRotOsc || s->p.runs < 2 || !stagger_enabled())
    return false;
  const long long tiles = (long long)s->p.runs * ((s->p.NP + 63) / 64);
  return tiles >= de::device_cus();
}

// A stream being captured into a graph gets the plain launches (event
// queries and timing are not allowed during capture).
bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) != hipSuccess ||
         cs != hipStreamCaptureStatusNone;
}

de_status stagger_setup(de_state* s) {
  if (s->grp[0]) return DE_OK;
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = DE_NOTE(hipStreamCreateWithFlags(&s->grp[k], hipStreamNonBlocking));
  if (e == hipSuccess)
    e = DE_NOTE(hipEventCreateWithFlags(&s->grp_fork, hipEventDisableTiming));
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = DE_NOTE(
        hipEventCreateWithFlags(&s->grp_join[k], hipEventDisableTiming));
  if (e == hipSuccess) e = DE_NOTE(hipEventCreate(&s->grp_t0));
  if (e == hipSuccess) e = DE_NOTE(hipEventCreate(&s->grp_t1));
  if (e != hipSuccess) {
    s->grp_failed = true;  // plain launches from now on
    return DE_E_DEVICE;
  }
  return DE_OK;
}

// Arguments of generation s->gen for runs [r0, r0 + nr).
GenArgs group_args(const de_state* s, int r0, int nr) {
  GenArgs a = base_args(s);
  const int b = (int)(s->gen & 1);
  const size_t rows0 = (size_t)r0 * s->p.NP;
  a.pop_cur = s->pop[b] + rows0 * s->ldx;
  a.fit_cur = s->fit[b] + rows0;
  a.pop_next = s->pop[b ^ 1] + rows0 * s->ldx;
  a.fit_next = s->fit[b ^ 1] + rows0;
  a.changed += rows0;
  a.best_key += r0;
  a.hit_gen += r0;
  a.accepted += r0;
  if (a.jde) {
    a.jp_cur += rows0;
    a.jp_next += rows0;
  }
  a.runs = nr;
  a.nrows = nr * s->p.NP;
  a.run_base = (uint32_t)r0;
  return a;
}

// Time per generation of an earlier timed call, once its events completed.
void read_gen_time(de_state* s) {
  if (s->grp_timed > 0 && hipEventQuery(s->grp_t1) == hipSuccess) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->grp_t0, s->grp_t1) == hipSuccess &&
        ms > 0.f)
      s->gen_us = ms * 1e3f / (float)s->grp_timed;
    s->grp_timed = 0;
  }
}

de_status run_staggered(de_state* s, int64_t n, hipStream_t st) {
  de_status rc = FROM_HIP(hipEventRecord(s->grp_fork, st));
  for (int k = 0; k < 2 && rc == DE_OK; ++k)
    rc = FROM_HIP(hipStreamWaitEvent(s->grp[k], s->grp_fork, 0));
  if (rc != DE_OK) return rc;
  const bool time_it = s->grp_timed == 0;
  if (time_it) rc = FROM_HIP(hipEventRecord(s->grp_t0, s->grp[0]));
  if (rc == DE_OK && s->gen_us > 0.f)
    rc = FROM_HIP(de::launch_delay((uint32_t)(s->gen_us * 500.f), s->grp[1]));
  const int half = s->p.runs / 2;
  for (int64_t k = 0; k < n && rc == DE_OK; ++k) {
    rc = FROM_HIP(de::launch_generation(group_args(s, 0, half), s->kind,
                                        s->prec, s->grp[0]));
    if (rc == DE_OK)
      rc = FROM_HIP(de::launch_generation(
          group_args(s, half, s->p.runs - half), s->kind, s->prec,
          s->grp[1]));
    if (rc == DE_OK) s->gen += 1;
  }
  if (rc == DE_OK && time_it) {
    rc = FROM_HIP(hipEventRecord(s->grp_t1, s->grp[0]));
    if (rc == DE_OK) s->grp_timed = n;
  }
  // the caller's stream waits for both halves (also after a failure, so
  // that nothing launched so far outlives the call's ordering)
  for (int k = 0; k < 2; ++k) {
    const de_status r1 = FROM_HIP(hipEventRecord(s->grp_join[k], s->grp[k]));
    const de_status r2 =
        r1 == DE_OK ? FROM_HIP(hipStreamWaitEvent(st, s->grp_join[k], 0)) : r1;
    if (rc == DE_OK) rc = r2;
  }
  return rc;
}

de_status run_plain(de_state* s, int64_t n, hipStream_t st);

de_status run_generations(de_state* s, int64_t n, hipStream_t st) {
  if (n > 0 && s->grp[0] && !s->grp_failed && !capturing(st)) {
    read_gen_time(s);
    if (n >= kStaggerMinGens) return run_staggered(s, n, st);
    // a short call: one launch per generation, timed for later offsets
    const bool time_it = s->grp_timed == 0;
    de_status rc = time_it ? FROM_HIP(hipEventRecord(s->grp_t0, st)) : DE_OK;
    if (rc == DE_OK) rc = run_plain(s, n, st);
    if (rc == DE_OK && time_it) {
      rc = FROM_HIP(hipEventRecord(s->grp_t1, st));
      if (rc == DE_OK) s->grp_timed = n;
    }
    return rc;
  }
  return run_plain(s, n, st);
}

de_status run_plain(de_state* s, int64_t n, hipStream_t st) {
  // small separable problems: several generations per launch, each run's
  // population resident in LDS (results equal the per-generation kernel's)
  if (n >= 2 && s->kind == de::kObjSphere && !s->jde &&
      de::sep_resident_fits(s->p.NP, s->ldx, s->p.D)) {
    while (n > 0) {
      const int m = (int)std::min<int64_t>(n, kResidentChunk);
      GenArgs a = base_args(s);
      const int b = (int)(s->gen & 1);
      a.pop_cur = s->pop[b];
      a.fit_cur = s->fit[b];
      a.pop_next = s->pop[b ^ 1];
      a.fit_next = s->fit[b ^ 1];
      const int fb = (int)((s->gen + m) & 1);
      const de_status rc = FROM_HIP(
          de::launch_sep_resident(a, m, s->pop[fb], s->fit[fb], st));
      if (rc != DE_OK) return rc;
      s->gen += m;
      n -= m;
    }
    return DE_OK;
  }
  for (int64_t k = 0; k < n; ++k) {
    GenArgs a = base_args(s);
    const int b = (int)(s->gen & 1);
    a.pop_cur = s->pop[b];
    a.fit_cur = s->fit[b];
    a.pop_next = s->pop[b ^ 1];
    a.fit_next = s->fit[b ^ 1];
    const de_status rc =
        FROM_HIP(de::launch_generation(a, s->kind, s->prec, st));
    if (rc != DE_OK) return rc;
    s->gen += 1;
  }
  return DE_OK;
}

}  // namespace

extern "C" {

DE_API int32_t de_abi_version(void) { return DE_ABI_VERSION; }

DE_API const char* de_strerror(de_status status) {
  switch (status) {
    case DE_OK: return "success";
    case DE_E_INVAL: return "invalid argument";
    case DE_E_NOMEM: return "host allocation failed";
    case DE_E_DEVICE: return "HIP runtime or kernel failure";
    case DE_E_STATE: return "invalid or destroyed handle, or wrong call order";
    case DE_E_UNSUPPORTED: return "size not supported by the library";
  }
  return "unknown status";
}

DE_API de_status de_workspace_bytes(const de_params* params,
                                    const de_objective* objective,
                                    size_t* bytes) {
  if (!bytes) return DE_E_INVAL;
  const de_status rc = check_problem(params, objective);
  if (rc != DE_OK) return rc;
  *bytes = layout_for(*params, objective->kind, objective->gemm_prec).total;
  return DE_OK;
}

}  // extern "C"

namespace {

// Adaptation constants of jDE: F' = F_lo + u F_span must stay a finite
// positive weight; tau are probabilities.
de_status check_jde(const de_jde* j) {
  if (!j) return DE_E_INVAL;
  if (!std::isfinite(j->F_lo) || !std::isfinite(j->F_span) ||
      !(j->F_lo >= 0.f) || !(j->F_span > 0.f) ||
      !std::isfinite(j->F_lo + j->F_span))
    return DE_E_INVAL;
  if (!(j->tau_F >= 0.f && j->tau_F <= 1.f) ||
      !(j->tau_CR >= 0.f && j->tau_CR <= 1.f))
    return DE_E_INVAL;
  return DE_OK;
}

de_status init_common(const de_params* params, const de_objective* objective,
                      const de_jde* jde, const de_buffers* buffers,
                      void* hip_stream, de_state** out) {
  if (!out || !buffers) return DE_E_INVAL;
  de_status rc = check_problem(params, objective);
  if (rc != DE_OK) return rc;
  if (jde && (rc = check_jde(jde)) != DE_OK) return rc;
  const de_params& p = *params;
  const int prec = objective->kind == de::kObjRotOsc ? objective->gemm_prec
                                                     : de::kPrecF32;
  if (buffers->reserved != 0) return DE_E_INVAL;
  for (int b = 0; b < 2; ++b) {
    if (check_rows(buffers->pop[b], 0, buffers->ldx, p.D) != DE_OK)
      return DE_E_INVAL;
    if (!buffers->fit[b] || !aligned(buffers->fit[b], 4)) return DE_E_INVAL;
  }
  if (buffers->pop[0] == buffers->pop[1] || buffers->fit[0] == buffers->fit[1])
    return DE_E_INVAL;
  if ((uint64_t)p.runs * p.NP * (uint64_t)buffers->ldx >
      (uint64_t)std::numeric_limits<int64_t>::max() / 4)
    return DE_E_INVAL;
  const Layout L = layout_for(p, objective->kind, prec);
  if (!buffers->work || !aligned(buffers->work, 256) ||
      buffers->work_bytes < L.total)
    return DE_E_INVAL;

  (void)hipGetLastError();  // clear a stale error left by unrelated calls
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  if (objective->kind == de::kObjRotOsc) {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DE_E_DEVICE;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                              dev) != hipSuccess)
      return DE_E_DEVICE;
    if (de::rot_lds_bytes_host(prec, dpad_for(p.D), jde != nullptr) >
        (size_t)lds)
      return DE_E_UNSUPPORTED;
  }

  de_state* s = new (std::nothrow) de_state();
  if (!s) return DE_E_NOMEM;
  s->magic = kMagic;
  s->p = p;
  s->kind = objective->kind;
  s->prec = prec;
  s->dpad = dpad_for(p.D);
  s->ldx = buffers->ldx;
  for (int b = 0; b < 2; ++b) {
    s->pop[b] = buffers->pop[b];
    s->fit[b] = buffers->fit[b];
  }
  s->work = reinterpret_cast<char*>(buffers->work);
  s->L = L;
  s->gen = 0;
  s->cr_threshold = (uint32_t)std::floor((double)p.CR * 16777216.0);
  s->target = -std::numeric_limits<float>::infinity();
  s->last_stream = st;
  s->jde = jde ? 1 : 0;
  if (jde) {
    s->jF_lo = jde->F_lo;
    s->jF_span = jde->F_span;
    s->jtau_F = (uint32_t)std::floor((double)jde->tau_F * 16777216.0);
    s->jtau_CR = (uint32_t)std::floor((double)jde->tau_CR * 16777216.0);
  }

  rc = FROM_HIP(de::launch_prep(objective->o, objective->R, objective->ldr,
                                p.D, s->dpad, s->kind, s->prec,
                                reinterpret_cast<float*>(s->work + L.opad),
                                L.rop ? s->work + L.rop : nullptr, st));
  if (rc == DE_OK && L.rf32)
    rc = FROM_HIP(de::launch_copy_rot(objective->R, objective->ldr, p.D,
                                      reinterpret_cast<float*>(s->work + L.rf32),
                                      st));
  if (rc == DE_OK) {
    GenArgs a = base_args(s);
    a.pop_next = s->pop[0];
    rc = FROM_HIP(de::launch_init(a, st));
  }
  if (rc == DE_OK && jde)
    rc = FROM_HIP(de::launch_fill_control(
        reinterpret_cast<float2*>(s->work + L.jp[0]), p.runs * p.NP, p.F,
        p.CR, st));
  if (rc == DE_OK) rc = eval_current_and_reset(s, st);
  if (rc != DE_OK) {
    s->magic = 0;
    delete s;
    return rc;
  }
  // the run-group streams of problems that take the split (a failure
  // leaves the handle on plain launches)
  if (stagger_shape(s)) (void)stagger_setup(s);
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(s);
  }
  *out = s;
  return DE_OK;
}

// (F, CR) of the current generation <-> host arrays.
de_status control_io(de_state* state, void* hip_stream, float* F, float* CR,
                     bool write) {
  if (!live(state)) return DE_E_STATE;
  if (!state->jde) return DE_E_STATE;
  if (!F || !CR) return DE_E_INVAL;
  const size_t n = (size_t)state->p.runs * state->p.NP;
  if (write) {
    for (size_t k = 0; k < n; ++k)
      if (!(F[k] > 0.f) || !std::isfinite(F[k]) || !(CR[k] >= 0.f) ||
          !(CR[k] <= 1.f))
        return DE_E_INVAL;
  }
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  float2* dev = reinterpret_cast<float2*>(state->work +
                                          state->L.jp[state->gen & 1]);
  std::vector<float2> h(n);
  de_status rc = DE_OK;
  if (write) {
    for (size_t k = 0; k < n; ++k) h[k] = make_float2(F[k], CR[k]);
    rc = FROM_HIP(hipMemcpyAsync(dev, h.data(), 8 * n, hipMemcpyHostToDevice,
                                 st));
    if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  } else {
    rc = FROM_HIP(hipMemcpyAsync(h.data(), dev, 8 * n, hipMemcpyDeviceToHost,
                                 st));
    if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
    if (rc == DE_OK)
      for (size_t k = 0; k < n; ++k) {
        F[k] = h[k].x;
        CR[k] = h[k].y;
      }
  }
  return rc;
}

}  // namespace

extern "C" {

DE_API de_status de_init_population(const de_params* params,
                                    const de_objective* objective,
                                    const de_buffers* buffers,
                                    void* hip_stream, de_state** out) {
  return init_common(params, objective, nullptr, buffers, hip_stream, out);
}

DE_API de_status de_init_population_jde(const de_params* params,
                                        const de_objective* objective,
                                        const de_jde* jde,
                                        const de_buffers* buffers,
                                        void* hip_stream, de_state** out) {
  if (!jde) return DE_E_INVAL;
  return init_common(params, objective, jde, buffers, hip_stream, out);
}

DE_API de_status de_get_control(de_state* state, void* hip_stream, float* F,
                                float* CR) {
  return control_io(state, hip_stream, F, CR, false);
}

DE_API de_status de_set_control(de_state* state, void* hip_stream,
                                const float* F, const float* CR) {
  return control_io(state, hip_stream, const_cast<float*>(F),
                    const_cast<float*>(CR), true);
}

DE_API de_status de_generation(de_state* state, int32_t n_gens,
                               void* hip_stream) {
  if (!live(state)) return DE_E_STATE;
  if (n_gens < 0) return DE_E_INVAL;
  if (state->gen + n_gens >= kGenLimit) return DE_E_INVAL;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  state->last_stream = st;
  return run_generations(state, n_gens, st);
}

DE_API de_status de_evolve(de_state* state, int64_t max_gens, double target,
                           int32_t check_every, void* hip_stream,
                           int64_t* gens_done, int64_t* hit_gen) {
  if (!live(state)) return DE_E_STATE;
  if (max_gens < 0 || check_every < 1 || std::isnan(target) || !gens_done)
    return DE_E_INVAL;
  if (state->gen + max_gens >= kGenLimit) return DE_E_INVAL;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  state->last_stream = st;
  *gens_done = 0;
  const float t32 = float_at_or_below(target);
  GenArgs a = base_args(state);
  de_status rc = DE_OK;
  // hit bookkeeping restarts for this target: clear, then runs already at
  // or below it hit at the current generation
  {
    GenArgs r = a;
    rc = FROM_HIP(de::launch_stats_reset(r, false, st));
    // launch_stats_reset also clears best; rebuild it from the current fit
    if (rc == DE_OK) {
      r.fit_cur = state->fit[state->gen & 1];
      rc = FROM_HIP(de::launch_best_from_fit(r, st));
    }
    if (rc == DE_OK) rc = FROM_HIP(de::launch_hit_check(r, key_of(t32), st));
  }
  state->target = t32;
  int64_t done_gens = 0;
  if (rc == DE_OK && !state->poll_slot) {
    void* h = nullptr;
    rc = FROM_HIP(hipHostMalloc(&h, 2 * sizeof(unsigned int),
                                hipHostMallocDefault));
    for (int k = 0; k < 2 && rc == DE_OK; ++k)
      rc = FROM_HIP(hipEventCreateWithFlags(&state->poll_ev[k],
                                            hipEventDisableTiming));
    state->poll_slot = static_cast<unsigned int*>(h);
  }
  // Runs already at the target before any generation: read synchronously.
  unsigned int* slot = state->poll_slot;
  if (rc == DE_OK) {
    rc = FROM_HIP(hipMemcpyAsync(&slot[0], a.done, sizeof(unsigned int),
                                 hipMemcpyDeviceToHost, st));
    if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  }
  if (rc == DE_OK && (int)slot[0] < state->p.runs) {
    // Overlapped polling (the solution-found flag copied to the host behind
    // every chunk): each chunk of check_every generations is followed on
    // the stream by a copy of the done counter into a pinned slot and an
    // event; the next chunk is queued before the host waits for the
    // previous chunk's event, so the device never idles on the host's round
    // trip.  The price is at most one chunk run past the chunk in which the
    // last run hit (the first-hit generations are exact on the device).
    int inflight = 0, head = 0, tail = 0;
    while (rc == DE_OK) {
      while (rc == DE_OK && inflight < 2 && done_gens < max_gens) {
        const int64_t n = std::min<int64_t>(check_every, max_gens - done_gens);
        rc = run_generations(state, n, st);
        if (rc != DE_OK) break;
        done_gens += n;
        rc = FROM_HIP(hipMemcpyAsync(&slot[tail], a.done, sizeof(unsigned int),
                                     hipMemcpyDeviceToHost, st));
        if (rc == DE_OK) rc = FROM_HIP(hipEventRecord(state->poll_ev[tail], st));
        tail ^= 1;
        ++inflight;
      }
      if (rc != DE_OK || inflight == 0) break;
      rc = FROM_HIP(hipEventSynchronize(state->poll_ev[head]));
      if (rc != DE_OK) break;
      const unsigned int done = slot[head];
      head ^= 1;
      --inflight;
      if ((int)done >= state->p.runs) break;
    }
  }
  state->target = -std::numeric_limits<float>::infinity();
  // a chunk queued ahead may still run: the call returns with the stream idle
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  *gens_done = done_gens;
  if (rc == DE_OK && hit_gen) {
    const int runs = state->p.runs;
    unsigned long long* tmp = new (std::nothrow) unsigned long long[runs];
    if (!tmp) return DE_E_NOMEM;
    rc = FROM_HIP(hipMemcpyAsync(tmp, a.hit_gen, 8 * (size_t)runs,
                                 hipMemcpyDeviceToHost, st));
    if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
    if (rc == DE_OK)
      for (int r = 0; r < runs; ++r)
        hit_gen[r] = tmp[r] == ~0ull ? -1 : (int64_t)tmp[r];
    delete[] tmp;
  }
  return rc;
}

DE_API de_status de_best(de_state* state, int32_t run, void* hip_stream,
                         float* x_host, double* f_host, int32_t* idx_host) {
  if (!live(state)) return DE_E_STATE;
  if (run < 0 || run >= state->p.runs || !f_host) return DE_E_INVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const GenArgs a = base_args(state);
  unsigned long long key = 0;
  de_status rc = FROM_HIP(hipMemcpyAsync(&key, a.best_key + run, 8,
                                         hipMemcpyDeviceToHost, st));
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  if (rc != DE_OK) return rc;
  if (key == ~0ull) return DE_E_STATE;
  const int32_t idx = (int32_t)(key & 0xFFFFFFFFu);
  if (idx < 0 || idx >= state->p.NP) return DE_E_STATE;
  *f_host = (double)f_of_key(key);
  if (idx_host) *idx_host = idx;
  if (x_host) {
    const float* row = state->pop[state->gen & 1] +
                       ((size_t)run * state->p.NP + idx) * state->ldx;
    rc = FROM_HIP(hipMemcpyAsync(x_host, row, sizeof(float) * state->p.D,
                                 hipMemcpyDeviceToHost, st));
    if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  }
  return rc;
}

DE_API de_status de_best_f64(de_state* state, void* hip_stream,
                             double* f_host, int32_t* idx_host) {
  if (!live(state)) return DE_E_STATE;
  if (!f_host) return DE_E_INVAL;
  if (state->kind == de::kObjRotOsc && state->p.D > 4096)
    return DE_E_UNSUPPORTED;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  GenArgs a = base_args(state);
  a.pop_cur = state->pop[state->gen & 1];
  double* f64 = reinterpret_cast<double*>(state->work + state->L.f64);
  int* idx = reinterpret_cast<int*>(state->work + state->L.idx);
  const float* rf32 = state->L.rf32
                          ? reinterpret_cast<const float*>(state->work +
                                                           state->L.rf32)
                          : nullptr;
  de_status rc = FROM_HIP(de::launch_best_f64(a, state->kind, rf32, f64, idx,
                                              st));
  const int runs = state->p.runs;
  if (rc == DE_OK)
    rc = FROM_HIP(hipMemcpyAsync(f_host, f64, 8 * (size_t)runs,
                                 hipMemcpyDeviceToHost, st));
  if (rc == DE_OK && idx_host)
    rc = FROM_HIP(hipMemcpyAsync(idx_host, idx, 4 * (size_t)runs,
                                 hipMemcpyDeviceToHost, st));
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  return rc;
}

DE_API de_status de_get_generation(const de_state* state, int64_t* gen) {
  if (!live(state)) return DE_E_STATE;
  if (!gen) return DE_E_INVAL;
  *gen = state->gen;
  return DE_OK;
}

DE_API de_status de_read_stats(de_state* state, void* hip_stream,
                               int64_t* accepted, double* best_f) {
  if (!live(state)) return DE_E_STATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const GenArgs a = base_args(state);
  const int runs = state->p.runs;
  unsigned long long* tmp = new (std::nothrow) unsigned long long[2 * runs];
  if (!tmp) return DE_E_NOMEM;
  de_status rc = FROM_HIP(hipMemcpyAsync(tmp, a.accepted, 8 * (size_t)runs,
                                         hipMemcpyDeviceToHost, st));
  if (rc == DE_OK)
    rc = FROM_HIP(hipMemcpyAsync(tmp + runs, a.best_key, 8 * (size_t)runs,
                                 hipMemcpyDeviceToHost, st));
  if (rc == DE_OK) rc = FROM_HIP(hipStreamSynchronize(st));
  if (rc == DE_OK) {
    for (int r = 0; r < runs; ++r) {
      if (accepted) accepted[r] = (int64_t)tmp[r];
      if (best_f) best_f[r] = (double)f_of_key(tmp[runs + r]);
    }
  }
  delete[] tmp;
  return rc;
}

DE_API de_status de_load_population(de_state* state, int64_t gen,
                                    void* hip_stream) {
  if (!live(state)) return DE_E_STATE;
  if (gen < 0 || gen >= kGenLimit) return DE_E_INVAL;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  state->last_stream = st;
  if (state->jde && ((gen ^ state->gen) & 1)) {
    // jDE: the control values move with the generation's parity
    const de_status rc = FROM_HIP(hipMemcpyAsync(
        state->work + state->L.jp[gen & 1],
        state->work + state->L.jp[state->gen & 1],
        8 * (size_t)state->p.runs * state->p.NP, hipMemcpyDeviceToDevice, st));
    if (rc != DE_OK) return rc;
  }
  state->gen = gen;
  return eval_current_and_reset(state, st);
}

DE_API de_status de_eval(de_state* state, const float* x_dev, int32_t n,
                         int32_t ldx, float* f_dev, void* hip_stream) {
  if (!live(state)) return DE_E_STATE;
  if (n < 0) return DE_E_INVAL;
  if (n == 0) return DE_OK;
  if (check_rows(x_dev, n, ldx, state->p.D) != DE_OK) return DE_E_INVAL;
  if (!f_dev || !aligned(f_dev, 4)) return DE_E_INVAL;
  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  GenArgs a = base_args(state);
  a.pop_cur = x_dev;
  a.fit_next = f_dev;
  a.nrows = n;
  a.ldx = ldx;
  return FROM_HIP(de::launch_eval(a, state->kind, state->prec, st));
}

DE_API de_status de_debug_draws(const de_state* state, int64_t gen,
                                int32_t* idx4_dev, uint32_t* mask_dev,
                                void* hip_stream) {
  if (!live(state)) return DE_E_STATE;
  if (gen < 0 || gen >= kGenLimit) return DE_E_INVAL;
  if (!idx4_dev && !mask_dev) return DE_OK;
  (void)hipGetLastError();
  GenArgs a = base_args(state);
  a.gen = (uint32_t)gen;
  return FROM_HIP(de::launch_debug_draws(
      a, idx4_dev, mask_dev, reinterpret_cast<hipStream_t>(hip_stream)));
}

DE_API de_status de_generation_noalloc(const de_params* params,
                                       const de_objective* objective,
                                       int64_t gen, const float* pop_cur,
                                       const float* fit_cur, float* pop_next,
                                       float* fit_next, int32_t ldx,
                                       void* hip_stream) {
  de_status rc = check_problem(params, objective);
  if (rc != DE_OK) return rc;
  const de_params& p = *params;
  if (gen < 0 || gen + 1 >= kGenLimit) return DE_E_INVAL;
  if (check_rows(pop_cur, 0, ldx, p.D) != DE_OK ||
      check_rows(pop_next, 0, ldx, p.D) != DE_OK)
    return DE_E_INVAL;
  if (!fit_cur || !fit_next || !aligned(fit_cur, 4) || !aligned(fit_next, 4))
    return DE_E_INVAL;
  if (pop_cur == pop_next || fit_cur == fit_next) return DE_E_INVAL;
  if ((uint64_t)p.runs * p.NP * (uint64_t)ldx >
      (uint64_t)std::numeric_limits<int64_t>::max() / 4)
    return DE_E_INVAL;
  const int prec = objective->kind == de::kObjRotOsc ? objective->gemm_prec
                                                     : de::kPrecF32;
  const Layout L = layout_for(p, objective->kind, prec, false);
  if (L.total > kStaticScratchBytes) return DE_E_UNSUPPORTED;

  (void)hipGetLastError();
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DE_E_DEVICE;
  if (objective->kind == de::kObjRotOsc) {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                              dev) != hipSuccess)
      return DE_E_DEVICE;
    if (de::rot_lds_bytes_host(prec, dpad_for(p.D)) > (size_t)lds)
      return DE_E_UNSUPPORTED;
  }
  void* work = nullptr;
  rc = FROM_HIP(static_scratch(&work));
  if (rc != DE_OK) return rc;

  // A handle on the stack over the caller's buffers and the scratch: the
  // step below is the one de_generation launches, so the results are the
  // same bit for bit.
  de_state s{};
  s.magic = kMagic;
  s.p = p;
  s.kind = objective->kind;
  s.prec = prec;
  s.dpad = dpad_for(p.D);
  s.ldx = ldx;
  const int b = (int)(gen & 1);
  s.pop[b] = const_cast<float*>(pop_cur);
  s.fit[b] = const_cast<float*>(fit_cur);
  s.pop[b ^ 1] = pop_next;
  s.fit[b ^ 1] = fit_next;
  s.work = static_cast<char*>(work);
  s.L = L;
  s.gen = gen;
  s.cr_threshold = (uint32_t)std::floor((double)p.CR * 16777216.0);
  s.target = -std::numeric_limits<float>::infinity();
  s.last_stream = st;
  // every section that must start from a known value is rewritten by a
  // kernel (no memset: the call may be captured into a graph): padded
  // shift and R operand layout, statistics, and "changed" for every row so
  // that the step writes every row of pop_next
  rc = FROM_HIP(de::launch_prep(objective->o, objective->R, objective->ldr,
                                p.D, s.dpad, s.kind, s.prec,
                                reinterpret_cast<float*>(s.work + L.opad),
                                L.rop ? s.work + L.rop : nullptr, st));
  const GenArgs a = base_args(&s);
  if (rc == DE_OK) rc = FROM_HIP(de::launch_stats_reset(a, true, st));
  if (rc == DE_OK) rc = FROM_HIP(de::launch_mark_changed(a, st));
  if (rc == DE_OK) rc = run_generations(&s, 1, st);
  return rc;
}

DE_API de_status de_destroy(de_state* state) {
  if (!state) return DE_OK;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    if (!g_live.count(state)) return DE_E_STATE;
    g_live.erase(state);
  }
  state->magic = 0;
  for (int k = 0; k < 2; ++k)
    if (state->poll_ev[k]) (void)hipEventDestroy(state->poll_ev[k]);
  if (state->poll_slot) (void)hipHostFree(state->poll_slot);
  for (int k = 0; k < 2; ++k) {
    if (state->grp[k]) {
      (void)hipStreamSynchronize(state->grp[k]);
      (void)hipStreamDestroy(state->grp[k]);
    }
    if (state->grp_join[k]) (void)hipEventDestroy(state->grp_join[k]);
  }
  for (hipEvent_t e : {state->grp_fork, state->grp_t0, state->grp_t1})
    if (e) (void)hipEventDestroy(e);
  delete state;
  return DE_OK;
}

}  // extern "C"
