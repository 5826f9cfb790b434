"""Python binding of libde.so (the C ABI declared in include/de.h).

Argument marshalling only: every step of DE runs in the library's HIP
kernels.  The ``de_*`` functions mirror the C entry points one to one;
``DifferentialEvolution`` is a convenience owner of the caller-side device
buffers, allocated with PyTorch (device memory and streams are all PyTorch
is used for).

The library must have been built (``python -m paper_2405_16551_amd.build``);
importing this module without it raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

# The library must bind to the HIP runtime PyTorch loads (PyTorch ships its
# own copy, and streams and device pointers come from it): import PyTorch
# before the library, or the process can end up with two HIP runtimes.
import torch  # noqa: F401

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libde.so")

DE_OK, DE_E_INVAL, DE_E_NOMEM, DE_E_DEVICE, DE_E_STATE, DE_E_UNSUPPORTED = range(6)
DE_OBJ_SPHERE, DE_OBJ_ROT_OSC = 0, 1
DE_GEMM_FP32, DE_GEMM_BF16 = 0, 1

_KINDS = {"sphere": DE_OBJ_SPHERE, "rot_osc": DE_OBJ_ROT_OSC}
_PRECS = {"fp32": DE_GEMM_FP32, "bf16": DE_GEMM_BF16}


class de_params(ctypes.Structure):
    _fields_ = [("runs", ctypes.c_int32), ("NP", ctypes.c_int32),
                ("D", ctypes.c_int32), ("F", ctypes.c_float),
                ("CR", ctypes.c_float), ("lo", ctypes.c_float),
                ("hi", ctypes.c_float), ("seed", ctypes.c_uint64)]


class de_objective(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("gemm_prec", ctypes.c_int32),
                ("ldr", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("o", ctypes.c_void_p), ("R", ctypes.c_void_p)]


class de_buffers(ctypes.Structure):
    _fields_ = [("pop", ctypes.c_void_p * 2), ("fit", ctypes.c_void_p * 2),
                ("ldx", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("work", ctypes.c_void_p), ("work_bytes", ctypes.c_size_t)]


class de_jde(ctypes.Structure):
    _fields_ = [("F_lo", ctypes.c_float), ("F_span", ctypes.c_float),
                ("tau_F", ctypes.c_float), ("tau_CR", ctypes.c_float)]


# Brest et al. (2006): F' = 0.1 + 0.9 u, tau_F = tau_CR = 0.1
JDE_BREST = dict(F_lo=0.1, F_span=0.9, tau_F=0.1, tau_CR=0.1)


class de_composition(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("ldr", ctypes.c_int32),
                ("sigma", ctypes.c_float), ("reserved", ctypes.c_int32),
                ("O", ctypes.c_void_p), ("R", ctypes.c_void_p),
                ("bias", ctypes.POINTER(ctypes.c_float))]


class de_surrogate_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("archive", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("warmup_gens", ctypes.c_int32),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("model_seed", ctypes.c_uint64)]


# The settings measured best on the 100-dimensional composition instances:
# one Adam step per generation at lr 5e-3 on 128 rows of an archive of the
# last 4096 evaluations.
SURROGATE_DEFAULTS = dict(k=4, hidden=256, archive=4096, batch=128, steps=1,
                          warmup_gens=5, lr=5e-3, beta1=0.9, beta2=0.999,
                          eps=1e-8, model_seed=7)


class de_run_spec(ctypes.Structure):
    _fields_ = [("NP", ctypes.c_int32), ("D", ctypes.c_int32),
                ("F", ctypes.c_float), ("CR", ctypes.c_float)]


class de_batch_instance(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("ldr", ctypes.c_int32),
                ("o", ctypes.c_void_p), ("R", ctypes.c_void_p)]


class de_batch_params(ctypes.Structure):
    _fields_ = [("nruns", ctypes.c_int32), ("ninst", ctypes.c_int32),
                ("runs", ctypes.POINTER(de_run_spec)),
                ("inst", ctypes.POINTER(de_batch_instance)),
                ("lo", ctypes.c_float), ("hi", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("gemm_prec", ctypes.c_int32),
                ("graph_gens", ctypes.c_int32), ("target", ctypes.c_double)]


DE_BATCH_AUTO, DE_BATCH_TILE64, DE_BATCH_TILE32, DE_BATCH_WIDE = -1, 0, 1, 2
DE_BATCH_NVARIANTS = 3
VARIANT_NAMES = {DE_BATCH_TILE64: "tile64", DE_BATCH_TILE32: "tile32",
                 DE_BATCH_WIDE: "wide"}

EXPORTS = ("de_abi_version", "de_strerror", "de_workspace_bytes",
           "de_init_population", "de_generation", "de_evolve", "de_best",
           "de_best_f64", "de_get_generation", "de_read_stats", "de_load_population",
           "de_eval", "de_debug_draws", "de_destroy",
           "de_init_population_jde", "de_get_control", "de_set_control",
           "de_generation_noalloc",
           # include/de_surrogate.h
           "de_sur_model_size", "de_sur_workspace_bytes", "de_sur_init",
           "de_sur_generation", "de_sur_read", "de_sur_get_generation",
           "de_sur_eval", "de_sur_predict", "de_sur_get_model",
           "de_sur_set_model", "de_sur_train", "de_sur_get_archive",
           "de_sur_last", "de_sur_destroy",
           # include/de_batch.h
           "de_batch_layout", "de_batch_create", "de_batch_plan",
           "de_batch_generation", "de_batch_read", "de_batch_get_generation",
           "de_batch_destroy")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_2405_16551_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    st = ctypes.c_int
    lib.de_abi_version.restype = i32
    lib.de_abi_version.argtypes = []
    lib.de_strerror.restype = ctypes.c_char_p
    lib.de_strerror.argtypes = [st]
    lib.de_workspace_bytes.restype = st
    lib.de_workspace_bytes.argtypes = [P(de_params), P(de_objective),
                                       P(ctypes.c_size_t)]
    lib.de_init_population.restype = st
    lib.de_init_population.argtypes = [P(de_params), P(de_objective),
                                       P(de_buffers), vp, P(vp)]
    lib.de_init_population_jde.restype = st
    lib.de_init_population_jde.argtypes = [P(de_params), P(de_objective),
                                           P(de_jde), P(de_buffers), vp,
                                           P(vp)]
    fp = P(ctypes.c_float)
    lib.de_get_control.restype = st
    lib.de_get_control.argtypes = [vp, vp, fp, fp]
    lib.de_set_control.restype = st
    lib.de_set_control.argtypes = [vp, vp, fp, fp]
    lib.de_generation.restype = st
    lib.de_generation.argtypes = [vp, i32, vp]
    lib.de_generation_noalloc.restype = st
    lib.de_generation_noalloc.argtypes = [P(de_params), P(de_objective), i64,
                                          vp, vp, vp, vp, i32, vp]
    lib.de_evolve.restype = st
    lib.de_evolve.argtypes = [vp, i64, ctypes.c_double, i32, vp, P(i64),
                              P(i64)]
    lib.de_best.restype = st
    lib.de_best.argtypes = [vp, i32, vp, P(ctypes.c_float),
                            P(ctypes.c_double), P(i32)]
    lib.de_best_f64.restype = st
    lib.de_best_f64.argtypes = [vp, vp, P(ctypes.c_double), P(i32)]
    lib.de_get_generation.restype = st
    lib.de_get_generation.argtypes = [vp, P(i64)]
    lib.de_read_stats.restype = st
    lib.de_read_stats.argtypes = [vp, vp, P(i64), P(ctypes.c_double)]
    lib.de_load_population.restype = st
    lib.de_load_population.argtypes = [vp, i64, vp]
    lib.de_eval.restype = st
    lib.de_eval.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.de_debug_draws.restype = st
    lib.de_debug_draws.argtypes = [vp, i64, vp, vp, vp]
    lib.de_destroy.restype = st
    lib.de_destroy.argtypes = [vp]
    szp = P(ctypes.c_size_t)
    fpp = P(ctypes.c_float)
    lib.de_sur_model_size.restype = i64
    lib.de_sur_model_size.argtypes = [i32, i32]
    lib.de_sur_workspace_bytes.restype = st
    lib.de_sur_workspace_bytes.argtypes = [P(de_params), P(de_composition),
                                           P(de_surrogate_params), szp]
    lib.de_sur_init.restype = st
    lib.de_sur_init.argtypes = [P(de_params), P(de_composition),
                                P(de_surrogate_params), P(de_buffers), vp,
                                P(vp)]
    lib.de_sur_generation.restype = st
    lib.de_sur_generation.argtypes = [vp, i32, vp]
    lib.de_sur_read.restype = st
    lib.de_sur_read.argtypes = [vp, vp, P(ctypes.c_double), P(i32), P(i64)]
    lib.de_sur_get_generation.restype = st
    lib.de_sur_get_generation.argtypes = [vp, P(i64)]
    lib.de_sur_eval.restype = st
    lib.de_sur_eval.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.de_sur_predict.restype = st
    lib.de_sur_predict.argtypes = [vp, i32, vp, i32, i32, vp, vp]
    lib.de_sur_get_model.restype = st
    lib.de_sur_get_model.argtypes = [vp, vp, fpp, fpp, fpp, P(i64)]
    lib.de_sur_set_model.restype = st
    lib.de_sur_set_model.argtypes = [vp, vp, fpp, fpp, fpp, i64]
    lib.de_sur_train.restype = st
    lib.de_sur_train.argtypes = [vp, i32, vp]
    lib.de_sur_get_archive.restype = st
    lib.de_sur_get_archive.argtypes = [vp, vp, fpp, fpp, P(i64)]
    lib.de_sur_last.restype = st
    lib.de_sur_last.argtypes = [vp, vp, fpp, fpp, P(i32)]
    lib.de_sur_destroy.restype = st
    lib.de_sur_destroy.argtypes = [vp]
    lib.de_batch_layout.restype = st
    lib.de_batch_layout.argtypes = [P(de_batch_params), P(i64), P(i32), P(i64),
                                    szp, szp, szp]
    lib.de_batch_create.restype = st
    lib.de_batch_create.argtypes = [P(de_batch_params), vp, vp, vp, vp, vp,
                                    ctypes.c_size_t, P(i32), vp, P(vp)]
    lib.de_batch_plan.restype = st
    lib.de_batch_plan.argtypes = [vp, P(i32), P(ctypes.c_float)]
    lib.de_batch_generation.restype = st
    lib.de_batch_generation.argtypes = [vp, i64, vp]
    lib.de_batch_read.restype = st
    lib.de_batch_read.argtypes = [vp, vp, P(ctypes.c_double), P(i32), P(i64),
                                  P(i64)]
    lib.de_batch_get_generation.restype = st
    lib.de_batch_get_generation.argtypes = [vp, P(i64)]
    lib.de_batch_destroy.restype = st
    lib.de_batch_destroy.argtypes = [vp]
    return lib


_lib = _load()


class DEError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {de_strerror(status)} (status {status})")


def _check(status: int, where: str):
    if status != DE_OK:
        raise DEError(status, where)


# ---- one-to-one wrappers of the C entry points ---------------------------

def de_abi_version() -> int:
    return int(_lib.de_abi_version())


def de_strerror(status: int) -> str:
    return _lib.de_strerror(status).decode()


def de_workspace_bytes(params: de_params, objective: de_objective) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib.de_workspace_bytes(ctypes.byref(params),
                                   ctypes.byref(objective), ctypes.byref(n)),
           "de_workspace_bytes")
    return int(n.value)


def de_init_population(params, objective, buffers, stream) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(_lib.de_init_population(ctypes.byref(params),
                                   ctypes.byref(objective),
                                   ctypes.byref(buffers), stream,
                                   ctypes.byref(h)), "de_init_population")
    return h


def de_init_population_jde(params, objective, jde, buffers, stream):
    h = ctypes.c_void_p()
    _check(_lib.de_init_population_jde(ctypes.byref(params),
                                       ctypes.byref(objective),
                                       ctypes.byref(jde),
                                       ctypes.byref(buffers), stream,
                                       ctypes.byref(h)),
           "de_init_population_jde")
    return h


def de_get_control(handle, stream, n: int):
    F = (ctypes.c_float * n)()
    CR = (ctypes.c_float * n)()
    _check(_lib.de_get_control(handle, stream, F, CR), "de_get_control")
    return list(F), list(CR)


def de_set_control(handle, stream, F, CR):
    n = len(F)
    _check(_lib.de_set_control(handle, stream, (ctypes.c_float * n)(*F),
                               (ctypes.c_float * n)(*CR)), "de_set_control")


def de_generation(handle, n_gens: int, stream):
    _check(_lib.de_generation(handle, n_gens, stream), "de_generation")


def de_generation_noalloc(params, objective, gen: int, pop_cur, fit_cur,
                          pop_next, fit_next, ldx: int, stream):
    """One generation gen -> gen + 1 without a handle or workspace (the
    library's static scratch); pointers are device addresses (ints)."""
    _check(_lib.de_generation_noalloc(ctypes.byref(params),
                                      ctypes.byref(objective), gen, pop_cur,
                                      fit_cur, pop_next, fit_next, ldx, stream),
           "de_generation_noalloc")


def de_evolve(handle, max_gens: int, target: float, check_every: int, stream,
              runs: int):
    done = ctypes.c_int64(0)
    hits = (ctypes.c_int64 * runs)()
    _check(_lib.de_evolve(handle, max_gens, target, check_every, stream,
                          ctypes.byref(done), hits), "de_evolve")
    return int(done.value), [int(v) for v in hits]


def de_best(handle, run: int, stream, D: int):
    x = (ctypes.c_float * D)()
    f = ctypes.c_double(0)
    idx = ctypes.c_int32(0)
    _check(_lib.de_best(handle, run, stream, x, ctypes.byref(f),
                        ctypes.byref(idx)), "de_best")
    return list(x), float(f.value), int(idx.value)


def de_best_f64(handle, stream, runs: int):
    f = (ctypes.c_double * runs)()
    idx = (ctypes.c_int32 * runs)()
    _check(_lib.de_best_f64(handle, stream, f, idx), "de_best_f64")
    return [float(v) for v in f], [int(v) for v in idx]


def de_get_generation(handle) -> int:
    g = ctypes.c_int64(0)
    _check(_lib.de_get_generation(handle, ctypes.byref(g)), "de_get_generation")
    return int(g.value)


def de_read_stats(handle, stream, runs: int):
    acc = (ctypes.c_int64 * runs)()
    best = (ctypes.c_double * runs)()
    _check(_lib.de_read_stats(handle, stream, acc, best), "de_read_stats")
    return [int(v) for v in acc], [float(v) for v in best]


def de_load_population(handle, gen: int, stream):
    _check(_lib.de_load_population(handle, gen, stream), "de_load_population")


def de_eval(handle, x_ptr: int, n: int, ldx: int, f_ptr: int, stream):
    _check(_lib.de_eval(handle, x_ptr, n, ldx, f_ptr, stream), "de_eval")


def de_debug_draws(handle, gen: int, idx4_ptr, mask_ptr, stream):
    _check(_lib.de_debug_draws(handle, gen, idx4_ptr, mask_ptr, stream),
           "de_debug_draws")


def de_destroy(handle):
    _check(_lib.de_destroy(handle), "de_destroy")


def de_batch_layout(params: de_batch_params):
    n = params.nruns
    pop_off = (ctypes.c_int64 * n)()
    ldx = (ctypes.c_int32 * n)()
    fit_off = (ctypes.c_int64 * n)()
    pf, ff, wb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.de_batch_layout(ctypes.byref(params), pop_off, ldx, fit_off,
                                ctypes.byref(pf), ctypes.byref(ff),
                                ctypes.byref(wb)), "de_batch_layout")
    return dict(pop_off=list(pop_off), ldx=list(ldx), fit_off=list(fit_off),
                pop_floats=int(pf.value), fit_floats=int(ff.value),
                work_bytes=int(wb.value))


def de_batch_create(params, pop0, pop1, fit0, fit1, work, work_bytes, plan,
                    stream):
    h = ctypes.c_void_p()
    pl = None
    if plan is not None:
        pl = (ctypes.c_int32 * len(plan))(*plan)
    _check(_lib.de_batch_create(ctypes.byref(params), pop0, pop1, fit0, fit1,
                                work, work_bytes, pl, stream, ctypes.byref(h)),
           "de_batch_create")
    return h


def de_batch_plan(handle, ninst: int):
    plan = (ctypes.c_int32 * ninst)()
    us = (ctypes.c_float * (ninst * DE_BATCH_NVARIANTS))()
    _check(_lib.de_batch_plan(handle, plan, us), "de_batch_plan")
    return list(plan), [list(us[k * DE_BATCH_NVARIANTS:(k + 1) * DE_BATCH_NVARIANTS])
                        for k in range(ninst)]


def de_batch_generation(handle, n_gens: int, stream):
    _check(_lib.de_batch_generation(handle, n_gens, stream),
           "de_batch_generation")


def de_batch_read(handle, stream, nruns: int):
    best = (ctypes.c_double * nruns)()
    idx = (ctypes.c_int32 * nruns)()
    acc = (ctypes.c_int64 * nruns)()
    hit = (ctypes.c_int64 * nruns)()
    _check(_lib.de_batch_read(handle, stream, best, idx, acc, hit),
           "de_batch_read")
    return dict(best_f=list(best), best_idx=list(idx), accepted=list(acc),
                hit_gen=list(hit))


def de_batch_get_generation(handle) -> int:
    g = ctypes.c_int64(0)
    _check(_lib.de_batch_get_generation(handle, ctypes.byref(g)),
           "de_batch_get_generation")
    return int(g.value)


def de_batch_destroy(handle):
    _check(_lib.de_batch_destroy(handle), "de_batch_destroy")


# ---- owner of the caller-side buffers --------------------------------------

class DifferentialEvolution:
    """Device buffers (PyTorch) plus a library handle for one problem.

    ``o`` (D floats) and, for 'rot_osc', ``R`` (D x D, row-major, z = R y)
    may be NumPy arrays or tensors; they are copied to the device.
    ``jde``: None (plain DE/rand/1/bin), True (Brest et al. constants) or a
    dict with F_lo, F_span, tau_F, tau_CR; F and CR are then the starting
    values of every individual.
    """

    def __init__(self, *, runs, NP, D, F, CR, lo=-100.0, hi=100.0, seed=1,
                 kind="sphere", o, R=None, gemm_prec="bf16", ldx=None,
                 device="cuda", stream=None, jde=None):
        import torch
        self.torch = torch
        self.runs, self.NP, self.D = int(runs), int(NP), int(D)
        self.kind = kind
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ldx = int(ldx) if ldx is not None else (self.D + 3) // 4 * 4
        dev = self.device
        self.o = torch.as_tensor(o, dtype=torch.float32).to(dev).contiguous()
        self.R = None
        if kind == "rot_osc":
            self.R = torch.as_tensor(R, dtype=torch.float32).to(dev).contiguous()
        self.params = de_params(self.runs, self.NP, self.D, float(F), float(CR),
                                float(lo), float(hi), int(seed))
        self.objective = de_objective(
            _KINDS[kind], _PRECS[gemm_prec], self.D, 0, self.o.data_ptr(),
            self.R.data_ptr() if self.R is not None else None)
        wbytes = de_workspace_bytes(self.params, self.objective)
        rows = self.runs * self.NP
        self.pop = [torch.zeros(rows * self.ldx, dtype=torch.float32, device=dev)
                    for _ in range(2)]
        self.fit = [torch.zeros(rows, dtype=torch.float32, device=dev)
                    for _ in range(2)]
        self.work = torch.zeros(wbytes + 256, dtype=torch.uint8, device=dev)
        wptr = (self.work.data_ptr() + 255) // 256 * 256
        self.buffers = de_buffers(
            (ctypes.c_void_p * 2)(self.pop[0].data_ptr(), self.pop[1].data_ptr()),
            (ctypes.c_void_p * 2)(self.fit[0].data_ptr(), self.fit[1].data_ptr()),
            self.ldx, 0, wptr, wbytes)
        if jde:
            j = dict(JDE_BREST) if jde is True else dict(jde)
            self.jde = de_jde(j["F_lo"], j["F_span"], j["tau_F"], j["tau_CR"])
            self.handle = de_init_population_jde(self.params, self.objective,
                                                 self.jde, self.buffers,
                                                 self._s())
        else:
            self.jde = None
            self.handle = de_init_population(self.params, self.objective,
                                             self.buffers, self._s())

    def _s(self):
        return self.stream.cuda_stream

    def close(self):
        if getattr(self, "handle", None) is not None:
            de_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def gen(self) -> int:
        return de_get_generation(self.handle)

    def generation(self, n: int = 1):
        de_generation(self.handle, n, self._s())

    def evolve(self, max_gens: int, target: float = 1e-8, check_every: int = 50):
        return de_evolve(self.handle, max_gens, target, check_every, self._s(),
                         self.runs)

    def best(self, run: int = 0):
        return de_best(self.handle, run, self._s(), self.D)

    def best_f64(self):
        """FP64 objective of each run's best row: (values, indices)."""
        return de_best_f64(self.handle, self._s(), self.runs)

    def stats(self):
        return de_read_stats(self.handle, self._s(), self.runs)

    def control(self):
        """jDE: (F, CR) of the current generation as float32 [runs, NP]."""
        import numpy as np
        F, CR = de_get_control(self.handle, self._s(), self.runs * self.NP)
        return (np.asarray(F, np.float32).reshape(self.runs, self.NP),
                np.asarray(CR, np.float32).reshape(self.runs, self.NP))

    def set_control(self, F, CR):
        import numpy as np
        de_set_control(self.handle, self._s(),
                       np.asarray(F, np.float32).ravel().tolist(),
                       np.asarray(CR, np.float32).ravel().tolist())

    def population(self, gen=None):
        """View [runs, NP, D] of pop[gen & 1] (current generation by default)."""
        g = self.gen if gen is None else gen
        return self.pop[g & 1].view(self.runs, self.NP, self.ldx)[:, :, :self.D]

    def fitness(self, gen=None):
        g = self.gen if gen is None else gen
        return self.fit[g & 1].view(self.runs, self.NP)

    def load_population(self, pop, gen: int):
        """Write pop [runs, NP, D] as generation `gen` and re-evaluate it."""
        self.pop[gen & 1].view(self.runs, self.NP, self.ldx)[:, :, :self.D].copy_(
            self.torch.as_tensor(pop, dtype=self.torch.float32))
        de_load_population(self.handle, gen, self._s())

    def eval(self, x):
        """Objective of rows x [n, D] (through the library's kernels)."""
        torch = self.torch
        x = torch.as_tensor(x, dtype=torch.float32).to(self.device)
        n = x.shape[0]
        xp = torch.zeros((n, self.ldx), dtype=torch.float32, device=self.device)
        xp[:, :self.D] = x
        f = torch.empty(n, dtype=torch.float32, device=self.device)
        de_eval(self.handle, xp.data_ptr(), n, self.ldx, f.data_ptr(), self._s())
        return f

    def debug_draws(self, gen: int):
        torch = self.torch
        idx = torch.empty((self.runs, self.NP, 4), dtype=torch.int32, device=self.device)
        nw = (self.D + 31) // 32
        mask = torch.empty((self.runs, self.NP, nw), dtype=torch.int32, device=self.device)
        de_debug_draws(self.handle, gen, idx.data_ptr(), mask.data_ptr(), self._s())
        return idx, mask


class DEBatch:
    """Many independent rotated-objective runs of mixed size (de_batch.h).

    ``specs``: sequence of (NP, D, F, CR).  ``instances``: dict D -> (o, R)
    (arrays, D floats and D x D row-major), one per distinct D.
    ``plan``: None (autotune), or a dict D -> variant (DE_BATCH_*).
    """

    def __init__(self, specs, instances, *, lo=-100.0, hi=100.0, seed=1,
                 graph_gens=16, target=1e-8, plan=None, device="cuda",
                 stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.specs = [(int(a), int(b), float(c), float(e)) for a, b, c, e in specs]
        self.nruns = len(self.specs)
        dims = sorted(instances)
        self.dims = dims
        dev = self.device
        self._o = [torch.as_tensor(instances[D][0], dtype=torch.float32).to(dev).contiguous()
                   for D in dims]
        self._R = [torch.as_tensor(instances[D][1], dtype=torch.float32).to(dev).contiguous()
                   for D in dims]
        self._runs = (de_run_spec * self.nruns)(*[de_run_spec(*s) for s in self.specs])
        self._inst = (de_batch_instance * len(dims))(
            *[de_batch_instance(D, D, o.data_ptr(), R.data_ptr())
              for D, o, R in zip(dims, self._o, self._R)])
        self.params = de_batch_params(self.nruns, len(dims), self._runs,
                                      self._inst, float(lo), float(hi),
                                      int(seed), DE_GEMM_BF16, int(graph_gens),
                                      float(target))
        lay = de_batch_layout(self.params)
        self.layout = lay
        self.pop = [torch.zeros(max(lay["pop_floats"], 1), dtype=torch.float32,
                                device=dev) for _ in range(2)]
        self.fit = [torch.zeros(max(lay["fit_floats"], 1), dtype=torch.float32,
                                device=dev) for _ in range(2)]
        wb = lay["work_bytes"]
        self.work = torch.zeros(wb + 256, dtype=torch.uint8, device=dev)
        wptr = (self.work.data_ptr() + 255) // 256 * 256
        pl = None
        if plan is not None:
            pl = [int(plan.get(D, DE_BATCH_AUTO)) for D in dims]
        self.handle = de_batch_create(
            self.params, self.pop[0].data_ptr(), self.pop[1].data_ptr(),
            self.fit[0].data_ptr(), self.fit[1].data_ptr(), wptr, wb, pl,
            self._s())
        # instance data was converted into the workspace
        del self._o, self._R

    def _s(self):
        return self.stream.cuda_stream

    def close(self):
        if getattr(self, "handle", None) is not None:
            de_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def gen(self) -> int:
        return de_batch_get_generation(self.handle)

    def generation(self, n: int = 1):
        de_batch_generation(self.handle, n, self._s())

    def read(self):
        return de_batch_read(self.handle, self._s(), self.nruns)

    def plan(self):
        """(variant per D, tuner microseconds per D and variant)."""
        plan, us = de_batch_plan(self.handle, len(self.dims))
        return dict(zip(self.dims, plan)), dict(zip(self.dims, us))

    def population(self, run: int, gen=None):
        """View [NP, D] of run `run` in generation gen (current by default)."""
        g = self.gen if gen is None else gen
        NP, D = self.specs[run][0], self.specs[run][1]
        off, ldx = self.layout["pop_off"][run], self.layout["ldx"][run]
        return self.pop[g & 1][off:off + NP * ldx].view(NP, ldx)[:, :D]

    def fitness(self, run: int, gen=None):
        g = self.gen if gen is None else gen
        off = self.layout["fit_off"][run]
        return self.fit[g & 1][off:off + self.specs[run][0]]


class SurrogateDE:
    """Surrogate-assisted DE on a composition objective (de_surrogate.h).

    ``comp``: (O [n, D], R [n, D, D], bias [n], sigma).  ``settings``:
    overrides of SURROGATE_DEFAULTS (whose archive grows to NP when NP is
    larger).  Populations are views as in
    DifferentialEvolution; the model state is read and written as NumPy.
    """

    def __init__(self, *, runs, NP, D, F, CR, comp, lo=-100.0, hi=100.0,
                 seed=1, device="cuda", stream=None, **settings):
        import numpy as np
        import torch
        self.torch, self.np = torch, np
        self.runs, self.NP, self.D = int(runs), int(NP), int(D)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ldx = (self.D + 3) // 4 * 4
        O, R, bias, sigma = comp
        dev = self.device
        self._O = torch.as_tensor(np.asarray(O, np.float32)).to(dev).contiguous()
        self._R = torch.as_tensor(np.asarray(R, np.float32)).to(dev).contiguous()
        self._bias = (ctypes.c_float * len(bias))(*[float(b) for b in bias])
        self.comp = de_composition(len(bias), self.D, float(sigma), 0,
                                   self._O.data_ptr(), self._R.data_ptr(),
                                   self._bias)
        cfg = dict(SURROGATE_DEFAULTS)
        # the archive holds at least one generation's evaluations
        cfg["archive"] = max(cfg["archive"], self.NP)
        cfg.update(settings)
        self.cfg = cfg
        self.sp = de_surrogate_params(*[cfg[f] for f, _ in de_surrogate_params._fields_])
        self.params = de_params(self.runs, self.NP, self.D, float(F), float(CR),
                                float(lo), float(hi), int(seed))
        wb = ctypes.c_size_t()
        _check(_lib.de_sur_workspace_bytes(ctypes.byref(self.params),
                                           ctypes.byref(self.comp),
                                           ctypes.byref(self.sp),
                                           ctypes.byref(wb)),
               "de_sur_workspace_bytes")
        rows = self.runs * self.NP
        self.pop = [torch.zeros(rows * self.ldx, dtype=torch.float32, device=dev)
                    for _ in range(2)]
        self.fit = [torch.zeros(rows, dtype=torch.float32, device=dev)
                    for _ in range(2)]
        self.work = torch.zeros(wb.value + 256, dtype=torch.uint8, device=dev)
        wptr = (self.work.data_ptr() + 255) // 256 * 256
        self.buffers = de_buffers(
            (ctypes.c_void_p * 2)(self.pop[0].data_ptr(), self.pop[1].data_ptr()),
            (ctypes.c_void_p * 2)(self.fit[0].data_ptr(), self.fit[1].data_ptr()),
            self.ldx, 0, wptr, wb.value)
        h = ctypes.c_void_p()
        _check(_lib.de_sur_init(ctypes.byref(self.params),
                                ctypes.byref(self.comp), ctypes.byref(self.sp),
                                ctypes.byref(self.buffers), self._s(),
                                ctypes.byref(h)), "de_sur_init")
        self.handle = h
        self.P = int(_lib.de_sur_model_size(self.D, cfg["hidden"]))

    def _s(self):
        return self.stream.cuda_stream

    def close(self):
        if getattr(self, "handle", None) is not None:
            _check(_lib.de_sur_destroy(self.handle), "de_sur_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def gen(self) -> int:
        g = ctypes.c_int64()
        _check(_lib.de_sur_get_generation(self.handle, ctypes.byref(g)),
               "de_sur_get_generation")
        return int(g.value)

    def generation(self, n: int = 1):
        _check(_lib.de_sur_generation(self.handle, n, self._s()),
               "de_sur_generation")

    def train(self, n: int = 1):
        _check(_lib.de_sur_train(self.handle, n, self._s()), "de_sur_train")

    def read(self):
        n = self.runs
        best = (ctypes.c_double * n)()
        idx = (ctypes.c_int32 * n)()
        acc = (ctypes.c_int64 * n)()
        _check(_lib.de_sur_read(self.handle, self._s(), best, idx, acc),
               "de_sur_read")
        return dict(best_f=list(best), best_idx=list(idx), accepted=list(acc))

    def population(self, gen=None):
        g = self.gen if gen is None else gen
        return self.pop[g & 1].view(self.runs, self.NP, self.ldx)[:, :, :self.D]

    def fitness(self, gen=None):
        g = self.gen if gen is None else gen
        return self.fit[g & 1].view(self.runs, self.NP)

    def _rows(self, x):
        torch = self.torch
        x = torch.as_tensor(x, dtype=torch.float32).to(self.device)
        xp = torch.zeros((x.shape[0], self.ldx), dtype=torch.float32,
                         device=self.device)
        xp[:, :self.D] = x
        return xp

    def eval(self, x):
        xp = self._rows(x)
        f = self.torch.empty(xp.shape[0], dtype=self.torch.float32,
                             device=self.device)
        _check(_lib.de_sur_eval(self.handle, xp.data_ptr(), xp.shape[0],
                                self.ldx, f.data_ptr(), self._s()),
               "de_sur_eval")
        return f

    def predict(self, run, x):
        xp = self._rows(x)
        y = self.torch.empty(xp.shape[0], dtype=self.torch.float32,
                             device=self.device)
        _check(_lib.de_sur_predict(self.handle, run, xp.data_ptr(),
                                   xp.shape[0], self.ldx, y.data_ptr(),
                                   self._s()), "de_sur_predict")
        return y

    def get_model(self):
        np = self.np
        n = self.runs * self.P
        th, m, v = (np.empty(n, np.float32) for _ in range(3))
        step = ctypes.c_int64()
        fp = ctypes.POINTER(ctypes.c_float)
        _check(_lib.de_sur_get_model(self.handle, self._s(),
                                     th.ctypes.data_as(fp), m.ctypes.data_as(fp),
                                     v.ctypes.data_as(fp), ctypes.byref(step)),
               "de_sur_get_model")
        shp = (self.runs, self.P)
        return th.reshape(shp), m.reshape(shp), v.reshape(shp), int(step.value)

    def set_model(self, theta, m, v, step):
        np = self.np
        fp = ctypes.POINTER(ctypes.c_float)
        arrs = [np.ascontiguousarray(a, np.float32).ravel() for a in (theta, m, v)]
        _check(_lib.de_sur_set_model(self.handle, self._s(),
                                     *[a.ctypes.data_as(fp) for a in arrs],
                                     int(step)), "de_sur_set_model")

    def archive(self):
        np = self.np
        cap = self.cfg["archive"]
        X = np.empty((self.runs, cap, self.D), np.float32)
        T = np.empty((self.runs, cap), np.float32)
        filled = (ctypes.c_int64 * self.runs)()
        fp = ctypes.POINTER(ctypes.c_float)
        _check(_lib.de_sur_get_archive(self.handle, self._s(),
                                       X.ctypes.data_as(fp),
                                       T.ctypes.data_as(fp), filled),
               "de_sur_get_archive")
        return X, T, list(filled)

    def last(self):
        np = self.np
        k = self.cfg["k"]
        cand = np.empty((self.runs, self.NP, k, self.D), np.float32)
        pred = np.empty((self.runs, self.NP, k), np.float32)
        choice = np.empty((self.runs, self.NP), np.int32)
        fp = ctypes.POINTER(ctypes.c_float)
        _check(_lib.de_sur_last(self.handle, self._s(), cand.ctypes.data_as(fp),
                                pred.ctypes.data_as(fp),
                                choice.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
               "de_sur_last")
        return cand, pred, choice
