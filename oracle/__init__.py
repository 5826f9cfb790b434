"""FP64 CPU oracle for DE/rand/1/bin -- TEST INFRASTRUCTURE, not product code.

Thin ctypes wrapper over ``de_oracle.c`` (plain scalar C, FP64).  Only the
test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the GPU library never does.

What it computes follows Section 2 of Janssen, Pullan & Liew (arXiv
2405.16551): random initialisation in the box, DE/rand/1 mutation (eq. 2),
binomial crossover (eq. 3) and greedy one-to-one selection, plus the
shifted/rotated objectives of Section 7.3.1.  The readings taken where the
paper is silent are listed in ``de_oracle.c``'s header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "de_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OBJ_SPHERE = 0
OBJ_ROT_OSC = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile de_oracle.c with gcc (-O2, no fast-math, OpenMP) in place."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
             "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if (not os.path.exists(_LIB)
            or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    u32p, i32p, i64p, dp = (P(ctypes.c_uint32), P(ctypes.c_int32),
                            P(ctypes.c_int64), P(ctypes.c_double))
    c_int, c_dbl, c_u64, c_i64 = (ctypes.c_int, ctypes.c_double,
                                  ctypes.c_uint64, ctypes.c_int64)
    lib.oracle_philox_batch.argtypes = [u32p, u32p, u32p, c_i64]
    lib.oracle_uniform_index.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.oracle_uniform_index.restype = ctypes.c_uint32
    lib.oracle_skip_triple.argtypes = [c_int, c_int, c_int, c_int, i32p]
    lib.oracle_draw_indices.argtypes = [c_u64, c_int, c_i64, c_int, c_int,
                                        c_int, i32p]
    lib.oracle_take_mutant.argtypes = [c_u64, c_int, c_i64, c_int, c_int,
                                       c_int, c_dbl]
    lib.oracle_take_mutant.restype = c_int
    lib.oracle_objective.argtypes = [c_int, c_int, dp, dp, dp]
    lib.oracle_objective.restype = c_dbl
    lib.oracle_objective_batch.argtypes = [c_int, c_int, c_i64, dp, dp, dp,
                                           dp, c_int]
    lib.oracle_init.argtypes = [c_int, c_int, c_int, c_int, c_dbl, c_dbl,
                                c_u64, dp]
    lib.oracle_generation.argtypes = [
        c_int, c_int, c_int, c_int, c_dbl, c_dbl, c_dbl, c_dbl, c_u64, c_i64, c_int,
        dp, dp, dp, dp, dp, dp, dp, dp, i32p, i32p, c_int]
    lib.oracle_jde_generation.argtypes = [
        c_int, c_int, c_int, c_int, c_dbl, c_dbl, c_dbl, c_dbl, c_dbl, c_dbl,
        c_u64, c_i64, c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp,
        i32p, dp, dp, c_int]
    lib.oracle_composition_batch.argtypes = [c_int, c_int, c_i64, dp, dp, dp,
                                             dp, c_dbl, dp, c_int]
    lib.oracle_mlp_size.argtypes = [c_int, c_int]
    lib.oracle_mlp_size.restype = c_i64
    lib.oracle_mlp_forward.argtypes = [c_int, c_int, dp, c_dbl, c_dbl, c_i64,
                                       dp, dp]
    lib.oracle_mlp_grad.argtypes = [c_int, c_int, dp, c_dbl, c_dbl, c_int, dp,
                                    dp, dp]
    lib.oracle_mlp_grad.restype = c_dbl
    lib.oracle_mlp_adam_step.argtypes = [c_int, c_int, dp, dp, dp, c_i64,
                                         c_dbl, c_dbl, c_dbl, c_dbl, c_dbl,
                                         c_dbl, c_int, dp, dp]
    lib.oracle_mlp_adam_step.restype = c_dbl
    lib.oracle_sur_generation.argtypes = [
        c_int, c_int, c_int, c_int, c_int, c_dbl, c_dbl, c_dbl, c_dbl, c_u64,
        c_i64, c_int, c_int, dp, c_int, dp, dp, dp, c_dbl, dp, dp, dp, dp, dp,
        dp, i32p, dp, i32p, c_int]
    lib.oracle_run.argtypes = [
        c_int, c_int, c_int, c_dbl, c_dbl, c_dbl, c_dbl, c_u64, c_int, dp, dp,
        c_i64, c_dbl, dp, i64p, i64p, dp, dp, c_int]
    lib.oracle_run.restype = c_int
    lib.oracle_max_threads.restype = c_int
    _lib = lib
    return lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def philox(ctr, key):
    """Philox4x32-10 of counters [n,4] under keys [n,2] (uint32) -> [n,4]."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    assert ctr.shape[0] == key.shape[0]
    out = np.empty_like(ctr)
    _load().oracle_philox_batch(_ptr(ctr, ctypes.c_uint32),
                                _ptr(key, ctypes.c_uint32),
                                _ptr(out, ctypes.c_uint32), ctr.shape[0])
    return out


def uniform_index(w: int, n: int) -> int:
    return int(_load().oracle_uniform_index(w, n))


def skip_triple(i: int, a: int, b: int, c: int):
    out = np.zeros(3, dtype=np.int32)
    _load().oracle_skip_triple(i, a, b, c, _ptr(out, ctypes.c_int32))
    return tuple(int(v) for v in out)


def draw_indices(seed: int, run: int, gen: int, i: int, NP: int, D: int):
    """(r1, r2, r3, j_rand) of individual i in generation gen."""
    out = np.zeros(4, dtype=np.int32)
    _load().oracle_draw_indices(seed, run, gen, i, NP, D,
                                _ptr(out, ctypes.c_int32))
    return tuple(int(v) for v in out)


def take_mutant(seed, run, gen, i, j, jrand, CR) -> bool:
    return bool(_load().oracle_take_mutant(seed, run, gen, i, j, jrand, CR))


def objective(kind: int, x, o, R=None) -> float:
    x, o = _f64(x), _f64(o)
    D = x.shape[-1]
    Rm = _f64(R) if R is not None else np.zeros(1)
    return float(_load().oracle_objective(kind, D, _ptr(x, ctypes.c_double),
                                          _ptr(o, ctypes.c_double),
                                          _ptr(Rm, ctypes.c_double)))


def objective_batch(kind: int, X, o, R=None, nthreads: int = 1):
    X, o = _f64(X), _f64(o)
    D = X.shape[-1]
    n = X.size // D
    Rm = _f64(R) if R is not None else np.zeros(1)
    f = np.empty(n, dtype=np.float64)
    _load().oracle_objective_batch(kind, D, n, _ptr(X, ctypes.c_double),
                                   _ptr(o, ctypes.c_double),
                                   _ptr(Rm, ctypes.c_double),
                                   _ptr(f, ctypes.c_double), nthreads)
    return f


def init_population(runs, NP, D, lo, hi, seed, run0: int = 0):
    """Generation 0 of runs run0 .. run0 + runs - 1 (run numbers enter the
    draw counter)."""
    pop = np.empty((runs, NP, D), dtype=np.float64)
    _load().oracle_init(runs, run0, NP, D, lo, hi, seed,
                        _ptr(pop, ctypes.c_double))
    return pop


def generation(pop, fit, *, F, CR, lo, hi, seed, gen, kind, o, R=None,
               nthreads: int = 1, run0: int = 0):
    """One synchronous generation.  pop [runs,NP,D], fit [runs,NP] (FP64);
    run r of the arrays is run number run0 + r of the draw counters.

    Returns a dict with pop_next, fit_next, trial, ftrial, accept, draws.
    """
    pop, fit, o = _f64(pop), _f64(fit), _f64(o)
    runs, NP, D = pop.shape
    Rm = _f64(R) if R is not None else np.zeros(1)
    out = dict(pop_next=np.empty_like(pop), fit_next=np.empty_like(fit),
               trial=np.empty_like(pop), ftrial=np.empty_like(fit),
               accept=np.empty((runs, NP), dtype=np.int32),
               draws=np.empty((runs, NP, 4), dtype=np.int32))
    dpt = ctypes.c_double
    _load().oracle_generation(
        runs, run0, NP, D, F, CR, lo, hi, seed, gen, kind, _ptr(o, dpt),
        _ptr(Rm, dpt), _ptr(pop, dpt), _ptr(fit, dpt),
        _ptr(out["pop_next"], dpt), _ptr(out["fit_next"], dpt),
        _ptr(out["trial"], dpt), _ptr(out["ftrial"], dpt),
        _ptr(out["accept"], ctypes.c_int32), _ptr(out["draws"], ctypes.c_int32),
        nthreads)
    return out


# jDE constants of Brest et al. (2006): F' = 0.1 + 0.9 u, tau_F = tau_CR = 0.1
JDE_F_LO, JDE_F_SPAN, JDE_TAU_F, JDE_TAU_CR = 0.1, 0.9, 0.1, 0.1


def jde_generation(pop, fit, F, CR, *, lo, hi, seed, gen, kind, o, R=None,
                   F_lo=JDE_F_LO, F_span=JDE_F_SPAN, tau_F=JDE_TAU_F,
                   tau_CR=JDE_TAU_CR, nthreads: int = 1, run0: int = 0):
    """One synchronous jDE generation.  pop [runs,NP,D], fit/F/CR [runs,NP]
    (FP64 holding FP32 control values).  F_lo, F_span, tau_F and tau_CR are
    taken as the float32 values the GPU library stores.  Returns a dict with
    pop_next, fit_next, F_next, CR_next, trial, ftrial, accept, Fp, CRp (the
    F' and CR' each trial used)."""
    pop, fit, o = _f64(pop), _f64(fit), _f64(o)
    F, CR = _f64(F), _f64(CR)
    runs, NP, D = pop.shape
    Rm = _f64(R) if R is not None else np.zeros(1)
    f32 = lambda v: float(np.float32(v))
    out = dict(pop_next=np.empty_like(pop), fit_next=np.empty_like(fit),
               F_next=np.empty_like(fit), CR_next=np.empty_like(fit),
               trial=np.empty_like(pop), ftrial=np.empty_like(fit),
               accept=np.empty((runs, NP), dtype=np.int32),
               Fp=np.empty_like(fit), CRp=np.empty_like(fit))
    dpt = ctypes.c_double
    _load().oracle_jde_generation(
        runs, run0, NP, D, f32(F_lo), f32(F_span), f32(tau_F), f32(tau_CR),
        lo, hi, seed, gen, kind, _ptr(o, dpt), _ptr(Rm, dpt), _ptr(pop, dpt),
        _ptr(fit, dpt), _ptr(F, dpt), _ptr(CR, dpt),
        _ptr(out["pop_next"], dpt), _ptr(out["fit_next"], dpt),
        _ptr(out["F_next"], dpt), _ptr(out["CR_next"], dpt),
        _ptr(out["trial"], dpt), _ptr(out["ftrial"], dpt),
        _ptr(out["accept"], ctypes.c_int32), _ptr(out["Fp"], dpt),
        _ptr(out["CRp"], dpt), nthreads)
    return out


def jde_run(*, runs, NP, D, F0, CR0, lo, hi, seed, kind, o, R=None, G,
            nthreads: int = 1, **jde):
    """A whole jDE run (init + G generations), returns best_trace
    [runs, G+1] and the final pop, fit, F, CR."""
    pop = init_population(runs, NP, D, lo, hi, seed)
    fit = objective_batch(kind, pop.reshape(-1, D), o, R,
                          nthreads=nthreads).reshape(runs, NP)
    F = np.full((runs, NP), float(np.float32(F0)))
    CR = np.full((runs, NP), float(np.float32(CR0)))
    best = np.empty((runs, G + 1))
    best[:, 0] = fit.min(axis=1)
    for g in range(G):
        out = jde_generation(pop, fit, F, CR, lo=lo, hi=hi, seed=seed, gen=g,
                             kind=kind, o=o, R=R, nthreads=nthreads, **jde)
        pop, fit, F, CR = (out["pop_next"], out["fit_next"], out["F_next"],
                           out["CR_next"])
        best[:, g + 1] = fit.min(axis=1)
    return dict(best_trace=best, pop=pop, fit=fit, F=F, CR=CR)


def run(*, runs, NP, D, F, CR, lo, hi, seed, kind, o, R=None, G, target=1e-8,
        nthreads: int = 1):
    """A whole run: init + G generations.  Returns best_trace [runs,G+1],
    hit_gen [runs] (-1 = never), accepted [runs], pop [runs,NP,D], fit."""
    o = _f64(o)
    Rm = _f64(R) if R is not None else np.zeros(1)
    best = np.empty((runs, G + 1), dtype=np.float64)
    hit = np.empty(runs, dtype=np.int64)
    acc = np.empty(runs, dtype=np.int64)
    pop = np.empty((runs, NP, D), dtype=np.float64)
    fit = np.empty((runs, NP), dtype=np.float64)
    dpt = ctypes.c_double
    rc = _load().oracle_run(runs, NP, D, F, CR, lo, hi, seed, kind,
                            _ptr(o, dpt), _ptr(Rm, dpt), G, target,
                            _ptr(best, dpt), _ptr(hit, ctypes.c_int64),
                            _ptr(acc, ctypes.c_int64), _ptr(pop, dpt),
                            _ptr(fit, dpt), nthreads)
    if rc != 0:
        raise MemoryError("oracle_run: allocation failed")
    return dict(best_trace=best, hit_gen=hit, accepted=acc, pop=pop, fit=fit)


# ---------------------------------------------------------------------------
# Composition objective, surrogate MLP and the surrogate-assisted generation.

def composition_batch(X, O, R, bias, sigma, nthreads: int = 1):
    """f of rows X [n, D] for the composition of len(bias) components:
    shifts O [n_c, D], rotations R [n_c, D, D]."""
    X = _f64(X)
    O, R, bias = _f64(O), _f64(R), _f64(bias)
    n_c, D = O.shape
    assert n_c <= 64
    X2 = X.reshape(-1, D)
    f = np.empty(X2.shape[0], dtype=np.float64)
    dpt = ctypes.c_double
    _load().oracle_composition_batch(D, n_c, X2.shape[0], _ptr(X2, dpt),
                                     _ptr(O, dpt), _ptr(R, dpt),
                                     _ptr(bias, dpt), float(sigma),
                                     _ptr(f, dpt), nthreads)
    return f.reshape(X.shape[:-1])


def mlp_size(D: int, H: int) -> int:
    return int(_load().oracle_mlp_size(D, H))


def mlp_forward(theta, X, *, D, H, lo, hi):
    theta, X = _f64(theta), _f64(X).reshape(-1, D)
    y = np.empty(X.shape[0], dtype=np.float64)
    dpt = ctypes.c_double
    _load().oracle_mlp_forward(D, H, _ptr(theta, dpt), lo, hi, X.shape[0],
                               _ptr(X, dpt), _ptr(y, dpt))
    return y


def mlp_grad(theta, X, T, *, D, H, lo, hi):
    theta, X, T = _f64(theta), _f64(X).reshape(-1, D), _f64(T)
    g = np.empty_like(theta)
    dpt = ctypes.c_double
    loss = _load().oracle_mlp_grad(D, H, _ptr(theta, dpt), lo, hi, X.shape[0],
                                   _ptr(X, dpt), _ptr(T, dpt), _ptr(g, dpt))
    return loss, g


def mlp_adam_step(theta, m, v, t, X, T, *, D, H, lo, hi, lr, beta1, beta2,
                  eps):
    """Returns (loss, theta', m', v') after one Adam step (t >= 1)."""
    theta, m, v = _f64(theta).copy(), _f64(m).copy(), _f64(v).copy()
    X, T = _f64(X).reshape(-1, D), _f64(T)
    dpt = ctypes.c_double
    loss = _load().oracle_mlp_adam_step(
        D, H, _ptr(theta, dpt), _ptr(m, dpt), _ptr(v, dpt), t, lr, beta1,
        beta2, eps, lo, hi, X.shape[0], _ptr(X, dpt), _ptr(T, dpt))
    return loss, theta, m, v


def sur_generation(pop, fit, theta, *, k, F, CR, lo, hi, seed, gen, use_model,
                   H, O, R, bias, sigma, run0: int = 0, nthreads: int = 1):
    """One surrogate-assisted generation; theta [runs, P] (one model per
    run).  Returns pop_next, fit_next, cand, pred, choice, ftrial, accept."""
    pop, fit = _f64(pop), _f64(fit)
    runs, NP, D = pop.shape
    theta = _f64(theta).reshape(runs, -1)
    O, R, bias = _f64(O), _f64(R), _f64(bias)
    out = dict(pop_next=np.empty_like(pop), fit_next=np.empty_like(fit),
               cand=np.empty((runs, NP, k, D)), pred=np.empty((runs, NP, k)),
               choice=np.empty((runs, NP), dtype=np.int32),
               ftrial=np.empty_like(fit),
               accept=np.empty((runs, NP), dtype=np.int32))
    dpt = ctypes.c_double
    _load().oracle_sur_generation(
        runs, run0, NP, D, k, F, CR, lo, hi, seed, gen, int(use_model), H,
        _ptr(theta, dpt), O.shape[0], _ptr(O, dpt), _ptr(R, dpt),
        _ptr(bias, dpt), float(sigma), _ptr(pop, dpt), _ptr(fit, dpt),
        _ptr(out["pop_next"], dpt), _ptr(out["fit_next"], dpt),
        _ptr(out["cand"], dpt), _ptr(out["pred"], dpt),
        _ptr(out["choice"], ctypes.c_int32), _ptr(out["ftrial"], dpt),
        _ptr(out["accept"], ctypes.c_int32), nthreads)
    return out
