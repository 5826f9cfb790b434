"""Shared helpers of the GPU parity tests (the oracle is the reference)."""
from __future__ import annotations

import math

import numpy as np

import oracle
from paper_2405_16551_amd import instances

LO, HI = -100.0, 100.0
FP32_RTOL = 1e-5  # one-generation fitness tolerance in FP32


def make_de(*, runs, NP, D, F=0.5, CR=0.9, seed=1, kind="sphere",
            gemm_prec="fp32", obj_seed=1, ldx=None, jde=None):
    from paper_2405_16551_amd.de import DifferentialEvolution
    o, R = instances.make_instance(kind, D, obj_seed)
    de = DifferentialEvolution(runs=runs, NP=NP, D=D, F=F, CR=CR, lo=LO,
                               hi=HI, seed=seed, kind=kind, o=o, R=R,
                               gemm_prec=gemm_prec, ldx=ldx, jde=jde)
    return de, o, R


def okind(kind: str) -> int:
    return oracle.OBJ_SPHERE if kind == "sphere" else oracle.OBJ_ROT_OSC


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def trial_atol(x1, x2, x3, F):
    """Bound on |fmaf(F, x2 - x3, x1) - (x1 + F (x2 - x3))| for FP32 inputs:
    one rounding of the difference and one of the fused result."""
    return 2.0 ** -22 * (np.abs(x1) + F * (np.abs(x2) + np.abs(x3))) + 1e-30


def rounding_band(kind, u, o, R, tol):
    """Bound on |f(u) - f(u')| when |u' - u| <= tol coordinate-wise: how far
    the FP32 rounding of the trial coordinates can move the objective.
    Sphere: sum 2|y_j| tol_j + tol_j^2.  Rotated: ||R (u' - u)|| <= ||tol||,
    |d/dz (z^2 + sin^2 3z)| <= 2|z| + 3 and the second derivative <= 20."""
    y = u - np.asarray(o, dtype=np.float64)
    if kind == oracle.OBJ_SPHERE:
        return float(np.sum(2 * np.abs(y) * tol + tol * tol))
    z = np.asarray(R, dtype=np.float64) @ y
    tn = float(np.linalg.norm(tol))
    return (2 * float(np.linalg.norm(z)) + 3 * math.sqrt(len(y))) * tn + 10 * tn * tn


def compare_generation(gpu_pop, gpu_fit, pop32, fit_gpu_prev, *, F, CR, seed,
                       gen, kind, o, R, f_rtol, rows=None, run0=0):
    """Compare one GPU generation g -> g+1 with the oracle's, started from
    the same FP32 population.  Returns (n_rows_compared, n_near_ties).

    gpu_pop [runs,NP,D] / gpu_fit [runs,NP]: GPU generation g+1.
    pop32 [runs,NP,D]: generation g (FP32, shared input).
    fit_gpu_prev: GPU fitness of generation g (the targets' f on the GPU).
    run0: run number of the first run (draw counter), for runs of a batch.

    Checks: the GPU's target fitness and the GPU's accepted trial's fitness
    against the oracle's FP64 evaluation of the same FP32 vectors (f_rtol);
    accepted trial coordinates within one FP32 fused rounding of the
    oracle's FP64 trial; rejected rows copied exactly; and the selection
    decision identical unless |f_trial - f_target| is within f_rtol plus the
    rounding band of the trial coordinates.
    """
    pop64 = pop32.astype(np.float64)
    runs, NP, D = pop64.shape
    fit64 = oracle.objective_batch(kind, pop64.reshape(-1, D), o, R,
                                   nthreads=8).reshape(runs, NP)
    np.testing.assert_allclose(fit_gpu_prev, fit64, rtol=f_rtol, atol=1e-30)
    out = oracle.generation(pop64, fit64, F=F, CR=CR, lo=LO, hi=HI, seed=seed,
                            gen=gen, kind=kind, o=o, R=R, nthreads=8,
                            run0=run0)
    ties = 0
    n = 0
    it = rows if rows is not None else [(r, i) for r in range(runs)
                                        for i in range(NP)]
    for r, i in it:
        fu, fx = out["ftrial"][r, i], fit64[r, i]
        d = out["draws"][r, i]
        tol = trial_atol(pop64[r, d[0]], pop64[r, d[1]], pop64[r, d[2]], F)
        band = (f_rtol * max(abs(fu), abs(fx)) +
                rounding_band(kind, out["trial"][r, i], o, R, tol))
        acc_o = bool(out["accept"][r, i])
        acc_g = not np.array_equal(gpu_pop[r, i], pop32[r, i]) or (
            gpu_fit[r, i] != fit_gpu_prev[r, i])
        n += 1
        if abs(fu - fx) <= band:
            ties += 1
            if not acc_g:
                np.testing.assert_array_equal(gpu_pop[r, i], pop32[r, i])
            continue
        assert acc_g == acc_o, (r, i, fu, fx, gpu_fit[r, i])
        if acc_o:
            err = np.abs(gpu_pop[r, i].astype(np.float64) - out["trial"][r, i])
            assert (err <= tol).all(), (r, i, err.max())
            f_own = oracle.objective(kind, gpu_pop[r, i].astype(np.float64), o, R)
            assert abs(gpu_fit[r, i] - f_own) <= f_rtol * f_own, (
                r, i, gpu_fit[r, i], f_own)
        else:
            np.testing.assert_array_equal(gpu_pop[r, i], pop32[r, i])
            assert gpu_fit[r, i] == fit_gpu_prev[r, i]
    return n, ties
