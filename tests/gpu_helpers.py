"""Shared helpers of the GPU parity tests (the oracle is the reference)."""
from __future__ import annotations

import math
import os

import numpy as np

import oracle
from paper_2405_16551_amd import instances

LO, HI = -100.0, 100.0
FP32_RTOL = 1e-5  # one-generation fitness tolerance in FP32


def make_de(*, runs, NP, D, F=0.5, CR=0.9, seed=1, kind="sphere",
            gemm_prec="fp32", obj_seed=1, ldx=None, jde=None, lo=LO, hi=HI):
    from paper_2405_16551_amd.de import DifferentialEvolution
    o, R = instances.make_instance(kind, D, obj_seed)
    de = DifferentialEvolution(runs=runs, NP=NP, D=D, F=F, CR=CR, lo=lo,
                               hi=hi, seed=seed, kind=kind, o=o, R=R,
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


def host_threads() -> int:
    """Host threads for the oracle: the CPUs this process may use, at most
    16 (the share of one GPU's host)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def rounding_band(kind, u, o, R, tol):
    """Bound on |f(u) - f(u')| when |u' - u| <= tol coordinate-wise: how far
    the FP32 rounding of the trial coordinates can move the objective.
    Sphere: sum 2|y_j| tol_j + tol_j^2.  Rotated: ||R (u' - u)|| <= ||tol||,
    |d/dz (z^2 + sin^2 3z)| <= 2|z| + 3 and the second derivative <= 20.
    u and tol may be [D] or [n, D] (one bound per row)."""
    y = np.asarray(u, dtype=np.float64) - np.asarray(o, dtype=np.float64)
    tol = np.asarray(tol, dtype=np.float64)
    if kind == oracle.OBJ_SPHERE:
        b = np.sum(2 * np.abs(y) * tol + tol * tol, axis=-1)
    else:
        z = y @ np.asarray(R, dtype=np.float64).T
        tn = np.linalg.norm(tol, axis=-1)
        b = ((2 * np.linalg.norm(z, axis=-1) + 3 * math.sqrt(y.shape[-1])) * tn
             + 10 * tn * tn)
    return float(b) if np.ndim(b) == 0 else b


# Near-tie ceiling.  A row is a near-tie when |f_trial - f_target| lies
# within the band (the fitness bar f_rtol, at most 8 * 2^-8 / sqrt(D) ~ 3% at
# D = 1 for the BF16 product, plus the trial's FP32 rounding band); there
# either selection outcome is correct and only the row's content is
# checked.  Away from the optimum a generation's trial/target ratios spread
# over far more than the band (trial and target differ in a fraction CR of
# their coordinates), so at most 10% of the rows may be near-ties: the other
# 90% must reproduce the oracle's decision exactly.  Next to the optimum,
# where the FP32 rounding of the trial's coordinates moves f by more than f
# itself, the decision is not fixed by the arithmetic and callers state so.
TIE_SHARE = 0.10
# With the FP32 product the bar is 1e-5 relative: the band is dominated by
# the trial's rounding, and at most 2% of the rows may be near-ties away
# from the optimum.
FP32_TIE_SHARE = 0.02


class GenCmp:
    """Outcome of one compared generation."""

    def __init__(self, n, ties, accepts, rejects):
        self.n, self.ties = n, ties
        self.accepts, self.rejects = accepts, rejects  # decided rows

    def __iter__(self):  # n, ties = compare_generation(...)
        return iter((self.n, self.ties))

    def report(self, label=""):
        print(f"{label}: rows {self.n}, decided {self.n - self.ties} "
              f"({self.accepts} accepted, {self.rejects} rejected), "
              f"near-ties {self.ties}", flush=True)

    def check(self, label="", share=None, floor=2):
        """Print the counts and assert the near-tie ceiling (share of the
        compared rows, TIE_SHARE unless given; at least `floor` rows)."""
        share = TIE_SHARE if share is None else share
        self.report(label)
        assert self.ties <= max(floor, share * self.n), (
            f"{label}: {self.ties} near-ties of {self.n} rows")


def compare_generation(gpu_pop, gpu_fit, pop32, fit_gpu_prev, *, F, CR, seed,
                       gen, kind, o, R, f_rtol, rows=None, run0=0,
                       lo=LO, hi=HI):
    """Compare one GPU generation g -> g+1 with the oracle's, started from
    the same FP32 population.  Returns a GenCmp (unpacks as n, ties).

    gpu_pop [runs,NP,D] / gpu_fit [runs,NP]: GPU generation g+1.
    pop32 [runs,NP,D]: generation g (FP32, shared input).
    fit_gpu_prev: GPU fitness of generation g (the targets' f on the GPU).
    run0: run number of the first run (draw counter), for runs of a batch.

    Checks, on every compared row: the GPU's target fitness against the
    oracle's FP64 evaluation of the same FP32 vector (f_rtol); a row the GPU
    replaced holds the trial (coordinates within one FP32 fused rounding of
    the oracle's FP64 trial) and its f within f_rtol of the oracle's FP64 f
    of that FP32 row; a row the GPU kept is copied exactly with its f; and
    the selection decision equals the oracle's unless |f_trial - f_target|
    is within f_rtol plus the rounding band of the trial coordinates (a
    near-tie: either outcome is correct).
    """
    pop64 = pop32.astype(np.float64)
    runs, NP, D = pop64.shape
    nt = host_threads()
    fit64 = oracle.objective_batch(kind, pop64.reshape(-1, D), o, R,
                                   nthreads=nt).reshape(runs, NP)
    np.testing.assert_allclose(fit_gpu_prev, fit64, rtol=f_rtol, atol=1e-30)
    out = oracle.generation(pop64, fit64, F=F, CR=CR, lo=lo, hi=hi, seed=seed,
                            gen=gen, kind=kind, o=o, R=R, nthreads=nt,
                            run0=run0)
    it = rows if rows is not None else [(r, i) for r in range(runs)
                                        for i in range(NP)]
    rr = np.array([r for r, _ in it], dtype=np.int64)
    ii = np.array([i for _, i in it], dtype=np.int64)
    d = out["draws"][rr, ii]
    tol = trial_atol(pop64[rr, d[:, 0]], pop64[rr, d[:, 1]],
                     pop64[rr, d[:, 2]], F)
    fu, fx = out["ftrial"][rr, ii], fit64[rr, ii]
    band = (f_rtol * np.maximum(np.abs(fu), np.abs(fx)) +
            rounding_band(kind, out["trial"][rr, ii], o, R, tol))
    near = np.abs(fu - fx) <= band
    acc_o = out["accept"][rr, ii].astype(bool)
    g_rows, g_fit = gpu_pop[rr, ii], gpu_fit[rr, ii]
    p_rows, p_fit = pop32[rr, ii], fit_gpu_prev[rr, ii]
    acc_g = (g_rows != p_rows).any(axis=1) | (g_fit != p_fit)
    # the decision, away from near-ties
    bad = np.nonzero(~near & (acc_g != acc_o))[0]
    assert bad.size == 0, [(int(rr[k]), int(ii[k]), fu[k], fx[k],
                            float(g_fit[k])) for k in bad[:5]]
    # kept rows: copied exactly, with their value
    kept = np.nonzero(~acc_g)[0]
    np.testing.assert_array_equal(g_rows[kept], p_rows[kept])
    np.testing.assert_array_equal(g_fit[kept], p_fit[kept])
    # replaced rows: the trial, and its value
    rep = np.nonzero(acc_g)[0]
    if rep.size:
        err = np.abs(g_rows[rep].astype(np.float64) - out["trial"][rr, ii][rep])
        over = np.nonzero((err > tol[rep]).any(axis=1))[0]
        assert over.size == 0, [(int(rr[rep[k]]), int(ii[rep[k]]),
                                 float(err[k].max())) for k in over[:5]]
        f_own = oracle.objective_batch(kind, g_rows[rep].astype(np.float64), o,
                                       R, nthreads=nt)
        ferr = np.abs(g_fit[rep] - f_own)
        off = np.nonzero(ferr > f_rtol * np.abs(f_own))[0]
        assert off.size == 0, [(int(rr[rep[k]]), int(ii[rep[k]]),
                                float(g_fit[rep[k]]), f_own[k])
                               for k in off[:5]]
    ties = int(near.sum())
    return GenCmp(len(it), ties, int((~near & acc_o).sum()),
                  int((~near & ~acc_o).sum()))
