"""GPU parity of jDE (per-individual F and CR, Brest et al. 2006; one of the
DE variants of Section 2, the cujDE of Section 8.2) against the FP64 oracle,
through the C ABI.

The adaptation constants are Brest et al.'s, not the paper's: parity is
pinned to the oracle's jDE rule (itself pinned to plain DE and to the rule's
distributions), not to values printed by the paper.

Bars: the trial's F' and CR' and every control value kept or replaced are
bit-exact (integer decisions, one fused rounding for F'); trial coordinates
within one FP32 fused rounding; fitness within 1e-5 (FP32) or the BF16 bar;
selection identical away from near-ties; 30-run distributions matched.
"""
import math

import numpy as np
import pytest

import oracle
from tests import de_stats
from tests.gpu_helpers import (FP32_RTOL, FP32_TIE_SHARE, HI, LO, GenCmp,
                               host, make_de, okind, rounding_band,
                               trial_atol)

pytestmark = pytest.mark.gpu


def bf16_rtol(D: int) -> float:
    return 8 * 2.0 ** -8 / math.sqrt(D)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    yield


def make_jde(**kw):
    return make_de(jde=kw.pop("jde", True), **kw)


@pytest.mark.parametrize("kind,prec,runs,NP,D", [
    ("sphere", "fp32", 3, 50, 37), ("sphere", "fp32", 2, 4, 1),
    ("sphere", "fp32", 3, 45, 600), ("sphere", "fp32", 2, 30, 1500),
    ("rot_osc", "fp32", 2, 70, 100), ("rot_osc", "bf16", 2, 130, 100),
    # more tiles (258) than compute units at padded width 256: 512-thread
    # tiles; at padded width 128 the same in the paired-row form
    ("rot_osc", "bf16", 2, 8256, 200),
    ("rot_osc", "bf16", 2, 8256, 100),
    # padded width 1024 (the headline width); NP = 100 leaves a ragged
    # last tile
    ("rot_osc", "bf16", 2, 100, 1000),
])
def test_jde_generation_matches_oracle(kind, prec, runs, NP, D):
    de, o, R = make_jde(runs=runs, NP=NP, D=D, F=0.5, CR=0.9, seed=3,
                        kind=kind, gemm_prec=prec)
    de.generation(7)
    g = de.gen
    pop32 = host(de.population()).copy()
    fprev = host(de.fitness()).copy()
    F0, CR0 = de.control()
    de.generation(1)
    pop_n, fit_n = host(de.population()), host(de.fitness())
    F1, CR1 = de.control()
    f_rtol = bf16_rtol(D) if prec == "bf16" else FP32_RTOL
    pop64 = pop32.astype(np.float64)
    fit64 = oracle.objective_batch(okind(kind), pop64.reshape(-1, D), o, R,
                                   nthreads=8).reshape(runs, NP)
    np.testing.assert_allclose(fprev, fit64, rtol=f_rtol, atol=1e-30)
    out = oracle.jde_generation(pop64, fit64, F0.astype(np.float64),
                                CR0.astype(np.float64), lo=LO, hi=HI, seed=3,
                                gen=g, kind=okind(kind), o=o, R=R, nthreads=8)
    ties = accepts = rejects = 0
    changed = 0
    for r in range(runs):
        for i in range(NP):
            Fp, CRp = out["Fp"][r, i], out["CRp"][r, i]
            changed += (Fp != F0[r, i]) or (CRp != CR0[r, i])
            d = oracle.draw_indices(3, r, g, i, NP, D)
            tol = trial_atol(pop64[r, d[0]], pop64[r, d[1]], pop64[r, d[2]],
                             Fp)
            fu, fx = out["ftrial"][r, i], fit64[r, i]
            band = (f_rtol * max(abs(fu), abs(fx)) +
                    rounding_band(okind(kind), out["trial"][r, i], o, R, tol))
            acc_g = not np.array_equal(pop_n[r, i], pop32[r, i]) or (
                fit_n[r, i] != fprev[r, i])
            # control values: the trial's (F', CR') exactly, kept iff accepted
            want = (Fp, CRp) if acc_g else (F0[r, i], CR0[r, i])
            assert (F1[r, i], CR1[r, i]) == (np.float32(want[0]),
                                             np.float32(want[1])), (r, i)
            if abs(fu - fx) <= band:
                ties += 1
                continue
            assert acc_g == bool(out["accept"][r, i]), (r, i, fu, fx)
            accepts += acc_g
            rejects += not acc_g
            if acc_g:
                err = np.abs(pop_n[r, i].astype(np.float64) - out["trial"][r, i])
                assert (err <= tol).all(), (r, i, err.max())
            else:
                np.testing.assert_array_equal(pop_n[r, i], pop32[r, i])
    GenCmp(runs * NP, ties, accepts, rejects).check(
        f"jDE {kind}/{prec} {runs}x{NP}x{D}",
        share=FP32_TIE_SHARE if prec == "fp32" else None)
    assert changed > 0  # some individuals drew new values


@pytest.mark.parametrize("kind,prec", [("sphere", "fp32"), ("rot_osc", "bf16")])
def test_jde_without_adaptation_equals_plain_de(kind, prec):
    kw = dict(runs=3, NP=64, D=50, F=0.5, CR=0.9, seed=2, kind=kind,
              gemm_prec=prec)
    a, _, _ = make_jde(jde=dict(F_lo=0.1, F_span=0.9, tau_F=0.0, tau_CR=0.0),
                       **kw)
    b, _, _ = make_de(**kw)
    a.generation(30)
    b.generation(30)
    np.testing.assert_array_equal(host(a.population()), host(b.population()))
    np.testing.assert_array_equal(host(a.fitness()), host(b.fitness()))
    F, CR = a.control()
    assert (F == np.float32(0.5)).all() and (CR == np.float32(0.9)).all()


def test_jde_checkpoint_restart_is_bit_exact():
    kw = dict(runs=2, NP=64, D=100, F=0.5, CR=0.9, seed=4, kind="rot_osc",
              gemm_prec="bf16")
    a, _, _ = make_jde(**kw)
    a.generation(40)
    b, _, _ = make_jde(**kw)
    b.generation(17)
    pop, (F, CR) = host(b.population()).copy(), b.control()
    c, _, _ = make_jde(**kw)
    c.load_population(pop, 17)
    c.set_control(F, CR)
    c.generation(23)
    np.testing.assert_array_equal(host(a.population()), host(c.population()))
    np.testing.assert_array_equal(host(a.fitness()), host(c.fitness()))
    Fa, CRa = a.control()
    Fc, CRc = c.control()
    np.testing.assert_array_equal(Fa, Fc)
    np.testing.assert_array_equal(CRa, CRc)


def test_jde_control_values_stay_in_range():
    de, _, _ = make_jde(runs=4, NP=100, D=10, seed=6)
    de.generation(200)
    F, CR = de.control()
    assert ((F == np.float32(0.5)) | ((F >= 0.1) & (F <= 1.0))).all()
    assert ((CR >= 0) & (CR <= 1)).all()
    # after 200 generations most individuals carry adapted values
    assert np.mean(F != np.float32(0.5)) > 0.5


@pytest.mark.parametrize("kind,prec,NP,D,G,checks", [
    ("sphere", "fp32", 64, 10, 300, (10, 100, 300)),
    ("rot_osc", "bf16", 48, 20, 200, (10, 100, 200)),
])
def test_jde_distribution_over_30_runs(kind, prec, NP, D, G, checks):
    runs = 30
    de, o, R = make_jde(runs=runs, NP=NP, D=D, F=0.5, CR=0.9, seed=1,
                        kind=kind, gemm_prec=prec)
    gpu, done = {}, 0
    for c in checks:
        de.generation(c - done)
        done = c
        gpu[c] = np.array(de.stats()[1])
    res = oracle.jde_run(runs=runs, NP=NP, D=D, F0=0.5, CR0=0.9, lo=LO, hi=HI,
                         seed=1, kind=okind(kind), o=o, R=R, G=G, nthreads=8)
    for c in checks:
        ok, pu, pks = de_stats.same_distribution(gpu[c],
                                                 res["best_trace"][:, c])
        assert ok, (c, pu, pks)
