"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (from the method's definition, Section 2 of arXiv 2405.16551, and the
arithmetic of each path):
  * integer work (donor indices, j_rand, crossover decisions) and the initial
    population: bit-exact;
  * one generation from a shared FP32 population: trial coordinates within
    one rounding of the FP32 fused multiply-add, fitness within 1e-5
    relative (FP32 paths), selection identical except near-ties below that
    tolerance;
  * BF16 rotation GEMM: the per-result error against FP64 is measured and
    bounded (see test_bf16_error_is_stated);
  * whole runs: best-fitness distributions over 30 runs match the oracle's
    under the paper's rank score (Mann-Whitney U) and KS, floored at the
    1e-8 success threshold of Section 7.3.4.
"""
import math
import os

import numpy as np
import pytest

import oracle
from tests import de_stats
from tests.gpu_helpers import (FP32_RTOL, FP32_TIE_SHARE, HI, LO,
                               compare_generation, host, make_de, okind)

pytestmark = pytest.mark.gpu



def bf16_rtol(D: int) -> float:
    """Relative tolerance of f with the BF16 rotation product.  Rounding R
    and y to BF16 (nearest-even, relative error <= 2^-9 per operand) moves
    sum z_i^2 by a sum of D^2 independent terms; its relative standard
    deviation works out near 2^-8 / sqrt(D) (R part 2^-8/sqrt(3D), y part
    2^-8 sqrt(0.6/D) for uniform y); the bar is eight of those."""
    return 8 * 2.0 ** -8 / math.sqrt(D)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    import paper_2405_16551_amd.de as de  # noqa: F401  (fails if not built)
    yield


# ---------------------------------------------------------------------------
# Initialisation and draws: bit-exact.

@pytest.mark.parametrize("runs,NP,D,ldx", [(1, 64, 10, None), (3, 37, 13, 20),
                                           (2, 5, 1, None), (2, 130, 1000, None)])
def test_init_population_bit_exact(runs, NP, D, ldx):
    de, o, R = make_de(runs=runs, NP=NP, D=D, seed=11, ldx=ldx)
    got = host(de.population(0))
    want = oracle.init_population(runs, NP, D, LO, HI, 11).astype(np.float32)
    np.testing.assert_array_equal(got, want)
    f = host(de.fitness(0))
    fo = oracle.objective_batch(oracle.OBJ_SPHERE, got.astype(np.float64).reshape(-1, D), o)
    np.testing.assert_allclose(f.ravel(), fo, rtol=FP32_RTOL)


@pytest.mark.parametrize("runs,NP,D,CR", [(2, 4, 3, 0.5), (3, 50, 37, 0.9),
                                          (1, 1024, 1000, 0.3), (2, 33, 64, 0.0),
                                          (1, 9, 70, 1.0)])
def test_debug_draws_bit_exact(runs, NP, D, CR):
    de, o, R = make_de(runs=runs, NP=NP, D=D, CR=CR, seed=7)
    nw = (D + 31) // 32
    for gen in (0, 1, 12345):
        idx, mask = de.debug_draws(gen)
        idx, mask = host(idx), host(mask).view(np.uint32)
        rows = [(r, i) for r in range(runs) for i in range(NP)]
        if len(rows) > 200:
            rows = [rows[k] for k in np.random.default_rng(gen).choice(
                len(rows), 200, replace=False)]
        for r, i in rows:
            want = oracle.draw_indices(7, r, gen, i, NP, D)
            assert tuple(idx[r, i]) == want
            bits = np.zeros(nw, dtype=np.uint32)
            for j in range(D):
                if oracle.take_mutant(7, r, gen, i, j, want[3], CR):
                    bits[j // 32] |= np.uint32(1 << (j % 32))
            np.testing.assert_array_equal(mask[r, i], bits)


# ---------------------------------------------------------------------------
# One generation from a shared FP32 population.

@pytest.mark.parametrize("kind,prec,runs,NP,D,CR", [
    ("sphere", "fp32", 3, 100, 37, 0.9),
    ("sphere", "fp32", 1, 64, 10, 0.9),
    ("sphere", "fp32", 2, 70, 1000, 0.9),
    ("sphere", "fp32", 2, 4, 1, 0.5),
    # one-wave-per-row form: rows of 257..512, 513..1024 (last chunk
    # partial), 1025..2048 and 2049..4096 coordinates; row counts that leave
    # workgroups partly empty; CR = 1 takes every coordinate
    ("sphere", "fp32", 3, 45, 300, 0.9),
    ("sphere", "fp32", 1, 33, 513, 0.7),
    ("sphere", "fp32", 1, 22, 1500, 1.0),
    ("sphere", "fp32", 1, 9, 3001, 0.3),
    ("rot_osc", "fp32", 2, 70, 100, 0.9),
    ("rot_osc", "fp32", 1, 40, 13, 0.3),
    ("rot_osc", "fp32", 1, 65, 250, 0.9),
    # paired rows (padded width <= 128): a last tile of 24 rows leaves each
    # wave three (one pair without its second row); D = 128 fills all 32
    # quads of a row
    ("rot_osc", "fp32", 2, 88, 100, 0.9),
    ("rot_osc", "fp32", 1, 50, 128, 0.5),
    # the smallest rotated problem: NP = 4, D = 1 (z = +-(x - o))
    ("rot_osc", "fp32", 2, 4, 1, 0.5),
])
def test_one_generation_matches_oracle(kind, prec, runs, NP, D, CR):
    de, o, R = make_de(runs=runs, NP=NP, D=D, CR=CR, seed=5, kind=kind,
                       gemm_prec=prec)
    # a few generations in, so that selection is not trivial
    de.generation(3)
    g = de.gen
    pop32 = host(de.population()).copy()
    fit_prev = host(de.fitness()).copy()
    de.generation(1)
    res = compare_generation(host(de.population()), host(de.fitness()),
                             pop32, fit_prev, F=0.5, CR=CR, seed=5, gen=g,
                             kind=okind(kind), o=o, R=R, f_rtol=FP32_RTOL)
    assert res.n == runs * NP
    res.check(f"{kind}/{prec} {runs}x{NP}x{D} CR={CR}", share=FP32_TIE_SHARE)


# (2, 70, 100): two ragged tiles per run; the smallest problems, NP = 4
# (three donors and the target) and D = 1 or 2 (one quad of a row, padded
# to 128 columns of which one or two are live); 65 rows: a last tile of one
# row
@pytest.mark.parametrize("runs,NP,D", [(2, 70, 100), (2, 4, 1), (3, 5, 2),
                                       (1, 65, 33)])
def test_one_generation_bf16_gemm(runs, NP, D):
    de, o, R = make_de(runs=runs, NP=NP, D=D, seed=5, kind="rot_osc",
                       gemm_prec="bf16")
    de.generation(2)
    g = de.gen
    pop32 = host(de.population()).copy()
    fit_prev = host(de.fitness()).copy()
    de.generation(1)
    res = compare_generation(host(de.population()), host(de.fitness()),
                             pop32, fit_prev, F=0.5, CR=0.9, seed=5, gen=g,
                             kind=oracle.OBJ_ROT_OSC, o=o, R=R,
                             f_rtol=bf16_rtol(D))
    assert res.n == runs * NP
    res.check(f"rot_osc/bf16 {runs}x{NP}x{D}")


@pytest.mark.parametrize("D", [256, 100])
def test_one_generation_bf16_two_tiles_per_cu(D):
    # more 64-row tiles (258) than compute units: the BF16 tile runs with
    # 512 threads, two workgroups per CU; at D = 100 (padded width 128) in
    # the paired-row form (trials built two rows per wave instruction)
    runs, NP = 2, 8256
    de, o, R = make_de(runs=runs, NP=NP, D=D, seed=5, kind="rot_osc",
                       gemm_prec="bf16")
    de.generation(2)
    g = de.gen
    pop32 = host(de.population()).copy()
    fit_prev = host(de.fitness()).copy()
    de.generation(1)
    res = compare_generation(host(de.population()), host(de.fitness()),
                             pop32, fit_prev, F=0.5, CR=0.9, seed=5, gen=g,
                             kind=oracle.OBJ_ROT_OSC, o=o, R=R,
                             f_rtol=bf16_rtol(D))
    assert res.n == runs * NP
    res.check(f"rot_osc/bf16 {runs}x{NP}x{D} (512-thread tiles)")


@pytest.mark.parametrize("kind,prec,runs,NP,D", [
    # the largest supported widths: the BF16 tile's LDS is exactly 160 KB at
    # padded width 1152; separable rows of 4096 fill the one-wave-per-row
    # form's last chunk exactly
    ("rot_osc", "bf16", 2, 70, 1152),
    ("rot_osc", "fp32", 1, 40, 1152),
    ("sphere", "fp32", 1, 20, 4096),
])
def test_one_generation_at_the_largest_supported_width(kind, prec, runs, NP,
                                                       D):
    de, o, R = make_de(runs=runs, NP=NP, D=D, seed=5, kind=kind,
                       gemm_prec=prec)
    de.generation(2)
    g = de.gen
    pop32 = host(de.population()).copy()
    fit_prev = host(de.fitness()).copy()
    de.generation(1)
    rtol = bf16_rtol(D) if prec == "bf16" else FP32_RTOL
    res = compare_generation(host(de.population()), host(de.fitness()),
                             pop32, fit_prev, F=0.5, CR=0.9, seed=5, gen=g,
                             kind=okind(kind), o=o, R=R, f_rtol=rtol)
    assert res.n == runs * NP
    res.check(f"{kind}/{prec} {runs}x{NP}x{D}")


# ---------------------------------------------------------------------------
# Objective evaluation through the generation kernels' arithmetic.

@pytest.mark.parametrize("kind,prec,D,n,rtol", [
    ("sphere", "fp32", 10, 130, FP32_RTOL),
    ("sphere", "fp32", 1000, 70, FP32_RTOL),
    ("rot_osc", "fp32", 100, 130, FP32_RTOL),
    ("rot_osc", "fp32", 1000, 70, FP32_RTOL),
    ("rot_osc", "bf16", 100, 130, bf16_rtol(100)),
    ("rot_osc", "bf16", 1000, 70, bf16_rtol(1000)),
    ("rot_osc", "bf16", 7, 3, bf16_rtol(7)),
])
def test_eval_matches_oracle(kind, prec, D, n, rtol):
    de, o, R = make_de(runs=1, NP=8, D=D, kind=kind, gemm_prec=prec)
    rng = np.random.default_rng(D + n)
    X = rng.uniform(LO, HI, (n, D)).astype(np.float32)
    X[0] = o  # the optimum: f = 0 exactly
    X[1] = o + np.float32(1e-3)  # near the optimum: small, still relative
    f = host(de.eval(X)).astype(np.float64)
    fo = oracle.objective_batch(okind(kind), X.astype(np.float64), o, R)
    assert f[0] == 0.0
    np.testing.assert_allclose(f, fo, rtol=rtol, atol=0)


def test_bf16_error_is_stated():
    # per-result relative error of the BF16 rotation GEMM against FP64, at
    # the metric's dimension D = 1000: typical 2^-8 / sqrt(D) ~ 1.2e-4
    de, o, R = make_de(runs=1, NP=8, D=1000, kind="rot_osc", gemm_prec="bf16")
    rng = np.random.default_rng(3)
    X = rng.uniform(LO, HI, (256, 1000)).astype(np.float32)
    scale = np.logspace(-4, 0, 256)[:, None].astype(np.float32)
    X = (o + (X - o) * scale).astype(np.float32)  # from near-optimum to far
    f = host(de.eval(X)).astype(np.float64)
    fo = oracle.objective_batch(oracle.OBJ_ROT_OSC, X.astype(np.float64), o, R,
                                nthreads=8)
    rel = np.abs(f - fo) / fo
    print(f"BF16 GEMM f rel. error vs FP64: median {np.median(rel):.2e}, "
          f"p99 {np.quantile(rel, 0.99):.2e}, max {rel.max():.2e}")
    assert np.median(rel) < 2.0 ** -8 / math.sqrt(1000)
    assert rel.max() < bf16_rtol(1000)


# ---------------------------------------------------------------------------
# Multi-generation behaviour.

def test_teacher_forced_trajectory_sphere():
    # generations 250 and 399 lie past the 1e-8 hit (generation ~280): there
    # the FP32 rounding of a trial's coordinates (~1e-5 at |x| ~ 80) moves f
    # by more than f itself, so selection is a near-tie for most rows and
    # only the rows' contents are checked; earlier generations are decided
    runs, NP, D, G = 2, 64, 10, 400
    de, o, R = make_de(runs=runs, NP=NP, D=D, seed=1)
    checkpoints = {0, 1, 10, 100, 250, 399}
    for g in range(G):
        if g in checkpoints:
            pop32 = host(de.population()).copy()
            fit_prev = host(de.fitness()).copy()
            de.generation(1)
            res = compare_generation(host(de.population()), host(de.fitness()),
                                     pop32, fit_prev, F=0.5, CR=0.9, seed=1,
                                     gen=g, kind=oracle.OBJ_SPHERE, o=o,
                                     R=None, f_rtol=FP32_RTOL)
            if g <= 100:
                res.check(f"sphere trajectory gen {g}", share=FP32_TIE_SHARE)
            else:
                res.report(f"sphere trajectory gen {g} (past the optimum)")
        else:
            de.generation(1)


def test_invariants_every_generation():
    runs, NP, D = 4, 32, 20
    de, o, R = make_de(runs=runs, NP=NP, D=D, seed=3, kind="rot_osc",
                       gemm_prec="bf16", CR=0.5)
    prev_acc, prev_best = de.stats()
    for _ in range(150):
        de.generation(1)
        pop = host(de.population())
        assert pop.min() >= LO and pop.max() <= HI
        acc, best = de.stats()
        for r in range(runs):
            assert 0 <= acc[r] - prev_acc[r] <= NP
            assert best[r] <= prev_best[r]
            assert best[r] == host(de.fitness())[r].min()
        prev_acc, prev_best = acc, best


def test_generation_split_does_not_matter():
    a, _, _ = make_de(runs=2, NP=40, D=30, seed=9, kind="rot_osc")
    b, _, _ = make_de(runs=2, NP=40, D=30, seed=9, kind="rot_osc")
    a.generation(25)
    for _ in range(25):
        b.generation(1)
    np.testing.assert_array_equal(host(a.population()), host(b.population()))
    np.testing.assert_array_equal(host(a.fitness()), host(b.fitness()))


@pytest.mark.parametrize("kind,prec", [("sphere", "fp32"), ("rot_osc", "bf16")])
def test_checkpoint_restart_is_bit_exact(kind, prec):
    a, _, _ = make_de(runs=2, NP=48, D=40, seed=4, kind=kind, gemm_prec=prec)
    a.generation(60)
    b, _, _ = make_de(runs=2, NP=48, D=40, seed=4, kind=kind, gemm_prec=prec)
    b.generation(23)
    snap = host(b.population()).copy()
    c, _, _ = make_de(runs=2, NP=48, D=40, seed=4, kind=kind, gemm_prec=prec)
    c.load_population(snap, 23)
    c.generation(37)
    np.testing.assert_array_equal(host(a.population()), host(c.population()))
    np.testing.assert_array_equal(host(a.fitness()), host(c.fitness()))


def test_empty_calls_change_nothing():
    # no generations, an evolve without budget, an evaluation of no rows:
    # status OK and nothing moves
    de, o, R = make_de(runs=2, NP=40, D=30, seed=3, kind="rot_osc",
                       gemm_prec="bf16")
    de.generation(2)
    pop, fit = host(de.population()).copy(), host(de.fitness()).copy()
    de.generation(0)
    gens, hits = de.evolve(0, target=-1.0)  # a target no run reaches
    f = de.eval(np.zeros((0, 30), np.float32))
    assert de.gen == 2 and gens == 0 and hits == [-1, -1]
    assert host(f).shape == (0,)
    np.testing.assert_array_equal(host(de.population()), pop)
    np.testing.assert_array_equal(host(de.fitness()), fit)


def test_evolve_stops_at_target_and_records_first_hit():
    runs, NP, D = 3, 64, 10
    de, o, R = make_de(runs=runs, NP=NP, D=D, seed=1)
    ref, _, _ = make_de(runs=runs, NP=NP, D=D, seed=1)
    gens_done, hits = de.evolve(2000, target=1e-8, check_every=64)
    assert all(h > 0 for h in hits)
    # the chunk after the one in which the last run hit may have run too
    assert max(hits) <= gens_done < max(hits) + 2 * 64
    assert gens_done % 64 == 0
    # replay generation by generation: first generation with best <= 1e-8
    first = [-1] * runs
    for g in range(1, max(hits) + 1):
        ref.generation(1)
        _, best = ref.stats()
        for r in range(runs):
            if first[r] < 0 and best[r] <= 1e-8:
                first[r] = g
    assert first == hits
    x, f, idx = de.best(0)
    assert f <= 1e-8
    np.testing.assert_allclose(x, o, atol=1e-3)


def test_best_reports_lowest_value_lowest_index():
    de, o, R = make_de(runs=2, NP=30, D=5, seed=2)
    de.generation(40)
    fit = host(de.fitness())
    for r in range(2):
        x, f, idx = de.best(r)
        assert idx == int(np.argmin(fit[r]))
        assert np.float32(f) == fit[r].min()
        np.testing.assert_array_equal(np.array(x, np.float32),
                                      host(de.population())[r, idx])


@pytest.mark.parametrize("kind,prec,runs,NP,D,G", [
    ("sphere", "fp32", 3, 40, 37, 30),
    ("rot_osc", "fp32", 2, 64, 100, 20),
    ("rot_osc", "bf16", 2, 64, 100, 20),
    ("rot_osc", "bf16", 1, 128, 1000, 3),
])
def test_best_f64_matches_oracle(kind, prec, runs, NP, D, G):
    # the FP64 re-evaluation of each run's best row equals the oracle's FP64
    # objective of that FP32 row (up to summation order), and it bounds the
    # error the generation step's own arithmetic made on that row
    de, o, R = make_de(runs=runs, NP=NP, D=D, kind=kind, gemm_prec=prec)
    de.generation(G)
    pop = host(de.population()).astype(np.float64)
    fit = host(de.fitness()).astype(np.float64)
    f64, idx = de.best_f64()
    for r in range(runs):
        _, fb, ib = de.best(r)
        assert idx[r] == ib
        fo = oracle.objective(okind(kind), pop[r, idx[r]], o, R)
        assert abs(f64[r] - fo) <= 1e-12 * fo
        rtol = bf16_rtol(D) if prec == "bf16" else FP32_RTOL
        assert abs(fit[r, idx[r]] - f64[r]) <= rtol * f64[r]
        print(f"{kind}/{prec} D={D} run {r}: f32-path {fit[r, idx[r]]:.9e} "
              f"fp64 {f64[r]:.9e} rel {abs(fit[r, idx[r]] - f64[r]) / f64[r]:.2e}")


# ---------------------------------------------------------------------------
# Whole runs: distributions over 30 runs against the oracle.

@pytest.mark.parametrize("kind,prec,NP,D,G,checks", [
    ("sphere", "fp32", 64, 10, 400, (10, 100, 200, 400)),
    ("rot_osc", "fp32", 48, 20, 300, (10, 100, 300)),
    ("rot_osc", "bf16", 48, 20, 300, (10, 100, 300)),
])
def test_best_distribution_over_30_runs(kind, prec, NP, D, G, checks):
    runs = 30
    de, o, R = make_de(runs=runs, NP=NP, D=D, seed=1, kind=kind,
                       gemm_prec=prec)
    gpu = {}
    done = 0
    for c in checks:
        de.generation(c - done)
        done = c
        gpu[c] = np.array(de.stats()[1])
    res = oracle.run(runs=runs, NP=NP, D=D, F=0.5, CR=0.9, lo=LO, hi=HI,
                     seed=1, kind=okind(kind), o=o, R=R, G=G, nthreads=8)
    for c in checks:
        ok, pu, pks = de_stats.same_distribution(gpu[c],
                                                 res["best_trace"][:, c])
        assert ok, (c, pu, pks, np.median(gpu[c]),
                    np.median(res["best_trace"][:, c]))


def test_c2_distribution_full_size():
    # 64 runs x NP 256, D 100, rotated, FP32 product, 3000 generations: the
    # GPU's best over the runs at every checkpoint against the FP64
    # oracle's stored distribution (tests/golden/make_c2_reference.py)
    import json
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "oracle_c2_distribution.json")) as f:
        gold = json.load(f)
    c = gold["config"]
    de, o, R = make_de(runs=c["runs"], NP=c["NP"], D=c["D"], F=c["F"],
                       CR=c["CR"], seed=c["seed"], kind=c["kind"],
                       gemm_prec="fp32")
    done = 0
    for g in gold["checkpoints"]:
        de.generation(g - done)
        done = g
        gpu = np.array(de.stats()[1])
        ok, pu, pks = de_stats.same_distribution(gpu, gold["best"][str(g)])
        print(f"c2 gen {g}: gpu median {np.median(gpu):.4e} oracle median "
              f"{np.median(gold['best'][str(g)]):.4e} p_U {pu:.3f} p_KS {pks:.3f}")
        assert ok, (g, pu, pks)


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_c3_distribution_full_size(prec):
    # 16 runs x NP 1024, D 1000, rotated, 2000 generations (the headline
    # workload as configured): the GPU's best over the runs at every
    # checkpoint against the FP64 oracle's stored distribution
    # (tests/golden/make_c3_reference.py), with the BF16 and the FP32
    # rotation product
    import json
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "oracle_c3_distribution.json")) as f:
        gold = json.load(f)
    c = gold["config"]
    de, o, R = make_de(runs=c["runs"], NP=c["NP"], D=c["D"], F=c["F"],
                       CR=c["CR"], seed=c["seed"], kind=c["kind"],
                       gemm_prec=prec)
    done = 0
    for g in gold["checkpoints"]:
        de.generation(g - done)
        done = g
        gpu = np.array(de.stats()[1])
        ok, pu, pks = de_stats.same_distribution(gpu, gold["best"][str(g)])
        print(f"c3 {prec} gen {g}: gpu median {np.median(gpu):.4e} oracle "
              f"median {np.median(gold['best'][str(g)]):.4e} p_U {pu:.3f} "
              f"p_KS {pks:.3f}", flush=True)
        assert ok, (g, pu, pks)
    acc, _ = de.stats()
    rate = sum(acc) / (c["runs"] * c["NP"] * c["G"])
    orate = sum(gold["accepted"]) / (c["runs"] * c["NP"] * c["G"])
    print(f"c3 {prec} acceptance over the run: gpu {rate:.4f} oracle "
          f"{orate:.4f}")
    assert abs(rate - orate) <= 0.1 * orate


# ---------------------------------------------------------------------------
# Full-size workloads (16 runs x NP 1024 x D 1000, the benchmark's launch
# configuration): every row of a generation against the oracle, early (the
# step from generation 1) and late (teacher-forced: the oracle steps the
# GPU's own population of generation 1500, which the oracle computes in
# about a second on 16 host threads).

@pytest.mark.parametrize("kind,prec,at", [
    ("sphere", "fp32", 1), ("sphere", "fp32", 1500),
    ("rot_osc", "bf16", 1), ("rot_osc", "bf16", 1500),
    ("rot_osc", "fp32", 1), ("rot_osc", "fp32", 1500),
])
def test_full_size_every_row(kind, prec, at):
    runs, NP, D = 16, 1024, 1000
    de, o, R = make_de(runs=runs, NP=NP, D=D, seed=1, kind=kind,
                       gemm_prec=prec)
    de.generation(at)
    g = de.gen
    pop32 = host(de.population()).copy()
    fit_prev = host(de.fitness()).copy()
    de.generation(1)
    rtol = bf16_rtol(D) if prec == "bf16" else FP32_RTOL
    res = compare_generation(host(de.population()), host(de.fitness()),
                             pop32, fit_prev, F=0.5, CR=0.9, seed=1, gen=g,
                             kind=okind(kind), o=o, R=R, f_rtol=rtol)
    assert res.n == runs * NP
    assert res.accepts > 0 and res.rejects > 0
    res.check(f"{kind}/{prec} 16x1024x1000 gen {g}",
              share=FP32_TIE_SHARE if prec == "fp32" else None)


# ---------------------------------------------------------------------------
# Bound repair: F = 2, CR = 1 sends many mutant coordinates out of the box.
# The box [-10, 10] lies inside the shift's range [-80, 80], so most of the
# optimum's coordinates are outside it: trials pushed onto the bounds are
# the good ones, and accepted trials carry many clamped coordinates.

@pytest.mark.parametrize("kind,prec,D", [
    ("sphere", "fp32", 37), ("sphere", "fp32", 600),
    ("rot_osc", "fp32", 100), ("rot_osc", "bf16", 100),
    ("rot_osc", "bf16", 300),
])
def test_clamped_coordinates_are_the_bounds(kind, prec, D):
    # every trial coordinate is the mutant x_r1 + 2 (x_r2 - x_r3); where its
    # exact value lies outside [lo, hi] by more than one FP32 rounding, the
    # GPU's accepted trial must hold lo or hi exactly
    runs, NP, F, CR, lo, hi = 2, 128, 2.0, 1.0, -10.0, 10.0
    de, o, R = make_de(runs=runs, NP=NP, D=D, F=F, CR=CR, seed=8, kind=kind,
                       gemm_prec=prec, lo=lo, hi=hi)
    rtol = bf16_rtol(D) if prec == "bf16" else FP32_RTOL
    clamped = 0
    for _ in range(3):
        g = de.gen
        pop32 = host(de.population()).copy()
        fit_prev = host(de.fitness()).copy()
        de.generation(1)
        pop_n, fit_n = host(de.population()), host(de.fitness())
        res = compare_generation(pop_n, fit_n, pop32, fit_prev, F=F, CR=CR,
                                 seed=8, gen=g, kind=okind(kind), o=o, R=R,
                                 f_rtol=rtol, lo=lo, hi=hi)
        res.check(f"{kind}/{prec} D={D} F=2 CR=1 gen {g}",
                  share=FP32_TIE_SHARE if prec == "fp32" else None)
        pop64 = pop32.astype(np.float64)
        for r in range(runs):
            for i in range(NP):
                if np.array_equal(pop_n[r, i], pop32[r, i]):
                    continue  # kept
                r1, r2, r3, _ = oracle.draw_indices(8, r, g, i, NP, D)
                m = pop64[r, r1] + F * (pop64[r, r2] - pop64[r, r3])
                tol = 2.0 ** -22 * (np.abs(pop64[r, r1]) + F * (
                    np.abs(pop64[r, r2]) + np.abs(pop64[r, r3])))
                below, above = m < lo - tol, m > hi + tol
                assert (pop_n[r, i][below] == np.float32(lo)).all(), (r, i)
                assert (pop_n[r, i][above] == np.float32(hi)).all(), (r, i)
                clamped += int(below.sum() + above.sum())
    print(f"{kind}/{prec} D={D}: {clamped} clamped coordinates checked")
    assert clamped > 0


# ---------------------------------------------------------------------------
# Error paths through the ABI on a live device.

def test_destroyed_handle_and_bad_calls():
    import paper_2405_16551_amd.de as d
    de, o, R = make_de(runs=1, NP=8, D=4)
    h = de.handle
    with pytest.raises(d.DEError) as e:
        d.de_generation(h, -1, de._s())
    assert e.value.status == d.DE_E_INVAL
    with pytest.raises(d.DEError) as e:
        d.de_best(h, 1, de._s(), 4)
    assert e.value.status == d.DE_E_INVAL
    de.close()
    with pytest.raises(d.DEError) as e:
        d.de_generation(h, 1, 0)
    assert e.value.status == d.DE_E_STATE


@pytest.mark.parametrize("runs,NP,D,ldx", [(1, 64, 10, None), (3, 37, 13, 20),
                                           (30, 64, 10, None), (2, 60, 100, None),
                                           (5, 4, 1, None), (2, 30, 256, None)])
def test_resident_separable_equals_per_generation(runs, NP, D, ldx):
    # calls of several generations on small separable problems keep each
    # run's population in LDS; single generations use the per-generation
    # kernel: both must agree bit for bit, statistics included
    a, _, _ = make_de(runs=runs, NP=NP, D=D, seed=3, ldx=ldx)
    b, _, _ = make_de(runs=runs, NP=NP, D=D, seed=3, ldx=ldx)
    a.generation(37)
    a.generation(2)
    for _ in range(39):
        b.generation(1)
    np.testing.assert_array_equal(host(a.population()), host(b.population()))
    np.testing.assert_array_equal(host(a.fitness()), host(b.fitness()))
    assert a.stats() == b.stats()
    # a per-generation step after a resident call rewrites rows correctly
    a.generation(1)
    b.generation(1)
    np.testing.assert_array_equal(host(a.population()), host(b.population()))
    a.close()
    b.close()
