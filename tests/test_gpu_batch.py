"""GPU parity of batched mixed-size runs (include/de_batch.h) against the
FP64 oracle, through the C ABI.

Each run of a batch is an independent DE/rand/1/bin run (Section 2) whose
draws use its batch index as the counter's run number, so the oracle checks
it on its own (oracle.generation with run0 = index, the run's F and CR).
Bars are those of the per-problem BF16 path: initial population bit-exact,
one generation from the GPU's FP32 population with f within the BF16 bar,
trial coordinates within one FP32 fused rounding, selection identical away
from near-ties.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2405_16551_amd import instances
from tests.gpu_helpers import (HI, LO, GenCmp, compare_generation, host,
                               make_de)

pytestmark = pytest.mark.gpu

OBJ = oracle.OBJ_ROT_OSC


def bf16_rtol(D: int) -> float:
    # same bar as the per-problem BF16 path (see test_gpu_parity.bf16_rtol)
    return 8 * 2.0 ** -8 / math.sqrt(D)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    yield


# NP from 4 to 130 (ragged tiles of 32 and 64), D from 1 to 257 (ragged 4-,
# 32- and 128-groups), F and CR per run, CR = 0 and 1 included
SPECS = [(4, 1, 0.5, 0.9), (37, 10, 0.45, 0.3), (64, 10, 0.8, 1.0),
         (130, 37, 0.6, 0.0), (33, 100, 0.5, 0.9), (96, 100, 0.7, 0.55),
         (65, 257, 0.55, 0.8), (128, 130, 0.9, 0.1)]


def make_batch(specs=SPECS, plan=None, graph_gens=16, seed=1, obj_seed=1):
    from paper_2405_16551_amd.de import DEBatch
    inst = instances.make_mixed_instances(specs, obj_seed)
    b = DEBatch(specs, inst, lo=LO, hi=HI, seed=seed, graph_gens=graph_gens,
                plan=plan)
    return b, inst


def all_variants(specs, v):
    return {D: v for D in {s[1] for s in specs}}


def test_batch_initial_population_bit_exact():
    b, inst = make_batch(plan=all_variants(SPECS, 0))
    for r, (NP, D, F, CR) in enumerate(SPECS):
        want = oracle.init_population(1, NP, D, LO, HI, 1, run0=r)[0]
        np.testing.assert_array_equal(host(b.population(r)),
                                      want.astype(np.float32))
        o, R = inst[D]
        f = host(b.fitness(r)).astype(np.float64)
        fo = oracle.objective_batch(OBJ, want.astype(np.float32).astype(
            np.float64), o, R, nthreads=8)
        np.testing.assert_allclose(f, fo, rtol=bf16_rtol(D), atol=0)
    b.close()


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_batch_generation_matches_oracle(variant):
    from paper_2405_16551_amd.de import DE_BATCH_WIDE
    b, inst = make_batch(plan=all_variants(SPECS, variant))
    assert set(b.plan()[0].values()) == {variant}
    b.generation(5)
    g = b.gen
    before = [(host(b.population(r)).copy(), host(b.fitness(r)).copy())
              for r in range(len(SPECS))]
    b.generation(1)
    tot = GenCmp(0, 0, 0, 0)
    for r, (NP, D, F, CR) in enumerate(SPECS):
        pop32, fprev = before[r]
        o, R = inst[D]
        res = compare_generation(
            host(b.population(r))[None], host(b.fitness(r))[None], pop32[None],
            fprev[None], F=F, CR=CR, seed=1, gen=g, kind=OBJ, o=o, R=R,
            f_rtol=bf16_rtol(D), run0=r)
        assert res.n == NP
        res.report(f"variant {variant} run {r} (NP {NP}, D {D}, CR {CR})")
        tot = GenCmp(tot.n + res.n, tot.ties + res.ties,
                     tot.accepts + res.accepts, tot.rejects + res.rejects)
    # near-ties (either decision valid) are rows whose two values differ by
    # less than the BF16 bar, which is wide at small D (3% at D = 1): at
    # most 10% of the batch's rows
    tot.check(f"variant {variant}, all runs")
    b.close()


@pytest.mark.parametrize("specs", [
    [(64, 200, 0.5, 0.9), (100, 200, 0.5, 0.9), (40, 600, 0.6, 0.8)],
    [(64, 100, 0.5, 0.9), (100, 100, 0.7, 0.3), (33, 60, 0.6, 1.0)],
    [(64, 1000, 0.5, 0.9), (68, 1000, 0.5, 0.9), (100, 500, 0.6, 0.8),
     (40, 700, 0.7, 0.3)],
], ids=["wide", "paired", "large"])
def test_wide_variant_equals_per_problem_handle(specs):
    # the wide variant runs the per-problem BF16 tile with the run's own
    # arguments: run r of a batch equals run r of a de.h handle bit for bit
    # (D = 200 pads to 256 in both: 512-thread tiles, two per CU; D = 600
    # pads to 640: 1024-thread tiles; one plan, two wide launches).  At
    # padded width 128 (D = 60, 100) the handle builds trials two rows per
    # wave instruction (paired rows) and the batch one row per instruction:
    # same draws, operations and order, so equal bit for bit as well.  At
    # padded widths 512, 768 and 1024 (D = 500, 700, 1000, the headline
    # width) with ragged last tiles: NP = 68 leaves a last tile of 4 rows,
    # so most waves of that tile have no row of their own.
    from paper_2405_16551_amd.de import DE_BATCH_WIDE
    b, inst = make_batch(specs, plan={D: DE_BATCH_WIDE for D in
                                      {s[1] for s in specs}},
                         graph_gens=4)
    single = []
    for r, (NP, D, F, CR) in enumerate(specs):
        de, _, _ = make_de(runs=r + 1, NP=NP, D=D, F=F, CR=CR, seed=1,
                           kind="rot_osc", gemm_prec="bf16")
        single.append(de)
    b.generation(30)
    for r, de in enumerate(single):
        de.generation(30)
        np.testing.assert_array_equal(host(b.population(r)),
                                      host(de.population())[r])
        np.testing.assert_array_equal(host(b.fitness(r)),
                                      host(de.fitness())[r])
        de.close()
    b.close()


@pytest.mark.parametrize("D", [200, 100])
def test_wide_tile_threads_do_not_change_results(D):
    # 300 runs: more wide tiles than compute units, so the batch runs
    # 512-thread tiles (two per CU); handles of at most 256 runs use
    # 1024-thread tiles, the handle of 300 runs 512-thread tiles.  Row sums
    # add column blocks in a fixed order, so the values agree bit for bit.
    # At D = 100 (padded width 128) every handle takes the paired-row tile
    # (1024 threads up to 256 runs, 512 beyond) against the batch's
    # one-row-per-instruction tile.
    specs = [(64, D, 0.5, 0.9)] * 300
    from paper_2405_16551_amd.de import DE_BATCH_WIDE
    b, inst = make_batch(specs, plan={D: DE_BATCH_WIDE}, graph_gens=4)
    b.generation(12)
    for r in (0, 200, 299):
        de, _, _ = make_de(runs=r + 1, NP=64, D=D, F=0.5, CR=0.9, seed=1,
                           kind="rot_osc", gemm_prec="bf16")
        de.generation(12)
        np.testing.assert_array_equal(host(b.population(r)),
                                      host(de.population())[r])
        np.testing.assert_array_equal(host(b.fitness(r)),
                                      host(de.fitness())[r])
        de.close()
    b.close()


def test_zero_generations_change_nothing():
    b, _ = make_batch(graph_gens=4)
    b.generation(3)
    before = [host(b.population(r)).copy() for r in range(len(SPECS))]
    b.generation(0)
    assert b.gen == 3
    for r in range(len(SPECS)):
        np.testing.assert_array_equal(host(b.population(r)), before[r])
    b.close()


def test_graph_replays_equal_direct_launches():
    plan = all_variants(SPECS, 0)
    plan[257] = 2
    a, _ = make_batch(plan=plan, graph_gens=4)
    c, _ = make_batch(plan=plan, graph_gens=1)
    # graph replays with host reads and direct launches in between
    for step in (4, 1, 8, 3, 4):
        a.generation(step)
        c.generation(step)
        ra, rc = a.read(), c.read()
        assert ra == rc
    assert a.gen == c.gen == 20
    for r in range(len(SPECS)):
        np.testing.assert_array_equal(host(a.population(r)),
                                      host(c.population(r)))
        np.testing.assert_array_equal(host(a.fitness(r)), host(c.fitness(r)))
    a.close()
    c.close()


def test_batch_statistics_and_invariants():
    b, _ = make_batch()
    prev = b.read()
    for _ in range(6):
        b.generation(5)
        st = b.read()
        for r, (NP, D, F, CR) in enumerate(SPECS):
            fit = host(b.fitness(r))
            assert st["best_f"][r] == float(fit.min())
            assert st["best_idx"][r] == int(np.argmin(fit))
            assert st["best_f"][r] <= prev["best_f"][r]
            assert 0 <= st["accepted"][r] - prev["accepted"][r] <= 5 * NP
            x = host(b.population(r))
            assert x.min() >= LO and x.max() <= HI
        prev = st
    b.close()


def test_autotuner_plan():
    from paper_2405_16551_amd.de import DE_BATCH_NVARIANTS
    b, _ = make_batch()
    plan, us = b.plan()
    for D, v in plan.items():
        times = us[D]
        assert 0 <= v < DE_BATCH_NVARIANTS
        timed = [t for t in times if t >= 0]
        assert timed and times[v] == min(timed)
    b.close()


def test_mixed_batch_full_size_sampled():
    # the benchmark's batch: 512 runs, NP in {32..1024}, D in {10..500},
    # F, CR per run, autotuned plan; every dimension's runs checked against
    # the oracle on sampled rows after a few generations
    specs = instances.make_mixed_specs(512, seed=1)
    b, inst = make_batch(specs, graph_gens=8)
    b.generation(9)
    g = b.gen
    rng = np.random.default_rng(5)
    picked = []
    for D in sorted({s[1] for s in specs}):
        rs = [r for r, s in enumerate(specs) if s[1] == D]
        picked += list(rng.choice(rs, size=2, replace=False))
    before = {r: (host(b.population(r)).copy(), host(b.fitness(r)).copy())
              for r in picked}
    b.generation(1)
    tot = GenCmp(0, 0, 0, 0)
    for r in picked:
        NP, D, F, CR = specs[r]
        pop32, fprev = before[r]
        o, R = inst[D]
        rows = [(0, int(i)) for i in rng.choice(NP, size=min(NP, 24),
                                                 replace=False)]
        res = compare_generation(host(b.population(r))[None],
                                 host(b.fitness(r))[None], pop32[None],
                                 fprev[None], F=F, CR=CR, seed=1, gen=g,
                                 kind=OBJ, o=o, R=R, f_rtol=bf16_rtol(D),
                                 rows=rows, run0=int(r))
        res.report(f"run {r} (NP {NP}, D {D}, CR {CR:.3f})")
        tot = GenCmp(tot.n + res.n, tot.ties + res.ties,
                     tot.accepts + res.accepts, tot.rejects + res.rejects)
    # at most 10% of the sampled rows may be near-ties, and decisions both
    # ways must have been checked
    tot.check("mixed batch, sampled rows")
    assert tot.accepts > 0 and tot.rejects > 0
    st = b.read()
    assert all(h == -1 for h in st["hit_gen"])
    b.close()
