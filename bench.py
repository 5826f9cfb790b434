"""Throughput of the DE/rand/1/bin generation step on one MI355X.

Workload (default): 16 independent runs, NP = 1024, D = 1000, rotated
oscillating objective z = R (x - o), f = sum z^2 + sin^2(3z), rotation
product in BF16 on MFMA with FP32 accumulation, F = 0.5, CR = 0.9, search
box [-100, 100]; synthetic instance (seeded shift and Haar rotation).  One
step = one synchronous generation of all 16 x 1024 trials (draws, mutation,
crossover, fitness, selection, write of the next generation).

Prints one JSON line.  value = trial evaluations per second over the timed
steps (inputs resident in HBM; the timed steps are five back-to-back
library calls of about K/5 generations each).  Also reported: generations
per second, the median and spread of the five segments, the handle's
initialisation time, the roofline position of the generation kernel (HIP
events around the K launches, algorithmic FLOPs 2 D^2 per trial), a
separable companion workload
(shifted sphere, same sizes; HBM roofline), the same rotated step with the
product in FP32, wall time to the 1e-8 target
on the small sphere workload (Section 7.3.4 early stopping), wall time to
the FP64 oracle's median final best on the rotated D = 100 workload (64
runs, with the oracle's own time to it extrapolated), the headline
workload as configured (2000 generations in BF16 and FP32: per-step time
and acceptance over the whole run, median best next to the FP64 oracle's,
wall time to the oracle's median final best), a batch of 512
independent runs of mixed NP, D, F and CR advanced by graph replays, the
measured device-copy and library BF16 GEMM ceilings, and the FP64 CPU
oracle timed on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 MFMA
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 (matrix and vector)

WORKLOADS = {
    "rot1000_bf16": dict(runs=16, NP=1024, D=1000, kind="rot_osc",
                         gemm_prec="bf16"),
    "rot1000_fp32": dict(runs=16, NP=1024, D=1000, kind="rot_osc",
                         gemm_prec="fp32"),
    "sphere1000": dict(runs=16, NP=1024, D=1000, kind="sphere",
                       gemm_prec="fp32"),
    "sphere1000_r64": dict(runs=64, NP=1024, D=1000, kind="sphere",
                           gemm_prec="fp32"),
    "rot100_r64": dict(runs=64, NP=256, D=100, kind="rot_osc",
                       gemm_prec="fp32"),
    "sphere10": dict(runs=1, NP=64, D=10, kind="sphere", gemm_prec="fp32"),
    # jDE (per-individual F, CR; Brest et al. constants), same sizes
    "rot1000_bf16_jde": dict(runs=16, NP=1024, D=1000, kind="rot_osc",
                             gemm_prec="bf16", jde=True),
    "sphere1000_jde": dict(runs=16, NP=1024, D=1000, kind="sphere",
                           gemm_prec="fp32", jde=True),
}


def describe(name):
    w = WORKLOADS[name]
    obj = ("shifted sphere" if w["kind"] == "sphere" else
           f"rotated oscillating, {w['gemm_prec']} rotation product")
    if w.get("jde"):
        return (f"jDE (DE/rand/1/bin, per-individual F and CR adapted as in "
                f"Brest et al. 2006), {w['runs']} runs x NP={w['NP']}, "
                f"D={w['D']}, {obj}, F=0.5, CR=0.9 at the start")
    return (f"DE/rand/1/bin, {w['runs']} runs x NP={w['NP']}, D={w['D']}, "
            f"{obj}, F=0.5, CR=0.9")


def algorithmic(w, trials, accept_rate):
    """Algorithmic work of one generation launch.  Rotated objective: FLOPs
    of the rotation product, 2 D^2 per trial.  Separable objective: HBM bytes
    every implementation of the step must move, per trial 4 D (read the
    target row) + 8 (read and write its fitness) + 4 D times the acceptance
    rate (write the replacing trial vector); donor rows are on-chip reuse."""
    D = w["D"]
    if w["kind"] == "rot_osc":
        return 2.0 * D * D * trials, "TFLOP/s"
    return (4.0 * D + 8.0 + accept_rate * 4.0 * D) * trials, "GB/s"


def kernel_sources_sha256():
    csrc = os.path.join(ROOT, "paper_2405_16551_amd", "csrc")
    h = hashlib.sha256()
    for f in ("de_kernels.hip", "de_tile.hpp", "de_device.hpp", "de_internal.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel_ms, w):
    """HBM GB/s of the generation kernel: bytes per generation from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by a copy of
    known size; the median dispatch times the launches per generation, two
    when the runs go as two staggered groups), divided by this run's average
    time per generation.  None when the kernel sources changed after the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    sha = kernel_sources_sha256()
    for entry in table.values():
        if entry.get("workload") == w and entry.get("source_sha256") == sha:
            per_gen = entry.get("hbm_bytes_per_generation",
                                entry["hbm_bytes_per_launch"])
            return round(per_gen / (kernel_ms * 1e-3) / 1e9, 1)
    return None


# Generations per timed library call: calls this long take the library's
# staggered run groups on the large rotated workloads (shorter calls are
# launched as one group).
SEG_MIN_GENS = 16


def time_workload(name, steps, warmup, seed=1):
    import torch

    from paper_2405_16551_amd import instances
    from paper_2405_16551_amd.de import DifferentialEvolution

    w = WORKLOADS[name]
    o, R = instances.make_instance(w["kind"], w["D"], 1)
    torch.cuda.synchronize()
    t_init = time.perf_counter()
    de = DifferentialEvolution(runs=w["runs"], NP=w["NP"], D=w["D"], F=0.5,
                               CR=0.9, seed=seed, kind=w["kind"], o=o, R=R,
                               gemm_prec=w["gemm_prec"],
                               jde=w.get("jde"))
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t_init) * 1e3
    stream = de.stream
    de.generation(warmup)
    torch.cuda.synchronize()
    acc0, _ = de.stats()
    # the K steps are library calls of at least SEG_MIN_GENS generations
    # each, five when K allows (launches back to back on the library's
    # stream); events on that stream bracket every call, so the average
    # launch duration includes the gaps between consecutive launches and
    # each call's start and end, and several segments give a median and a
    # spread
    nseg = max(1, min(5, steps // SEG_MIN_GENS))
    cuts = [steps * k // nseg for k in range(nseg + 1)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nseg + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(nseg):
        de.generation(cuts[k + 1] - cuts[k])
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = ev[0].elapsed_time(ev[nseg]) / steps
    seg_ms = sorted(ev[k].elapsed_time(ev[k + 1]) / (cuts[k + 1] - cuts[k])
                    for k in range(nseg))
    trials = w["runs"] * w["NP"]
    acc1, best = de.stats()
    accept_rate = (sum(acc1) - sum(acc0)) / float(trials * steps)
    # after the timed region: each run's best as the step computed it
    # (FP32 / BF16 product) against an FP64 re-evaluation of the same row
    f64, _ = de.best_f64()
    rel = [abs(b - e) / e if e > 0 else abs(b) for b, e in zip(best, f64)]
    work, unit = algorithmic(w, trials, accept_rate)
    if unit == "TFLOP/s":
        achieved = work / (kern_ms * 1e-3) / 1e12
        peak = BF16_PEAK_TFLOPS if w["gemm_prec"] == "bf16" else FP32_PEAK_TFLOPS
        bound = "mfma"
    else:
        achieved = work / (kern_ms * 1e-3) / 1e9
        peak = HBM_PEAK_GBS
        bound = "hbm"
    de.close()
    return dict(wall_s=wall, ms_per_step=wall / steps * 1e3,
                kernel_ms=kern_ms, init_ms=init_ms,
                segments=dict(n=nseg, median_ms_per_step=round(
                    seg_ms[nseg // 2], 5), min_ms_per_step=round(seg_ms[0], 5),
                    max_ms_per_step=round(seg_ms[-1], 5)),
                evals_per_s=trials * steps / wall,
                gens_per_s=steps / wall, accept_rate=round(accept_rate, 4),
                roofline=dict(bound=bound, achieved=round(achieved, 3),
                              peak=peak, unit=unit,
                              frac=round(achieved / peak, 4),
                              traffic=measured_traffic(kern_ms, name)),
                best_median=float(sorted(best)[len(best) // 2]),
                best_vs_fp64=dict(max_rel_err=float(f"{max(rel):.3e}"),
                                  median_rel_err=float(
                                      f"{sorted(rel)[len(rel) // 2]:.3e}")))


MIXED_RUNS = 512
MIXED_GRAPH_GENS = 16


def describe_mixed(nruns=MIXED_RUNS):
    return (f"DE/rand/1/bin, {nruns} independent runs of mixed size: NP from "
            "{32,64,128,256,512,1024}, D from {10,30,50,100,500}, F ~ "
            "U[0.4,0.9], CR ~ U[0.1,1.0] per run, rotated oscillating, bf16 "
            f"rotation product, autotuned tiles, {MIXED_GRAPH_GENS} generations "
            "per graph launch")


def time_batch(steps, warmup, nruns=MIXED_RUNS, graph_gens=MIXED_GRAPH_GENS):
    """The mixed batch: every run advances one generation per step; timed
    with HIP events on the batch's stream around whole graph replays."""
    import torch

    from paper_2405_16551_amd import instances
    from paper_2405_16551_amd.de import VARIANT_NAMES, DEBatch

    specs = instances.make_mixed_specs(nruns, seed=1)
    inst = instances.make_mixed_instances(specs, 1)
    t0 = time.perf_counter()
    b = DEBatch(specs, inst, graph_gens=graph_gens, seed=1)
    create_s = time.perf_counter() - t0
    steps = max(graph_gens, (steps + graph_gens - 1) // graph_gens * graph_gens)
    warm = max(graph_gens, (warmup + graph_gens - 1) // graph_gens * graph_gens)
    b.generation(warm)
    torch.cuda.synchronize()
    acc0 = sum(b.read()["accepted"])
    stream = b.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    b.generation(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    st = b.read()
    trials = sum(s[0] for s in specs)
    flops = sum(2.0 * s[0] * s[1] * s[1] for s in specs)
    plan, us = b.plan()
    b.close()
    achieved = flops / (ms * 1e-3) / 1e12
    return dict(
        workload=describe_mixed(nruns), runs=nruns, trials_per_gen=trials,
        steps=steps, warmup=warm, gens_per_s=round(steps / wall, 2),
        evals_per_s=round(trials * steps / wall, 1),
        ms_per_gen=round(ms, 5), wall_s=wall,
        accept_rate=round((sum(st["accepted"]) - acc0) / (trials * steps), 4),
        roofline=dict(bound="mfma", achieved=round(achieved, 3),
                      peak=BF16_PEAK_TFLOPS, unit="TFLOP/s",
                      frac=round(achieved / BF16_PEAK_TFLOPS, 4),
                      traffic=None,
                      scope="all kernels of one generation (2 D^2 FLOPs "
                            "per trial, unpadded)"),
        plan={str(D): VARIANT_NAMES[v] for D, v in plan.items()},
        tuner_us={str(D): [round(t, 1) for t in ts] for D, ts in us.items()},
        create_s=round(create_s, 3))


SUR_RUNS = 30
SUR_COMPONENTS = (8, 16, 32, 64)


def describe_surrogate(runs=SUR_RUNS, ncomp=8):
    return (f"surrogate-assisted DE/rand/1/bin, {runs} runs x NP=512, D=100, "
            f"composition of {ncomp} rotated oscillating components (weights "
            "exp(-d/(2*50^2)), biases 100k), F=0.5, CR=0.9; BF16 MLP "
            "100-256-256-1 trained online (Adam, lr 5e-3, minibatch 128, 1 "
            "step per generation, archive 4096), k=4 candidates per target, "
            "1 true evaluation")


def time_surrogate(gens=300, check_every=2, runs=SUR_RUNS, ncomp=8,
                   warm=True, tol=1e-6):
    """Plain form (k = 1, no model, same kernels) for `gens` generations,
    then the surrogate form for up to 2 * gens generations, on the
    composition of `ncomp` components (the objective's cost per evaluation
    grows with ncomp; the model's does not).  Two criteria of "the same
    best":
      median: the surrogate form's median best over the runs reaches the
              plain form's final median best;
      per run: every run's best is within `tol` (relative) of the plain
              form's final best of the same run (same run number, so the
              same population at generation 0); the time until half of the
              runs are there, and how many get there at all.
    Reported: GPU time to the same best from each form's steady-state time
    per generation (HIP events; the host reads every `check_every`
    generations are left out), wall clock of both (host loop included),
    true evaluations used."""
    import numpy as np
    import torch

    from paper_2405_16551_amd import instances
    from paper_2405_16551_amd.de import SurrogateDE

    comp = instances.make_composition(100, ncomp, 1)
    common = dict(runs=runs, NP=512, D=100, F=0.5, CR=0.9, comp=comp, seed=1,
                  hidden=256, batch=128, archive=4096, lr=5e-3)
    if warm:  # clocks up before anything is timed: a throwaway run of both
        for kw in (dict(k=1, steps=0, warmup_gens=0),
                   dict(k=4, steps=1, warmup_gens=0)):
            w = SurrogateDE(**kw, **dict(common, seed=99))
            w.generation(60)
            w.read()
            w.close()
    plain = SurrogateDE(k=1, steps=0, warmup_gens=0, **common)
    sur = SurrogateDE(k=4, steps=1, warmup_gens=5, **common)
    torch.cuda.synchronize()

    def gen_ms(s, n=30):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.generation(n)
        e1.record(s.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    # plain: `gens` generations, trace of every run's best
    t0 = time.perf_counter()
    done, tr_plain = 0, []
    while done < gens:
        plain.generation(check_every)
        done += check_every
        tr_plain.append(np.array(plain.read()["best_f"]))
    tp = time.perf_counter() - t0
    gp = done
    final = tr_plain[-1]
    target = float(np.median(final))
    # surrogate: until both criteria hold or 2 * gens generations
    t0 = time.perf_counter()
    done, med_at, half_at = 0, None, None
    first = np.full(runs, -1)
    while done < 2 * gens:
        sur.generation(check_every)
        done += check_every
        b = np.array(sur.read()["best_f"])
        first[(first < 0) & (b <= final * (1 + tol))] = done
        if med_at is None and float(np.median(b)) <= target:
            med_at = done
        if half_at is None and np.sum(first >= 0) >= (runs + 1) // 2:
            half_at = done
        if med_at is not None and half_at is not None:
            break
    ts = time.perf_counter() - t0
    gs = done
    mp, ms_ = gen_ms(plain), gen_ms(sur)
    plain.close()
    sur.close()
    out = dict(
        workload=describe_surrogate(runs, ncomp), runs=runs,
        components=ncomp,
        plain=dict(generations=gp, seconds=round(tp, 3),
                   gpu_ms_per_gen=round(mp, 4), median_best=target),
        surrogate=dict(generations=gs, seconds=round(ts, 3),
                       gpu_ms_per_gen=round(ms_, 4),
                       generations_to_median=med_at,
                       generations_to_half_runs=half_at,
                       runs_reaching_own_plain_best=int(np.sum(first >= 0))),
        per_run_tolerance=tol)
    if med_at is not None:
        out["gpu_time_speedup_median"] = round(gp * mp / (med_at * ms_), 3)
        out["true_evals_ratio_median"] = round(med_at / gp, 3)
    if half_at is not None:
        # per run: the plain form's time for half of the runs to reach their
        # own final best is the full `gens` generations
        out["gpu_time_speedup_half_runs"] = round(gp * mp / (half_at * ms_), 3)
    return out


def surrogate_crossover(gens=300):
    """The surrogate comparison on compositions of SUR_COMPONENTS components:
    where the model's fixed cost per generation is repaid by the saved true
    evaluations."""
    rows = []
    for k, n in enumerate(SUR_COMPONENTS):
        r = time_surrogate(gens=gens, ncomp=n, warm=(k == 0))
        rows.append(dict(components=n,
                         plain_gpu_ms_per_gen=r["plain"]["gpu_ms_per_gen"],
                         surrogate_gpu_ms_per_gen=r["surrogate"][
                             "gpu_ms_per_gen"],
                         true_evals_ratio_median=r.get(
                             "true_evals_ratio_median"),
                         gpu_time_speedup_median=r.get(
                             "gpu_time_speedup_median"),
                         gpu_time_speedup_half_runs=r.get(
                             "gpu_time_speedup_half_runs"),
                         runs_reaching_own_plain_best=r["surrogate"][
                             "runs_reaching_own_plain_best"]))
    return rows


def copy_ceiling(nbytes=1 << 30, reps=20):
    """Device-to-device copy of nbytes (read + write), timed with events:
    the measured HBM ceiling next to the 8 TB/s specification."""
    import torch
    n = nbytes // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return dict(bytes_moved=2 * nbytes, ms=round(ms, 4),
                GBps=round(2 * nbytes / (ms * 1e-3) / 1e9, 1))


def gemm_ceiling(reps=20):
    """BF16 library products (torch.mm, hipBLASLt on ROCm; contiguous 2-D
    operands, FP32 accumulation) timed with events: a large square product,
    and the rotation product of the 16-run, NP 1024, D 1000 step alone (16384
    trial rows x 1024 x 1024 padded, without building the trials, the
    objective or the selection).  The measured MFMA ceilings next to the
    2.5 PFLOP/s specification."""
    import torch
    out = {}
    for name, (m, k, n) in (("square_8192", (8192, 8192, 8192)),
                            ("step_product_16384x1024x1024",
                             (16384, 1024, 1024))):
        a = torch.randn(m, k, device="cuda").to(torch.bfloat16).contiguous()
        b = torch.randn(k, n, device="cuda").to(torch.bfloat16).contiguous()
        c = torch.mm(a, b)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            torch.mm(a, b, out=c)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = 2.0 * m * n * k / (ms * 1e-3) / 1e12
        out[name] = dict(us=round(ms * 1e3, 2), TFLOPs=round(tf, 1),
                         frac_of_peak=round(tf / BF16_PEAK_TFLOPS, 4))
        del a, b, c
    return out


def time_to_target(target=1e-8, max_gens=5000, check_every=30):
    import torch

    from paper_2405_16551_amd import instances
    from paper_2405_16551_amd.de import DifferentialEvolution

    o, _ = instances.make_instance("sphere", 10, 1)
    de = DifferentialEvolution(runs=1, NP=64, D=10, F=0.5, CR=0.9, seed=1,
                               kind="sphere", o=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, hits = de.evolve(max_gens, target=target, check_every=check_every)
    t = time.perf_counter() - t0
    de.close()
    return dict(workload=describe("sphere10"), target=target, seconds=t,
                first_hit_generation=hits[0], generations_run=done,
                check_every=check_every)


def time_to_target_c2(with_oracle, max_gens=6000, check_every=50):
    """Rotated D = 100, 64 runs x NP 256, FP32 product: wall time until half
    of the runs reach the FP64 oracle's median best after 3000 generations
    (the value tests/golden/make_c2_reference.py stores).  The GPU side is
    one de_evolve call; the time until half of the runs have hit is that
    call's wall time per generation times the generation at which the
    (n/2)-th run first hit.
    With with_oracle, the oracle's time to the same point is extrapolated
    from a timed sample of its generations on the host cores."""
    import numpy as np
    import torch

    import oracle
    from paper_2405_16551_amd import instances
    from paper_2405_16551_amd.de import DifferentialEvolution

    with open(os.path.join(ROOT, "tests", "golden",
                           "oracle_c2_distribution.json")) as f:
        ref = json.load(f)
    c = ref["config"]
    target = ref["median_final_best"]
    o, R = instances.make_instance(c["kind"], c["D"], c["obj_seed"])
    de = DifferentialEvolution(runs=c["runs"], NP=c["NP"], D=c["D"], F=c["F"],
                               CR=c["CR"], seed=c["seed"], kind=c["kind"],
                               o=o, R=R, gemm_prec="fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, hits = de.evolve(max_gens, target=target, check_every=check_every)
    t = time.perf_counter() - t0
    de.close()

    def half_hit(v):
        # generation by which half of the runs have reached the target (the
        # n/2-th smallest first-hit generation; never reached = infinity)
        h = np.sort(np.array([x if x >= 0 else np.inf for x in v],
                             dtype=np.float64))
        m = float(h[(len(h) + 1) // 2 - 1])
        return (m if np.isfinite(m) else None), int(np.isfinite(h).sum())

    gmed, ghit = half_hit(hits)
    out = dict(
        workload=(f"DE/rand/1/bin, {c['runs']} runs x NP={c['NP']}, "
                  f"D={c['D']}, rotated oscillating, fp32 rotation product"),
        target=target,
        target_source=("median over the runs of the FP64 oracle's best after "
                       f"{c['G']} generations (same seeds and instance)"),
        generations_run=done, seconds=round(t, 4), check_every=check_every,
        runs_at_target=ghit, generation_half_at_target=gmed,
        seconds_to_half_at_target=(round(gmed * t / done, 4) if gmed
                                   else None))
    if with_oracle:
        omed, _ = half_hit(ref["oracle_first_gen_at_target"])
        threads = oracle.max_threads()
        ng = 10
        t1 = time.perf_counter()
        oracle.run(runs=c["runs"], NP=c["NP"], D=c["D"], F=c["F"], CR=c["CR"],
                   lo=c["lo"], hi=c["hi"], seed=c["seed"],
                   kind=oracle.OBJ_ROT_OSC, o=o, R=R, G=ng, nthreads=threads)
        per_gen = (time.perf_counter() - t1) / ng
        out["oracle"] = dict(
            generation_half_at_target=omed, cores=threads,
            seconds_per_generation=round(per_gen, 4),
            seconds_to_half_at_target=(round(omed * per_gen, 2) if omed
                                       else None),
            sample=f"{ng} generations of all {c['runs']} runs in FP64, "
                   "extrapolated")
    return out


def c3_run(with_oracle, max_gens=4000, check_every=50):
    """The rotated D = 1000 workload as configured (16 runs x NP 1024, 2000
    generations), BF16 and FP32 product: per-step time and acceptance over
    the whole run (one library call, HIP events on the library's stream),
    median best after 2000 generations next to the FP64 oracle's (stored by
    tests/golden/make_c3_reference.py), and the wall time of one de_evolve
    call until half of the runs reach the oracle's median final best (the
    time to the (n/2)-th run's first hit, from the call's wall time per
    generation).  With with_oracle, the oracle's time to the same point is
    extrapolated from one timed generation of all 16 runs on the host
    cores."""
    import numpy as np
    import torch

    import oracle
    from paper_2405_16551_amd import instances
    from paper_2405_16551_amd.de import DifferentialEvolution

    with open(os.path.join(ROOT, "tests", "golden",
                           "oracle_c3_distribution.json")) as f:
        ref = json.load(f)
    c = ref["config"]
    G = c["G"]
    o, R = instances.make_instance(c["kind"], c["D"], c["obj_seed"])
    trials = c["runs"] * c["NP"]

    def make(prec):
        return DifferentialEvolution(runs=c["runs"], NP=c["NP"], D=c["D"],
                                     F=c["F"], CR=c["CR"], seed=c["seed"],
                                     kind=c["kind"], o=o, R=R, gemm_prec=prec)

    out = dict(workload=(f"DE/rand/1/bin, {c['runs']} runs x NP={c['NP']}, "
                         f"D={c['D']}, rotated oscillating, {G} generations"),
               oracle_median_best=float(np.median(ref["best"][str(G)])))
    for prec in ("bf16", "fp32"):
        de = make(prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(de.stream)
        de.generation(G)
        e1.record(de.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        acc, best = de.stats()
        out[prec] = dict(ms_per_step=round(ms / G, 5),
                         run_seconds=round(ms * 1e-3, 4),
                         accept_rate=round(sum(acc) / float(trials * G), 4),
                         median_best=float(np.median(best)))
        de.close()
    # wall time to the oracle's median final best (BF16 product)
    target = ref["median_final_best"]
    de = make("bf16")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, hits = de.evolve(max_gens, target=target, check_every=check_every)
    t = time.perf_counter() - t0
    de.close()
    h = np.sort(np.array([x if x >= 0 else np.inf for x in hits], float))
    gmed = float(h[(len(h) + 1) // 2 - 1])
    ohits = np.sort(np.array([x if x >= 0 else np.inf
                              for x in ref["oracle_first_gen_at_target"]],
                             float))
    omed = float(ohits[(len(ohits) + 1) // 2 - 1])
    tt = dict(target=target,
              target_source=("median over the runs of the FP64 oracle's best "
                             f"after {G} generations (same seeds and instance)"),
              generations_run=done, seconds=round(t, 4),
              check_every=check_every,
              runs_at_target=int(np.isfinite(h).sum()),
              generation_half_at_target=(gmed if np.isfinite(gmed) else None),
              seconds_to_half_at_target=(round(gmed * t / done, 4)
                                         if np.isfinite(gmed) else None))
    if with_oracle:
        threads = oracle.max_threads()
        pop = oracle.init_population(c["runs"], c["NP"], c["D"], c["lo"],
                                     c["hi"], c["seed"])
        fit = oracle.objective_batch(oracle.OBJ_ROT_OSC,
                                     pop.reshape(-1, c["D"]), o, R,
                                     nthreads=threads).reshape(c["runs"], -1)
        t1 = time.perf_counter()
        oracle.generation(pop, fit, F=c["F"], CR=c["CR"], lo=c["lo"],
                          hi=c["hi"], seed=c["seed"], gen=0,
                          kind=oracle.OBJ_ROT_OSC, o=o, R=R, nthreads=threads)
        per_gen = time.perf_counter() - t1
        tt["oracle"] = dict(
            generation_half_at_target=omed, cores=threads,
            seconds_per_generation=round(per_gen, 3),
            seconds_to_half_at_target=round(omed * per_gen, 1),
            sample=f"1 generation of all {c['runs']} runs in FP64, "
                   "extrapolated")
    out["time_to_target"] = tt
    return out


def cpu_baseline(name, budget_s=15.0):
    """The FP64 oracle on the host cores, one generation of one run of the
    workload (NP trials), repeated while the budget lasts."""
    import numpy as np

    import oracle
    from paper_2405_16551_amd import instances

    w = WORKLOADS[name]
    D, NP = w["D"], w["NP"]
    kind = oracle.OBJ_SPHERE if w["kind"] == "sphere" else oracle.OBJ_ROT_OSC
    o, R = instances.make_instance(w["kind"], D, 1)
    threads = oracle.max_threads()
    pop = oracle.init_population(1, NP, D, -100.0, 100.0, 1)
    fit = oracle.objective_batch(kind, pop.reshape(-1, D), o, R,
                                 nthreads=threads).reshape(1, NP)
    gens, t0 = 0, time.perf_counter()
    while True:
        out = oracle.generation(pop, fit, F=0.5, CR=0.9, lo=-100.0, hi=100.0,
                                seed=1, gen=gens, kind=kind, o=o, R=R,
                                nthreads=threads)
        pop, fit = out["pop_next"], out["fit_next"]
        gens += 1
        el = time.perf_counter() - t0
        if el >= budget_s or gens >= 10000:
            break
    assert np.isfinite(fit).all()
    return dict(value=NP * gens / el, unit="trial evals/s", cores=threads,
                kind="oracle",
                sample=(f"{gens} generation(s) of 1 run (NP={NP}, D={D}, "
                        f"{w['kind']}) in FP64, {el:.1f} s, OpenMP over "
                        f"individuals"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="rot1000_bf16",
                    choices=sorted(WORKLOADS) + ["mixed512", "surrogate"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device copy first (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the DE step runs on one GPU "
              "(independent runs would shard across GPUs with no exchange); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_calibration:
        copy_ceiling(nbytes=256 << 20, reps=1)
    if args.workload == "surrogate":
        r = time_surrogate()
        r["crossover"] = surrogate_crossover()
        print(json.dumps({"metric": "wall-time to the plain form's best",
                          "n_gpus": 1, "data": "synthetic", **r}), flush=True)
        return
    if args.workload == "mixed512":
        r = time_batch(args.steps, args.warmup)
        print(json.dumps({
            "metric": "trial evals/sec and gens/sec of a mixed batch "
                      "(% roofline)",
            "value": r["evals_per_s"], "unit": "trial evals/s", "n_gpus": 1,
            "steps": r["steps"], "warmup": r["warmup"],
            "ms_per_step": round(r["wall_s"] / r["steps"] * 1e3, 5),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16", "data": "synthetic",
            "config": {"workload": r["workload"], "runs": r["runs"]},
            "gens_per_s": r["gens_per_s"], "roofline": r["roofline"],
            "plan": r["plan"], "tuner_us": r["tuner_us"]}), flush=True)
        return
    main_res = time_workload(args.workload, args.steps, args.warmup)
    w = WORKLOADS[args.workload]
    line = {
        "metric": "trial evals/sec and gens/sec at NP=1024,D=1000 "
                  "(% roofline); wall-time to target",
        "value": round(main_res["evals_per_s"], 1),
        "unit": "trial evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if w["gemm_prec"] == "bf16" and w["kind"] == "rot_osc"
                 else "f32",
        "data": "synthetic",
        "config": {"workload": describe(args.workload),
                   "runs": w["runs"], "NP": w["NP"], "D": w["D"],
                   "objective": w["kind"], "gemm": w["gemm_prec"]},
        "gens_per_s": round(main_res["gens_per_s"], 2),
        "kernel_ms_per_step": round(main_res["kernel_ms"], 5),
        "segments": main_res["segments"],
        "init_ms": round(main_res["init_ms"], 3),
        "roofline": main_res["roofline"],
        "accept_rate": main_res["accept_rate"],
        "best_vs_fp64": main_res["best_vs_fp64"],
    }
    if not args.no_extras:
        comp = "sphere1000" if w["kind"] == "rot_osc" else "rot1000_bf16"
        c = time_workload(comp, max(50, args.steps // 2), args.warmup)
        line["companion"] = {
            "workload": describe(comp), "evals_per_s": round(c["evals_per_s"], 1),
            "gens_per_s": round(c["gens_per_s"], 2),
            "kernel_ms_per_step": round(c["kernel_ms"], 5),
            "accept_rate": c["accept_rate"], "roofline": c["roofline"]}
        if args.workload == "rot1000_bf16":
            # the same step with the rotation product in FP32 (the other
            # GPU arm of this workload; the FP64 oracle is cpu_baseline)
            f = time_workload("rot1000_fp32", 40, min(args.warmup, 5))
            line["fp32_product"] = {
                "workload": describe("rot1000_fp32"),
                "evals_per_s": round(f["evals_per_s"], 1),
                "kernel_ms_per_step": round(f["kernel_ms"], 5),
                "accept_rate": f["accept_rate"], "roofline": f["roofline"]}
        jname = "rot1000_bf16_jde" if w["kind"] == "rot_osc" else "sphere1000_jde"
        j = time_workload(jname, max(50, args.steps // 4), args.warmup)
        line["jde"] = {
            "workload": describe(jname), "evals_per_s": round(j["evals_per_s"], 1),
            "kernel_ms_per_step": round(j["kernel_ms"], 5),
            "accept_rate": j["accept_rate"], "roofline": j["roofline"]}
        line["batched"] = time_batch(max(64, args.steps // 4), args.warmup)
        line["surrogate"] = time_surrogate()
        line["surrogate_crossover"] = surrogate_crossover()
        line["time_to_target"] = time_to_target()
        line["time_to_target_c2"] = time_to_target_c2(
            with_oracle=not args.no_cpu_baseline)
        if args.workload == "rot1000_bf16":
            line["c3_run"] = c3_run(with_oracle=not args.no_cpu_baseline)
        line["copy_ceiling"] = copy_ceiling()
        line["gemm_ceiling"] = gemm_ceiling()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
