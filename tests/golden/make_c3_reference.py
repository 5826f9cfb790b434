"""Writes oracle_c3_distribution.json: the FP64 oracle's best-fitness
distribution over the 16 runs of the rotated D = 1000 workload (NP = 1024,
F = 0.5, CR = 0.9, box [-100, 100], Philox seed 1, instance seed 1,
2000 generations) at fixed checkpoints, the acceptance count of every run,
and the median final best, which serves as the wall-time-to-target
threshold for that workload (Section 7.3.4: record the minimum error and
the time a run needs to reach it).

Calls only the FP64 oracle (and the seeded instance generator for its
inputs).  Takes about 30 minutes on 8 host threads.

    python tests/golden/make_c3_reference.py [threads]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2405_16551_amd import instances  # noqa: E402

CONFIG = dict(runs=16, NP=1024, D=1000, F=0.5, CR=0.9, lo=-100.0, hi=100.0,
              seed=1, obj_seed=1, kind="rot_osc", G=2000)
CHECKPOINTS = [10, 100, 500, 1000, 1500, 2000]
TRACE_EVERY = 10


def main():
    c = CONFIG
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    o, R = instances.make_instance(c["kind"], c["D"], c["obj_seed"])
    t0 = time.perf_counter()
    res = oracle.run(runs=c["runs"], NP=c["NP"], D=c["D"], F=c["F"],
                     CR=c["CR"], lo=c["lo"], hi=c["hi"], seed=c["seed"],
                     kind=oracle.OBJ_ROT_OSC, o=o, R=R, G=c["G"],
                     nthreads=threads)
    seconds = time.perf_counter() - t0
    trace = res["best_trace"]
    final = trace[:, c["G"]]
    target = float(np.median(final))
    # first generation at which each oracle run's best is at or below it
    hit = [int(np.argmax(trace[r] <= target)) if np.any(trace[r] <= target)
           else -1 for r in range(c["runs"])]
    out = dict(
        config=c, checkpoints=CHECKPOINTS,
        best={str(g): [float(v) for v in trace[:, g]] for g in CHECKPOINTS},
        trace_every=TRACE_EVERY,
        trace=[[float(v) for v in trace[r, ::TRACE_EVERY]]
               for r in range(c["runs"])],
        accepted=[int(v) for v in res["accepted"]],
        median_final_best=target,
        oracle_first_gen_at_target=hit,
        oracle_seconds=round(seconds, 1), oracle_threads=threads)
    with open(os.path.join(HERE, "oracle_c3_distribution.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"median final best {target:.6e}; oracle {seconds:.1f} s")


if __name__ == "__main__":
    main()
