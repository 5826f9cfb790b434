"""Writes oracle_c2_distribution.json: the FP64 oracle's best-fitness
distribution over the 64 runs of the rotated D = 100 workload (NP = 256,
F = 0.5, CR = 0.9, box [-100, 100], Philox seed 1, instance seed 1,
3000 generations) at fixed checkpoints, and its median final best, which
serves as the wall-time-to-target threshold for that workload.

Calls only the FP64 oracle (and the seeded instance generator for its
inputs).  Takes about 1.5 minutes on 8 host threads.

    python tests/golden/make_c2_reference.py
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

CONFIG = dict(runs=64, NP=256, D=100, F=0.5, CR=0.9, lo=-100.0, hi=100.0,
              seed=1, obj_seed=1, kind="rot_osc", G=3000)
CHECKPOINTS = [20, 100, 300, 1000, 3000]


def main():
    c = CONFIG
    o, R = instances.make_instance(c["kind"], c["D"], c["obj_seed"])
    threads = 8
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
        median_final_best=target,
        oracle_first_gen_at_target=hit,
        oracle_seconds=round(seconds, 2), oracle_threads=threads)
    with open(os.path.join(HERE, "oracle_c2_distribution.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"median final best {target:.6e}; oracle {seconds:.1f} s")


if __name__ == "__main__":
    main()
