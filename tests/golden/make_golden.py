"""Writes the oracle regression fixtures in this folder.

Calls only the FP64 oracle (and the seeded instance generator for its
inputs).  The paper prints no worked numerical example for DE/rand/1/bin,
so these files pin the oracle against accidental change, not against the
paper: any later change to them must name the passage that justifies it.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2405_16551_amd import instances  # noqa: E402


def main():
    out = {}
    # sphere, 1 run, NP=64, D=10, F=0.5, CR=0.9, box [-100,100], seed 1
    o, _ = instances.make_instance("sphere", 10, 1)
    res = oracle.run(runs=1, NP=64, D=10, F=0.5, CR=0.9, lo=-100.0, hi=100.0,
                     seed=1, kind=0, o=o, G=400, target=1e-8)
    gens = [0, 1, 10, 50, 100, 200, 400]
    out["sphere_np64_d10_seed1"] = dict(
        generations=gens,
        best=[float(res["best_trace"][0, g]) for g in gens],
        hit_gen=int(res["hit_gen"][0]), accepted=int(res["accepted"][0]))
    # rotated oscillating, 2 runs, NP=16, D=8, obj_seed 1, seed 7
    o, R = instances.make_instance("rot_osc", 8, 1)
    res = oracle.run(runs=2, NP=16, D=8, F=0.5, CR=0.9, lo=-100.0, hi=100.0,
                     seed=7, kind=1, o=o, R=R, G=100, target=1e-8)
    gens = [0, 1, 10, 50, 100]
    out["rot_osc_np16_d8_seed7"] = dict(
        generations=gens,
        best=[[float(res["best_trace"][r, g]) for g in gens] for r in range(2)],
        accepted=[int(v) for v in res["accepted"]])
    # first draws of individual 0..3, seed 1, run 0, gen 0, NP=64, D=10
    out["draws_seed1_np64_d10"] = [list(oracle.draw_indices(1, 0, 0, i, 64,
                                                            10))
                                   for i in range(4)]
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
