"""Staggered run groups (rotated objective, problems with at least as many
tiles as compute units): the runs are split into two halves launched on two
streams, the second half offset by half a generation.  Every run's draws and
arithmetic are those of the single launch, so the populations, values and
statistics must equal, bit for bit, those of a process that turns the
stagger off (DE_STAGGER=0).
"""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from tests.gpu_helpers import host, make_de

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# 16 runs x NP 1024 -> 256 tiles of 64 rows: at least one per compute unit;
# 17 runs: halves of 8 and 9 runs
CASES = {
    "bf16": dict(runs=16, NP=1024, D=1000, kind="rot_osc", gemm_prec="bf16"),
    "bf16_odd_runs": dict(runs=17, NP=1000, D=700, kind="rot_osc",
                          gemm_prec="bf16"),
    "bf16_jde": dict(runs=16, NP=1024, D=1000, kind="rot_osc",
                     gemm_prec="bf16", jde=True),
    "fp32": dict(runs=16, NP=1024, D=300, kind="rot_osc", gemm_prec="fp32"),
}

SCRIPT = r"""
import hashlib, json, sys
sys.path.insert(0, sys.argv[1])
import torch
from tests.gpu_helpers import make_de
kw = json.loads(sys.argv[2])
de, _, _ = make_de(F=0.5, CR=0.9, seed=3, **kw)
de.generation(16)
torch.cuda.synchronize()
de.generation(20)
torch.cuda.synchronize()
h = hashlib.sha256()
h.update(de.population().cpu().numpy().tobytes())
h.update(de.fitness().cpu().numpy().tobytes())
acc, best = de.stats()
print(json.dumps(dict(digest=h.hexdigest(), acc=list(acc), best=list(best))))
de.close()
"""


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    yield


@pytest.mark.parametrize("name", list(CASES))
def test_staggered_groups_equal_single_launch(name):
    import torch
    kw = CASES[name]
    # this process: staggered (calls of at least 16 generations; the first
    # call runs without an offset, the second with one, once the first
    # call's time per generation is known)
    de, _, _ = make_de(F=0.5, CR=0.9, seed=3, **kw)
    de.generation(16)
    torch.cuda.synchronize()
    de.generation(20)
    torch.cuda.synchronize()
    h = hashlib.sha256()
    h.update(host(de.population()).tobytes())
    h.update(host(de.fitness()).tobytes())
    acc, best = de.stats()
    mine = dict(digest=h.hexdigest(), acc=list(acc), best=list(best))
    assert sum(acc) > 0
    de.close()
    # a separate process with the stagger off
    env = dict(os.environ, DE_STAGGER="0")
    out = subprocess.run([sys.executable, "-c", SCRIPT, ROOT, json.dumps(kw)],
                         env=env, cwd=ROOT, capture_output=True, text=True,
                         timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    ref = json.loads(out.stdout.strip().splitlines()[-1])
    print(name, mine["digest"][:16], ref["digest"][:16], flush=True)
    assert mine == ref


EVOLVE_SCRIPT = r"""
import hashlib, json, sys
sys.path.insert(0, sys.argv[1])
import torch
from tests.gpu_helpers import make_de
kw = json.loads(sys.argv[2])
de, _, _ = make_de(F=0.5, CR=0.9, seed=3, **kw)
de.generation(int(sys.argv[3]))
torch.cuda.synchronize()
h = hashlib.sha256()
h.update(de.population().cpu().numpy().tobytes())
h.update(de.fitness().cpu().numpy().tobytes())
acc, best = de.stats()
print(json.dumps(dict(digest=h.hexdigest(), acc=list(acc), best=list(best))))
de.close()
"""


def test_evolve_with_run_groups_equals_plain_generations():
    # de_evolve in chunks of 32 generations (each chunk a staggered call,
    # the next chunk enqueued before the previous chunk's flag is read) with
    # a target no run reaches: the same generations as one unsplit call in
    # a process with the stagger off
    import torch
    kw = CASES["bf16"]
    gens = 64
    de, _, _ = make_de(F=0.5, CR=0.9, seed=3, **kw)
    done, hits = de.evolve(gens, target=-1e30, check_every=32)
    torch.cuda.synchronize()
    assert done == gens and all(h < 0 for h in hits)
    h = hashlib.sha256()
    h.update(host(de.population()).tobytes())
    h.update(host(de.fitness()).tobytes())
    acc, best = de.stats()
    mine = dict(digest=h.hexdigest(), acc=list(acc), best=list(best))
    de.close()
    env = dict(os.environ, DE_STAGGER="0")
    out = subprocess.run([sys.executable, "-c", EVOLVE_SCRIPT, ROOT,
                          json.dumps(kw), str(gens)],
                         env=env, cwd=ROOT, capture_output=True, text=True,
                         timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    ref = json.loads(out.stdout.strip().splitlines()[-1])
    print("evolve", mine["digest"][:16], ref["digest"][:16], flush=True)
    assert mine["digest"] == ref["digest"]
    assert mine["best"] == ref["best"]
