"""Seeded synthetic objective instances (shift vector o, rotation matrix R).

Section 7.3.1 of Janssen, Pullan & Liew (arXiv 2405.16551) defines every
benchmark function on the box [-100, 100]^D, shifted by a vector o whose
entries lie in [-80, 80], then rotated, z = M (x - o).  The paper takes o
and M from the CEC'14/'17 data files; those are not available, so this
module draws stand-ins of the same shape and distribution from a seed:

* o ~ U[-80, 80]^D, rounded to FP32 (so x = o, f = 0 is reachable in FP32);
* R Haar-distributed orthogonal: Q of the QR factorisation of a D x D
  standard Gaussian matrix, with column signs fixed by sign(diag(R_qr)),
  rounded to FP32.

The module holds none of the DE arithmetic; it only produces input data,
fed identically to the FP64 oracle and to the GPU library.
"""
from __future__ import annotations

import numpy as np

SHIFT_LO = -80.0
SHIFT_HI = 80.0


def _rng(obj_seed: int, D: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(obj_seed),
                                                         int(D), stream]))


def make_shift(D: int, obj_seed: int = 1) -> np.ndarray:
    """o ~ U[-80, 80]^D as float32."""
    return _rng(obj_seed, D, 0).uniform(SHIFT_LO, SHIFT_HI, size=D).astype(
        np.float32)


def make_rotation(D: int, obj_seed: int = 1) -> np.ndarray:
    """Haar-random orthogonal D x D matrix (row-major, z = R y) as float32."""
    g = _rng(obj_seed, D, 1).standard_normal((D, D))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    return np.ascontiguousarray(q.astype(np.float32))


def make_instance(kind: str, D: int, obj_seed: int = 1):
    """kind 'sphere' -> (o, None); 'rot_osc' -> (o, R)."""
    o = make_shift(D, obj_seed)
    if kind == "sphere":
        return o, None
    if kind == "rot_osc":
        return o, make_rotation(D, obj_seed)
    raise ValueError(f"unknown objective kind {kind!r}")


MIXED_NP = (32, 64, 128, 256, 512, 1024)
MIXED_D = (10, 30, 50, 100, 500)


def make_mixed_specs(nruns: int, seed: int = 1, NPs=MIXED_NP, Ds=MIXED_D,
                     F_range=(0.4, 0.9), CR_range=(0.1, 1.0)):
    """Run sizes and control parameters of a mixed batch: NP and D drawn
    uniformly from the given sets, F ~ U[F_range], CR ~ U[CR_range], all
    per run and rounded to float32.  Returns a list of (NP, D, F, CR)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 7]))
    NP = rng.choice(np.asarray(NPs), size=nruns)
    D = rng.choice(np.asarray(Ds), size=nruns)
    F = rng.uniform(*F_range, size=nruns).astype(np.float32)
    CR = rng.uniform(*CR_range, size=nruns).astype(np.float32)
    return [(int(a), int(b), float(c), float(e))
            for a, b, c, e in zip(NP, D, F, CR)]


def make_mixed_instances(specs, obj_seed: int = 1):
    """One rotated-objective instance (o, R) per distinct D of `specs`."""
    return {D: make_instance("rot_osc", D, obj_seed)
            for D in sorted({s[1] for s in specs})}


COMPOSITION_SIGMA = 50.0


def make_composition(D: int, n: int = 8, obj_seed: int = 1):
    """Composition of n rotated oscillating components (Section 7.3.3
    composition functions): shifts O [n, D] ~ U[-80, 80], Haar rotations
    R [n, D, D] (float32), biases 100 k (the component with the smallest
    bias holds the global optimum, as in the paper's definition), weight
    width sigma = 50.  Returns (O, R, bias, sigma)."""
    O = np.stack([_rng(obj_seed, D, 2 + 2 * k).uniform(
        SHIFT_LO, SHIFT_HI, size=D) for k in range(n)]).astype(np.float32)
    R = []
    for k in range(n):
        g = _rng(obj_seed, D, 3 + 2 * k).standard_normal((D, D))
        q, r = np.linalg.qr(g)
        R.append(q * np.sign(np.diag(r))[None, :])
    R = np.ascontiguousarray(np.stack(R).astype(np.float32))
    bias = (100.0 * np.arange(n)).astype(np.float32)
    return O, R, bias, COMPOSITION_SIGMA
