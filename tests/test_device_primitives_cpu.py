"""The GPU library's device primitives, compiled for the host, against the
independent FP64 oracle (draws) and NumPy (sin^2, ordering).  Runs on CPU.

The primitives are the ones every kernel uses: Philox4x32-10 blocks, the
donor sampler of eq. 2, the crossover test of eq. 3, the clamped mutant
coordinate, sin^2 of the rotated objective, the ordered (f, index) key and
the XCD block remap.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def prim(tmp_path_factory):
    exe = tmp_path_factory.mktemp("prim") / "device_primitives"
    src = os.path.join(HERE, "pins", "device_primitives.cpp")
    inc = os.path.join(ROOT, "paper_2405_16551_amd", "csrc")
    try:
        subprocess.run(["hipcc", "-O2", "-I", inc, "-o", str(exe), src],
                       check=True, capture_output=True, timeout=600)
    except (OSError, subprocess.CalledProcessError) as e:  # pragma: no cover
        pytest.skip(f"hipcc unavailable: {e}")

    def run(mode, lines):
        out = subprocess.run([str(exe), mode], input="\n".join(lines) + "\n",
                             capture_output=True, text=True, check=True,
                             timeout=600)
        return out.stdout.strip().splitlines()
    return run


def f32_bits(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


def bits_f32(b):
    return np.asarray(b, dtype=np.uint32).view(np.float32)


def test_philox_blocks_match_oracle(prim):
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**32, (2000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, (2000, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0], key[0] = 0, 0
    ctr[1], key[1] = 0xFFFFFFFF, 0xFFFFFFFF
    got = prim("philox", [f"{k[0]} {k[1]} {c[0]} {c[1]} {c[2]} {c[3]}"
                          for c, k in zip(ctr.tolist(), key.tolist())])
    got = np.array([[int(v) for v in ln.split()] for ln in got], dtype=np.uint64)
    np.testing.assert_array_equal(got.astype(np.uint32), oracle.philox(ctr, key))


def test_donors_match_oracle(prim):
    rng = np.random.default_rng(2)
    q = []
    for _ in range(3000):
        NP = int(rng.integers(4, 3000))
        q.append((int(rng.integers(0, 2**64 - 1, dtype=np.uint64)),
                  int(rng.integers(0, 1 << 24)), int(rng.integers(0, 2**32)),
                  int(rng.integers(0, NP)), NP, int(rng.integers(1, 2000))))
    for NP in (4, 5, 6):  # the smallest populations, every target
        for i in range(NP):
            q.append((9, 1, 2, i, NP, 3))
    got = prim("donors", [" ".join(map(str, t)) for t in q])
    for t, ln in zip(q, got):
        assert tuple(int(v) for v in ln.split()) == oracle.draw_indices(*t)


def test_crossover_word_test_is_the_24_bit_comparison(prim):
    # eq. 3 on the 2^-24 lattice: take the mutant iff (w >> 8) <= threshold;
    # the library compares the whole word with 256 threshold + 255, so check
    # words on both sides of every boundary, thresholds up to 2^24 (CR = 1)
    rng = np.random.default_rng(8)
    lines, want = [], []
    for thr in (0, 1, 2, 1 << 23, (1 << 24) - 2, (1 << 24) - 1, 1 << 24):
        words = {0, 1, 255, 256, 0xFFFFFFFF, 0xFFFFFF00, 0xFFFFFEFF}
        for d in (-1, 0, 255, 256):
            words.add((thr * 256 + d) % 2**32)
        words.update(int(v) for v in rng.integers(0, 2**32, 64))
        for w in sorted(words):
            lines.append(f"{w} {thr}")
            want.append("1" if (w >> 8) <= thr else "0")
    assert prim("xover", lines) == want


def test_crossover_mask_matches_oracle(prim):
    rng = np.random.default_rng(3)
    lines, want = [], []
    for CR in (0.0, 2**-24, 0.1, 0.5, 0.9, 1 - 2**-24, 1.0):
        thr = math.floor(CR * 2**24)
        for _ in range(8):
            seed, run, gen = 5, int(rng.integers(0, 64)), int(rng.integers(0, 10**6))
            i, D = int(rng.integers(0, 1024)), int(rng.integers(1, 300))
            jr = oracle.draw_indices(seed, run, gen, i, 1024, D)[3]
            lines.append(f"{seed} {run} {gen} {i} {D} {jr} {thr}")
            want.append("".join("1" if oracle.take_mutant(seed, run, gen, i, j,
                                                          jr, CR) else "0"
                                for j in range(D)))
    assert prim("mask", lines) == want


def test_sin_squared_accuracy(prim):
    rng = np.random.default_rng(4)
    t = np.concatenate([
        rng.uniform(-20000, 20000, 20000),
        rng.uniform(-4, 4, 5000),
        np.arange(-2000, 2000) * (np.pi / 2) + rng.uniform(-1e-4, 1e-4, 4000),
        np.logspace(-30, 1, 500), -np.logspace(-30, 1, 500),
        [0.0, -0.0, np.pi / 4, 3 * np.pi / 4]]).astype(np.float32)
    got = bits_f32(np.array([int(v) for v in prim(
        "sin2", [str(int(b)) for b in f32_bits(t)])], dtype=np.uint64).astype(
            np.uint32)).astype(np.float64)
    want = np.sin(t.astype(np.float64)) ** 2
    err = np.abs(got - want)
    # a few FP32 ulps relative to the value, plus half an ulp of 0.5
    assert (err <= 6e-7 * want + 3e-8).all(), float(np.max(err / (want + 1e-30)))
    assert got[-4] == 0.0 and got[-3] == 0.0


def test_mutant_coordinate_is_one_fused_rounding_and_clamped(prim):
    rng = np.random.default_rng(5)
    n = 5000
    x = rng.uniform(-100, 100, (n, 3)).astype(np.float32)
    F = rng.uniform(0.1, 2.0, n).astype(np.float32)
    lines = [" ".join(str(int(v)) for v in f32_bits([a, b, c, f, -100.0, 100.0]))
             for (a, b, c), f in zip(x, F)]
    got = bits_f32(np.array([int(v) for v in prim("mutant", lines)],
                            dtype=np.uint64).astype(np.uint32))
    x64 = x.astype(np.float64)
    d = (x[:, 1] - x[:, 2]).astype(np.float64)  # FP32 difference, then exact
    exact = np.clip(x64[:, 0] + F.astype(np.float64) * d, -100, 100)
    np.testing.assert_array_equal(got, exact.astype(np.float32))


def test_fit_key_orders_values_then_indices(prim):
    vals = np.array([-np.inf, -1e30, -1.0, -1e-30, -0.0, 0.0, 1e-30, 1.0,
                     1e30, np.inf, np.nan], dtype=np.float32)
    lines = []
    for v in vals:
        for idx in (0, 7):
            lines.append(f"{int(f32_bits(v))} {idx}")
    keys = [int(v) for v in prim("key", lines)]
    assert keys == sorted(keys)  # monotone in value, then index
    assert keys[8] < keys[10]   # -0.0 < +0.0 as keys: ties broken by bits


def test_xcd_remap_is_a_bijection(prim):
    ns = [1, 2, 7, 8, 9, 15, 16, 17, 255, 256, 257, 4095, 4096, 4097]
    assert prim("xcd", [str(n) for n in ns]) == ["ok"] * len(ns)
