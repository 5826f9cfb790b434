"""GPU parity of the surrogate-assisted variant (include/de_surrogate.h)
against the FP64 oracle, through the C ABI.

Parts and bars:
  * composition objective (Section 7.3.3 composition functions), FP32:
    within 2e-5 relative of the oracle on the same FP32 rows;
  * initial population bit-exact (same draws as the plain path), its
    fitness and the archive's first round;
  * MLP inference in BF16 on MFMA: |y - y_FP64| <= 4 * 2^-8 * S, S the same
    network evaluated on absolute values (each BF16 operand rounding moves a
    product by at most 2^-9 of its magnitude; ReLU is 1-Lipschitz);
  * one Adam step (FP32): the step's gradient, recovered from the first
    moment, within 1e-4 of its largest entry plus 1e-3 relative of the
    oracle's backpropagated gradient on the same minibatch (rows drawn by
    the documented counter), except for a small share of entries whose
    ReLU decision flips between FP32 and FP64; the update consistent with
    Adam on the GPU's own moments;
  * one screened generation: candidates within one FP32 fused rounding of
    the oracle's, predictions within the inference bar, the chosen
    candidate's oracle prediction within twice the bar of the minimum,
    evaluated f and selection as in the plain path.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2405_16551_amd import instances
from tests.gpu_helpers import HI, LO, host, trial_atol

pytestmark = pytest.mark.gpu

F_RTOL = 2e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    yield


def make_sur(runs=2, NP=64, D=20, n=8, F=0.5, CR=0.9, seed=1, **kw):
    from paper_2405_16551_amd.de import SurrogateDE
    comp = instances.make_composition(D, n, 1)
    s = SurrogateDE(runs=runs, NP=NP, D=D, F=F, CR=CR, comp=comp, lo=LO,
                    hi=HI, seed=seed, **kw)
    return s, comp


def comp_f(X, comp):
    O, R, bias, sigma = comp
    return oracle.composition_batch(np.asarray(X, np.float64), O, R, bias,
                                    sigma, nthreads=8)


def split(theta, D, H):
    o = 0
    W1 = theta[o:o + H * D].reshape(H, D); o += H * D
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    return W1, b1, W2, b2, w3, theta[o]


def abs_scale(theta, X, D, H):
    """The network on absolute values: bounds every partial sum."""
    W1, b1, W2, b2, w3, b3 = (np.abs(np.asarray(t, np.float64))
                              for t in split(np.asarray(theta, np.float64), D, H))
    xs = np.abs((2 * np.asarray(X, np.float64) - (LO + HI)) / (HI - LO))
    h1 = xs @ W1.T + b1
    h2 = h1 @ W2.T + b2
    return h2 @ w3 + b3


def test_composition_objective_matches_oracle():
    s, comp = make_sur(runs=1, NP=8, D=100)
    O = comp[0]
    rng = np.random.default_rng(0)
    X = rng.uniform(LO, HI, (64, 100)).astype(np.float32)
    scale = np.logspace(-6, 0, 64)[:, None].astype(np.float32)
    X[:32] = (O[1] + (X[:32] - O[1]) * scale[:32]).astype(np.float32)
    X[0] = O[0]
    f = host(s.eval(X)).astype(np.float64)
    fo = comp_f(X, comp)
    np.testing.assert_allclose(f, fo, rtol=F_RTOL, atol=1e-30)
    s.close()


def test_initial_population_archive_and_fitness():
    s, comp = make_sur(runs=3, NP=40, D=30)
    want = oracle.init_population(3, 40, 30, LO, HI, 1).astype(np.float32)
    pop = host(s.population())
    np.testing.assert_array_equal(pop, want)
    f = host(s.fitness()).astype(np.float64)
    np.testing.assert_allclose(f, comp_f(want.reshape(-1, 30), comp).reshape(3, 40),
                               rtol=F_RTOL)
    X, T, filled = s.archive()
    assert filled == [40, 40, 40]
    np.testing.assert_array_equal(X[:, :40], pop)
    np.testing.assert_allclose(T[:, :40], np.log10(host(s.fitness()) + 1e-8),
                               rtol=1e-6)
    st = s.read()
    assert st["best_f"] == [float(v) for v in host(s.fitness()).min(axis=1)]
    s.close()


@pytest.mark.parametrize("D,H", [(100, 256), (20, 64)])
def test_model_inference_within_bf16_bound(D, H):
    s, _ = make_sur(runs=2, NP=64, D=D, hidden=H, steps=3, warmup_gens=1)
    s.generation(4)  # trained weights with nonzero biases
    theta, _, _, _ = s.get_model()
    rng = np.random.default_rng(1)
    X = rng.uniform(LO, HI, (100, D)).astype(np.float32)
    for run in range(2):
        y = host(s.predict(run, X)).astype(np.float64)
        yo = oracle.mlp_forward(theta[run].astype(np.float64), X, D=D, H=H,
                                lo=LO, hi=HI)
        bound = 4 * 2.0 ** -8 * abs_scale(theta[run], X, D, H)
        err = np.abs(y - yo)
        print(f"D={D} H={H} run {run}: max err {err.max():.3e}, "
              f"max err/bound {(err / bound).max():.3f}")
        assert (err <= bound).all()
    s.close()


# (20, 64, 64): the general training kernels; (100, 256, 128) and
# (100, 256, 256): the configured model, whose forward pass has
# compile-time K extents and whose gradient product requests its operands
# 32 K-steps ahead (minibatches of 128 and 256)
@pytest.mark.parametrize("D,H,B", [(20, 64, 64), (100, 256, 128),
                                   (100, 256, 256)])
def test_adam_step_matches_oracle(D, H, B):
    lr = 1e-3
    s, _ = make_sur(runs=2, NP=64, D=D, hidden=H, batch=B, steps=0,
                    archive=256, model_seed=9, lr=lr)
    s.generation(3)  # archive: 4 rounds of 64 rows
    theta0, m0, v0, t0 = s.get_model()
    assert t0 == 0
    X, T, filled = s.archive()
    s.train(1)
    theta1, m1, v1, t1 = s.get_model()
    assert t1 == 1
    key = np.array([9, 0], dtype=np.uint32)
    for run in range(2):
        idx = []
        for b in range(B):
            w = oracle.philox([0, b, t1, (5 << 24) | run], key)[0]
            idx.append(oracle.uniform_index(int(w[0]), filled[run]))
        Xb = X[run, idx].astype(np.float64)
        Tb = T[run, idx].astype(np.float64)
        loss, g = oracle.mlp_grad(theta0[run].astype(np.float64), Xb, Tb,
                                  D=D, H=H, lo=LO, hi=HI)
        g_gpu = m1[run].astype(np.float64) / 0.1  # first step: m = (1-b1) g
        tol = 1e-4 * np.abs(g).max() + 1e-3 * np.abs(g)
        bad = np.abs(g_gpu - g) > tol
        print(f"run {run}: loss {loss:.4f}, gradient entries off "
              f"{bad.sum()} / {g.size}")
        assert bad.mean() < 2e-3
        # the update is Adam on the GPU's own moments
        mh = m1[run].astype(np.float64) / 0.1
        vh = v1[run].astype(np.float64) / (1 - 0.999)
        upd = theta0[run] - lr * mh / (np.sqrt(vh) + 1e-8)
        np.testing.assert_allclose(theta1[run], upd, rtol=1e-5, atol=1e-8)
    s.close()


def test_model_state_roundtrip():
    s, _ = make_sur(runs=2, NP=32, D=10, hidden=32, batch=32, archive=64)
    th, m, v, t = s.get_model()
    rng = np.random.default_rng(3)
    th2 = (th + rng.normal(0, 0.01, th.shape)).astype(np.float32)
    m2 = rng.normal(0, 1e-3, m.shape).astype(np.float32)
    v2 = np.abs(rng.normal(0, 1e-6, v.shape)).astype(np.float32)
    s.set_model(th2, m2, v2, 17)
    a, b, c, t3 = s.get_model()
    np.testing.assert_array_equal(a, th2)
    np.testing.assert_array_equal(b, m2)
    np.testing.assert_array_equal(c, v2)
    assert t3 == 17
    s.close()


@pytest.mark.parametrize("k,warmup", [(4, 2), (1, 0), (3, 100)])
def test_screened_generation_matches_oracle(k, warmup):
    D, H, NP, runs = 20, 64, 48, 2
    s, comp = make_sur(runs=runs, NP=NP, D=D, hidden=H, k=k,
                       warmup_gens=warmup, steps=2, batch=32, archive=512,
                       F=0.6, CR=0.8, seed=3)
    s.generation(4)
    g = s.gen
    pop32 = host(s.population()).copy()
    fit32 = host(s.fitness()).copy()
    theta, _, _, _ = s.get_model()
    s.generation(1)
    cand, pred, choice = s.last()
    pop_n, fit_n = host(s.population()), host(s.fitness())
    use = k > 1 and g >= warmup
    O, R, bias, sigma = comp
    out = oracle.sur_generation(pop32, fit32, theta, k=k, F=0.6, CR=0.8,
                                lo=LO, hi=HI, seed=3, gen=g, use_model=use,
                                H=H, O=O, R=R, bias=bias, sigma=sigma,
                                nthreads=8)
    pop64 = pop32.astype(np.float64)
    ties = 0
    for r in range(runs):
        for i in range(NP):
            for c in range(k):
                ci = i | (c << 24)
                key = np.array([3, 0], dtype=np.uint32)
                w = oracle.philox([0, ci, g, (2 << 24) | r], key)[0]
                a_, b_, c_ = (oracle.uniform_index(int(w[0]), NP - 1),
                              oracle.uniform_index(int(w[1]), NP - 2),
                              oracle.uniform_index(int(w[2]), NP - 3))
                r1, r2, r3 = oracle.skip_triple(i, a_, b_, c_)
                tol = trial_atol(pop64[r, r1], pop64[r, r2], pop64[r, r3], 0.6)
                err = np.abs(cand[r, i, c].astype(np.float64) - out["cand"][r, i, c])
                assert (err <= tol).all(), (r, i, c, err.max())
            ch = int(choice[r, i])
            if use:
                po = oracle.mlp_forward(theta[r].astype(np.float64),
                                        cand[r, i].astype(np.float64), D=D,
                                        H=H, lo=LO, hi=HI)
                bound = 4 * 2.0 ** -8 * abs_scale(theta[r], cand[r, i], D, H)
                assert (np.abs(pred[r, i].astype(np.float64) - po) <= bound).all()
                assert po[ch] <= po.min() + 2 * bound.max()
            else:
                assert ch == 0
                assert (pred[r, i] == 0).all()
            fu = comp_f(cand[r, i, ch][None], comp)[0]
            fx = fit32[r, i]
            acc_g = not np.array_equal(pop_n[r, i], pop32[r, i]) or (
                fit_n[r, i] != fx)
            if abs(fu - fx) <= F_RTOL * max(abs(fu), abs(fx)):
                ties += 1
                continue
            assert acc_g == (fu < fx), (r, i, fu, fx)
            if acc_g:
                np.testing.assert_array_equal(pop_n[r, i], cand[r, i, ch])
                assert abs(fit_n[r, i] - fu) <= F_RTOL * fu
            else:
                np.testing.assert_array_equal(pop_n[r, i], pop32[r, i])
                assert fit_n[r, i] == fx
    assert ties <= 0.05 * runs * NP
    # the evaluated candidates entered the archive with log10(f + 1e-8)
    X, T, filled = s.archive()
    assert filled[0] == min(512, (g + 2) * NP)
    pos = [((g + 1) * NP + i) % 512 for i in range(NP)]
    for r in range(runs):
        chosen = cand[r, np.arange(NP), choice[r]]
        np.testing.assert_array_equal(X[r, pos], chosen)
    s.close()


def test_zero_generations_change_nothing():
    s, _ = make_sur()
    s.generation(2)
    pop, fit = host(s.population()).copy(), host(s.fitness()).copy()
    s.generation(0)
    assert s.gen == 2
    np.testing.assert_array_equal(host(s.population()), pop)
    np.testing.assert_array_equal(host(s.fitness()), fit)
    s.close()


def test_surrogate_runs_make_progress():
    s, _ = make_sur(runs=4, NP=128, D=20, hidden=64, batch=128, archive=2048,
                    warmup_gens=3, steps=2)
    b0 = s.read()["best_f"]
    s.generation(60)
    b1 = s.read()["best_f"]
    assert all(x1 < x0 for x0, x1 in zip(b0, b1))
    X, T, filled = s.archive()
    assert filled == [2048] * 4
    assert np.isfinite(T).all()
    s.close()
