"""GPU test of de_generation_noalloc (include/de.h): the generation step for
callers that cannot allocate, whose scratch is the library's fixed device
array instead of a workspace.  Through the C ABI, its output must equal that
of de_generation on a handle holding the same generation, bit for bit (same
kernels, draws and arithmetic), on two calls in a row, the second smaller
than the first, so that whatever the first call left in the shared array
cannot leak into the second.
"""
import numpy as np
import pytest

from tests.gpu_helpers import host, make_de

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    yield


def _noalloc_equals_handle(kind, prec, runs, NP, D, before):
    import torch

    import paper_2405_16551_amd.de as d
    print(f"no-alloc step: {kind}/{prec} runs {runs} NP {NP} D {D} "
          f"after {before} generations", flush=True)
    de, o, R = make_de(runs=runs, NP=NP, D=D, seed=4, kind=kind,
                       gemm_prec=prec)
    de.generation(before)
    g = de.gen
    pop_cur = de.pop[g & 1].clone()
    fit_cur = de.fit[g & 1].clone()
    pop_next = torch.full_like(pop_cur, float("nan"))
    fit_next = torch.full_like(fit_cur, float("nan"))
    d.de_generation_noalloc(de.params, de.objective, g, pop_cur.data_ptr(),
                            fit_cur.data_ptr(), pop_next.data_ptr(),
                            fit_next.data_ptr(), de.ldx, de._s())
    de.generation(1)
    want_pop, want_fit = host(de.population()), host(de.fitness())
    got_pop = host(pop_next.view(runs, NP, de.ldx)[:, :, :D])
    got_fit = host(fit_next.view(runs, NP))
    assert not np.isnan(got_pop).any() and not np.isnan(got_fit).any()
    np.testing.assert_array_equal(got_pop, want_pop)
    np.testing.assert_array_equal(got_fit, want_fit)
    # the step replaced some rows and kept others
    prev = host(pop_cur.view(runs, NP, de.ldx)[:, :, :D])
    moved = (got_pop != prev).any(axis=2)
    assert moved.any() and not moved.all()
    de.close()


@pytest.mark.parametrize("calls", [
    # the headline size (BF16 product, 1024-thread tiles), then a paired-row
    # BF16 tile at padded width 128
    [("rot_osc", "bf16", 16, 1024, 1000, 3), ("rot_osc", "bf16", 2, 64, 100, 7)],
    # FP32 product: padded width 384, then 128 (paired rows)
    [("rot_osc", "fp32", 2, 130, 300, 4), ("rot_osc", "fp32", 1, 40, 13, 2)],
    # separable: one wave per row, then lane groups
    [("sphere", "fp32", 3, 100, 1000, 5), ("sphere", "fp32", 2, 33, 10, 9)],
], ids=["rot-bf16", "rot-fp32", "sphere"])
def test_noalloc_step_equals_handle_step(calls):
    for kind, prec, runs, NP, D, before in calls:
        _noalloc_equals_handle(kind, prec, runs, NP, D, before)
