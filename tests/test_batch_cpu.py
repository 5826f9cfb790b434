"""Batched mixed-size runs (include/de_batch.h): host-side layout and the
argument checks, which are synchronous and precede any device access."""
import ctypes
import math

import pytest

import paper_2405_16551_amd.de as d
from paper_2405_16551_amd import instances

FAKE = 1 << 20  # a 256-aligned non-null "device address"; never dereferenced


def params(specs, dims=None, **kw):
    dims = dims if dims is not None else sorted({s[1] for s in specs})
    runs = (d.de_run_spec * len(specs))(*[d.de_run_spec(*s) for s in specs])
    inst = (d.de_batch_instance * len(dims))(
        *[d.de_batch_instance(D, D, FAKE, FAKE)
          for D in dims])
    base = dict(lo=-100.0, hi=100.0, seed=1, gemm_prec=d.DE_GEMM_BF16,
                graph_gens=16, target=1e-8)
    base.update(kw)
    p = d.de_batch_params(len(specs), len(dims), runs, inst, base["lo"],
                          base["hi"], base["seed"], base["gemm_prec"],
                          base["graph_gens"], base["target"])
    p._keep = (runs, inst)
    return p


def layout_status(p):
    n = max(p.nruns, 1)
    a, b, c = (ctypes.c_int64 * n)(), (ctypes.c_int32 * n)(), (ctypes.c_int64 * n)()
    s1, s2, s3 = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    return d._lib.de_batch_layout(ctypes.byref(p), a, b, c, ctypes.byref(s1),
                                  ctypes.byref(s2), ctypes.byref(s3))


def test_layout_of_a_mixed_batch():
    specs = instances.make_mixed_specs(200, seed=3)
    lay = d.de_batch_layout(params(specs))
    end = 0
    fit = 0
    for r, (NP, D, F, CR) in enumerate(specs):
        assert lay["ldx"][r] == (D + 3) // 4 * 4
        assert lay["pop_off"][r] % 64 == 0
        assert lay["pop_off"][r] >= end  # runs do not overlap, in order
        end = lay["pop_off"][r] + NP * lay["ldx"][r]
        assert lay["fit_off"][r] == fit
        fit += NP
    assert lay["pop_floats"] >= end and lay["pop_floats"] - end < 64
    assert lay["fit_floats"] == fit
    # statistics, flags, tables, tile lists and BF16 R copies
    dims = sorted({s[1] for s in specs})
    rop = sum(2 * ((D + 31) // 32 * 32) ** 2 for D in dims)
    assert lay["work_bytes"] >= rop + fit


def test_mixed_specs_follow_the_recipe():
    specs = instances.make_mixed_specs(512, seed=1)
    assert len(specs) == 512
    assert {s[0] for s in specs} == set(instances.MIXED_NP)
    assert {s[1] for s in specs} == set(instances.MIXED_D)
    assert all(0.4 <= s[2] <= 0.9 and 0.1 <= s[3] <= 1.0 for s in specs)
    assert specs == instances.make_mixed_specs(512, seed=1)
    assert specs != instances.make_mixed_specs(512, seed=2)


GOOD = [(64, 10, 0.5, 0.9), (32, 30, 0.6, 0.2)]


@pytest.mark.parametrize("specs,dims,kw,want", [
    ([], [10], {}, d.DE_E_INVAL),                          # no runs
    (GOOD, [10], {}, d.DE_E_INVAL),                        # D=30 has no instance
    (GOOD, [10, 30, 30], {}, d.DE_E_INVAL),                # duplicate D
    ([(3, 10, 0.5, 0.9)], [10], {}, d.DE_E_INVAL),         # NP < 4
    ([(64, 10, 0.0, 0.9)], [10], {}, d.DE_E_INVAL),        # F = 0
    ([(64, 10, math.nan, 0.9)], [10], {}, d.DE_E_INVAL),
    ([(64, 10, 0.5, 1.5)], [10], {}, d.DE_E_INVAL),        # CR > 1
    ([(64, 10, 0.5, -0.1)], [10], {}, d.DE_E_INVAL),
    (GOOD, None, dict(lo=1.0, hi=1.0), d.DE_E_INVAL),
    (GOOD, None, dict(hi=math.inf), d.DE_E_INVAL),
    (GOOD, None, dict(graph_gens=0), d.DE_E_INVAL),
    (GOOD, None, dict(graph_gens=1025), d.DE_E_INVAL),
    (GOOD, None, dict(target=math.nan), d.DE_E_INVAL),
    (GOOD, None, dict(gemm_prec=7), d.DE_E_INVAL),
    (GOOD, None, dict(gemm_prec=d.DE_GEMM_FP32), d.DE_E_UNSUPPORTED),
    ([(64, 5000, 0.5, 0.9)], [5000], {}, d.DE_E_UNSUPPORTED),  # LDS
])
def test_invalid_batches_rejected(specs, dims, kw, want):
    assert layout_status(params(specs, dims, **kw)) == want


def test_instance_checks():
    p = params(GOOD)
    p.inst[0].ldr = 9
    assert layout_status(p) == d.DE_E_INVAL
    p = params(GOOD)
    p.inst[1].o = None
    assert layout_status(p) == d.DE_E_INVAL
    p = params(GOOD)
    p.inst[1].R = FAKE + 2
    assert layout_status(p) == d.DE_E_INVAL
    assert layout_status(params(GOOD)) == d.DE_OK


def create_status(p, pops=(FAKE, FAKE, FAKE, FAKE), work=FAKE, wbytes=None,
                  plan=None):
    lay = d.de_batch_layout(p)
    wb = lay["work_bytes"] if wbytes is None else wbytes
    h = ctypes.c_void_p()
    pl = (ctypes.c_int32 * len(plan))(*plan) if plan is not None else None
    return d._lib.de_batch_create(ctypes.byref(p), *pops, work, wb, pl, None,
                                  ctypes.byref(h))


def test_create_checks_precede_device_access():
    p = params(GOOD)
    assert create_status(p, pops=(None, FAKE, FAKE, FAKE)) == d.DE_E_INVAL
    assert create_status(p, pops=(FAKE + 4, FAKE, FAKE, FAKE)) == d.DE_E_INVAL
    assert create_status(p, work=FAKE + 16) == d.DE_E_INVAL
    assert create_status(p, work=None) == d.DE_E_INVAL
    lay = d.de_batch_layout(p)
    assert create_status(p, wbytes=lay["work_bytes"] - 1) == d.DE_E_INVAL
    assert create_status(p, plan=[0, 3]) == d.DE_E_INVAL
    assert create_status(p, plan=[-2, 0]) == d.DE_E_INVAL
    big = params([(64, 1500, 0.5, 0.9)])
    assert create_status(big, plan=[d.DE_BATCH_WIDE]) == d.DE_E_UNSUPPORTED
    h = ctypes.c_void_p()
    assert d._lib.de_batch_create(ctypes.byref(p), FAKE, FAKE, FAKE, FAKE,
                                  FAKE, 1 << 30, None, None, None) == d.DE_E_INVAL
    assert d._lib.de_batch_create(None, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 30,
                                  None, None, ctypes.byref(h)) == d.DE_E_INVAL


def test_calls_on_missing_handles():
    plan = (ctypes.c_int32 * 1)()
    g = ctypes.c_int64()
    assert d._lib.de_batch_plan(None, plan, None) == d.DE_E_STATE
    assert d._lib.de_batch_generation(None, 1, None) == d.DE_E_STATE
    assert d._lib.de_batch_read(None, None, None, None, None, None) == d.DE_E_STATE
    assert d._lib.de_batch_get_generation(None, ctypes.byref(g)) == d.DE_E_STATE
    assert d._lib.de_batch_destroy(None) == d.DE_E_STATE
    bogus = ctypes.c_void_p(FAKE)
    assert d._lib.de_batch_generation(bogus, 1, None) == d.DE_E_STATE
