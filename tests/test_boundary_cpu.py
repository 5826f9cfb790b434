"""C-ABI boundary checks that need no GPU: exported symbols, version,
argument validation (always synchronous and before any device call),
handle-state errors, and the separation of the product from the oracle."""
import ctypes
import math
import os
import re
import subprocess
import sys

import pytest

import paper_2405_16551_amd.de as d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "de.h")
HEADERS = [os.path.join(ROOT, "include", h)
           for h in ("de.h", "de_batch.h", "de_surrogate.h")]


def declared_functions():
    names = []
    for h in HEADERS:
        names += re.findall(r"DE_API\s+[\w\s\*]+?\b(de_\w+)\s*\(",
                            open(h).read())
    return names


def test_every_header_is_covered():
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == sorted(
        os.path.basename(h) for h in HEADERS)


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) == 39
    assert set(names) == set(d.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", d.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for n in names:
        assert n in exported, n
        assert hasattr(d._lib, n)
    # nothing else leaks from the library's C++ internals
    assert {n for n in exported if n.startswith("de_")} == set(names)


def test_abi_version_matches_header():
    m = re.search(r"#define DE_ABI_VERSION (\d+)", open(HEADER).read())
    assert d.de_abi_version() == int(m.group(1))


def test_strerror_covers_every_status():
    for s in range(6):
        assert d.de_strerror(s)
    assert d.de_strerror(99) == "unknown status"


def P(**kw):
    base = dict(runs=16, NP=1024, D=1000, F=0.5, CR=0.9, lo=-100.0, hi=100.0,
                seed=1)
    base.update(kw)
    return d.de_params(*[base[k] for k in ("runs", "NP", "D", "F", "CR", "lo",
                                           "hi", "seed")])


def O(kind=1, prec=1, ldr=1000, reserved=0, o=256, R=256):
    return d.de_objective(kind, prec, ldr, reserved, o, R)


def ws_status(p, o):
    n = ctypes.c_size_t(0)
    return d._lib.de_workspace_bytes(ctypes.byref(p), ctypes.byref(o),
                                     ctypes.byref(n)), n.value


@pytest.mark.parametrize("kw", [
    dict(runs=0), dict(runs=1 << 24), dict(NP=3), dict(NP=-5), dict(D=0),
    dict(F=0.0), dict(F=-0.5), dict(F=math.nan), dict(F=math.inf),
    dict(CR=-0.01), dict(CR=1.01), dict(CR=math.nan), dict(lo=100.0),
    dict(lo=200.0), dict(lo=-math.inf), dict(hi=math.nan),
    dict(lo=-3e38, hi=3e38), dict(runs=1 << 20, NP=1 << 12)])
def test_invalid_params_rejected(kw):
    assert ws_status(P(**kw), O())[0] == d.DE_E_INVAL


@pytest.mark.parametrize("okw", [
    dict(kind=2), dict(kind=-1), dict(prec=2), dict(reserved=1), dict(o=None),
    dict(R=None), dict(ldr=999), dict(o=258)])
def test_invalid_objective_rejected(okw):
    assert ws_status(P(), O(**okw))[0] == d.DE_E_INVAL


def test_sphere_ignores_rotation_fields():
    st, n = ws_status(P(), O(kind=0, prec=7, ldr=0, R=None))
    assert st == d.DE_OK and n > 0


def test_unsupported_sizes():
    assert ws_status(P(D=5000), O(ldr=5000))[0] == d.DE_E_UNSUPPORTED
    assert ws_status(P(D=5000), O(kind=0))[0] == d.DE_E_UNSUPPORTED
    assert ws_status(P(D=4096), O(kind=0))[0] == d.DE_OK
    assert ws_status(P(D=1088), O(ldr=1088))[0] == d.DE_OK
    # the largest supported widths: rotated D = 1152 (padded 1152; the BF16
    # tile then fills the 160 KB of LDS), separable D = 4096
    for prec in (0, 1):
        assert ws_status(P(D=1152), O(prec=prec, ldr=1152))[0] == d.DE_OK
        assert ws_status(P(D=1153), O(prec=prec, ldr=1153))[0] == \
            d.DE_E_UNSUPPORTED
    assert ws_status(P(D=4097), O(kind=0))[0] == d.DE_E_UNSUPPORTED


def test_workspace_bytes_layout():
    st, sep = ws_status(P(), O(kind=0))
    st2, bf = ws_status(P(), O(prec=1))
    st3, f32 = ws_status(P(), O(prec=0))
    assert st == st2 == st3 == d.DE_OK
    assert sep % 256 == 0 and bf % 256 == 0
    # rotated adds R in the operand layout (D padded to 1024) and an FP32
    # row-major copy of R for the FP64 re-evaluation
    copy = 1000 * 1000 * 4
    assert bf - sep == 1024 * 1024 * 2 + copy
    assert f32 - sep == 1024 * 1024 * 4 + copy
    assert d.de_workspace_bytes(P(), O(kind=0)) == sep


def _bufs(**kw):
    base = dict(pop0=1 << 20, pop1=2 << 20, fit0=3 << 20, fit1=4 << 20,
                ldx=1000, reserved=0, work=5 << 20, work_bytes=1 << 30)
    base.update(kw)
    return d.de_buffers((ctypes.c_void_p * 2)(base["pop0"], base["pop1"]),
                        (ctypes.c_void_p * 2)(base["fit0"], base["fit1"]),
                        base["ldx"], base["reserved"], base["work"],
                        base["work_bytes"])


@pytest.mark.parametrize("kw", [
    dict(pop0=None), dict(pop1=(2 << 20) + 4), dict(pop1=1 << 20),
    dict(fit1=3 << 20), dict(fit0=None), dict(ldx=999), dict(ldx=1002),
    dict(reserved=1), dict(work=None), dict(work=(5 << 20) + 64),
    dict(work_bytes=1024)])
def test_invalid_buffers_rejected_before_any_launch(kw):
    h = ctypes.c_void_p()
    st = d._lib.de_init_population(ctypes.byref(P()), ctypes.byref(O()),
                                   ctypes.byref(_bufs(**kw)), None,
                                   ctypes.byref(h))
    assert st == d.DE_E_INVAL
    assert h.value is None


def test_null_out_pointer_rejected():
    st = d._lib.de_init_population(ctypes.byref(P()), ctypes.byref(O()),
                                   ctypes.byref(_bufs()), None, None)
    assert st == d.DE_E_INVAL


def test_calls_without_a_live_handle():
    lib = d._lib
    i64 = ctypes.c_int64(0)
    dbl = ctypes.c_double(0)
    bogus = ctypes.c_void_p(0x12345670)
    for h in (None, bogus):
        assert lib.de_generation(h, 1, None) == d.DE_E_STATE
        assert lib.de_evolve(h, 10, 1e-8, 1, None, ctypes.byref(i64),
                             None) == d.DE_E_STATE
        assert lib.de_best(h, 0, None, None, ctypes.byref(dbl),
                           None) == d.DE_E_STATE
        assert lib.de_get_generation(h, ctypes.byref(i64)) == d.DE_E_STATE
        assert lib.de_read_stats(h, None, None, None) == d.DE_E_STATE
        assert lib.de_load_population(h, 0, None) == d.DE_E_STATE
        assert lib.de_eval(h, 16, 1, 4, 16, None) == d.DE_E_STATE
        assert lib.de_debug_draws(h, 0, None, None, None) == d.DE_E_STATE
        assert lib.de_best_f64(h, None, ctypes.byref(dbl), None) == d.DE_E_STATE
    assert lib.de_destroy(None) == d.DE_OK
    assert lib.de_destroy(bogus) == d.DE_E_STATE


def test_binding_fails_loudly_without_the_library(monkeypatch):
    monkeypatch.setattr(d, "LIB_PATH", "/nonexistent/libde.so")
    with pytest.raises(ImportError):
        d._load()


def test_product_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2405_16551_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                src = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src,
                                     re.M), fn
                assert "liboracle" not in src and "de_oracle" not in src, fn
    # and the oracle never touches the product
    for fn in os.listdir(os.path.join(ROOT, "oracle")):
        if fn.endswith((".py", ".c", ".h")):
            src = open(os.path.join(ROOT, "oracle", fn)).read()
            assert "paper_2405_16551_amd" not in src, fn
            assert "de_device" not in src and "libde" not in src, fn


@pytest.mark.parametrize("jkw", [
    dict(F_span=0.0), dict(F_span=-0.5), dict(F_lo=-0.1), dict(F_lo=math.nan),
    dict(F_span=math.inf), dict(tau_F=-0.1), dict(tau_F=1.5),
    dict(tau_CR=math.nan), dict(tau_CR=2.0)])
def test_invalid_jde_constants_rejected(jkw):
    base = dict(d.JDE_BREST)
    base.update(jkw)
    j = d.de_jde(base["F_lo"], base["F_span"], base["tau_F"], base["tau_CR"])
    h = ctypes.c_void_p()
    bufs = d.de_buffers((ctypes.c_void_p * 2)(256, 512),
                        (ctypes.c_void_p * 2)(768, 1024), 1000, 0, 1 << 20,
                        1 << 40)
    st = d._lib.de_init_population_jde(ctypes.byref(P()), ctypes.byref(O()),
                                       ctypes.byref(j), ctypes.byref(bufs),
                                       None, ctypes.byref(h))
    assert st == d.DE_E_INVAL
    assert d._lib.de_init_population_jde(ctypes.byref(P()), ctypes.byref(O()),
                                         None, ctypes.byref(bufs), None,
                                         ctypes.byref(h)) == d.DE_E_INVAL


def test_control_calls_need_a_jde_handle():
    f = (ctypes.c_float * 4)()
    assert d._lib.de_get_control(None, None, f, f) == d.DE_E_STATE
    assert d._lib.de_set_control(None, None, f, f) == d.DE_E_STATE


# --------------------------------------------------------------------------
# Surrogate-assisted variant (include/de_surrogate.h): checks are synchronous
# and precede any device access.

def _sur(**kw):
    base = dict(d.SURROGATE_DEFAULTS)
    base.update(kw)
    return d.de_surrogate_params(*[base[f] for f, _ in
                                   d.de_surrogate_params._fields_])


def _comp(n=8, ldr=100, sigma=50.0, reserved=0, bias_val=0.0):
    bias = (ctypes.c_float * n)(*([bias_val] * n))
    c = d.de_composition(n, ldr, sigma, reserved, 256, 512, bias)
    c._keep = bias
    return c


def sur_status(p, c, s):
    n = ctypes.c_size_t(0)
    return d._lib.de_sur_workspace_bytes(ctypes.byref(p), ctypes.byref(c),
                                         ctypes.byref(s), ctypes.byref(n)), n.value


def test_surrogate_workspace_and_model_size():
    p = P(runs=30, NP=512, D=100)
    st, n = sur_status(p, _comp(), _sur())
    assert st == d.DE_OK and n > 0
    assert d._lib.de_sur_model_size(100, 256) == 256 * 100 + 256 * 256 + 3 * 256 + 1
    # more runs need more workspace
    assert sur_status(P(runs=31, NP=512, D=100), _comp(), _sur())[1] > n


@pytest.mark.parametrize("skw", [
    dict(k=0), dict(k=17), dict(hidden=48), dict(hidden=512), dict(batch=48),
    dict(batch=2048), dict(archive=100), dict(steps=-1), dict(warmup_gens=-1),
    dict(lr=0.0), dict(lr=math.nan), dict(beta1=1.0), dict(beta2=-0.1),
    dict(eps=0.0)])
def test_invalid_surrogate_settings_rejected(skw):
    assert sur_status(P(runs=2, NP=512, D=100), _comp(), _sur(**skw))[0] == d.DE_E_INVAL


@pytest.mark.parametrize("ckw", [
    dict(n=0), dict(n=65), dict(ldr=99), dict(sigma=0.0), dict(sigma=math.inf),
    dict(reserved=1), dict(bias_val=math.nan)])
def test_invalid_composition_rejected(ckw):
    assert sur_status(P(runs=2, NP=512, D=100), _comp(**ckw), _sur())[0] == d.DE_E_INVAL


def test_surrogate_calls_on_missing_handles():
    f = (ctypes.c_float * 4)()
    g = ctypes.c_int64()
    assert d._lib.de_sur_generation(None, 1, None) == d.DE_E_STATE
    assert d._lib.de_sur_read(None, None, None, None, None) == d.DE_E_STATE
    assert d._lib.de_sur_get_generation(None, ctypes.byref(g)) == d.DE_E_STATE
    assert d._lib.de_sur_get_model(None, None, f, f, f, None) == d.DE_E_STATE
    assert d._lib.de_sur_train(None, 1, None) == d.DE_E_STATE
    assert d._lib.de_sur_destroy(None) == d.DE_E_STATE


def test_bench_refuses_more_than_one_gpu():
    # the step runs on one GPU; asking for more exits with a message
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_binding_binds_to_one_hip_runtime():
    # libde.so links against the HIP runtime; PyTorch ships its own copy.
    # Loading the library before PyTorch left a process with two HIP
    # runtimes, which crashed at the first device call.  The binding imports
    # PyTorch first: in a fresh interpreter, torch must be imported when the
    # library is loaded, and exactly one HIP runtime may be mapped after it.
    code = f"""
import ctypes, sys
sys.path.insert(0, {ROOT!r})
seen = []
_orig = ctypes.CDLL.__init__
def _init(self, name, *a, **k):
    if name and str(name).endswith("libde.so"):
        seen.append("torch" in sys.modules)
    _orig(self, name, *a, **k)
ctypes.CDLL.__init__ = _init
import paper_2405_16551_amd.de
maps = open("/proc/self/maps").read().splitlines()
hip = sorted({{ln.split()[-1] for ln in maps if "libamdhip64.so" in ln}})
print(seen, len(hip))
"""
    out = subprocess.run([sys.executable, "-c", code], capture_output=True,
                         text=True, timeout=300, check=True).stdout.split()
    assert out[0] == "[True]", out
    assert out[1] == "1", out


def _noalloc(p, o, gen=3, pop_cur=1 << 20, fit_cur=3 << 20, pop_next=2 << 20,
             fit_next=4 << 20, ldx=1000):
    return d._lib.de_generation_noalloc(ctypes.byref(p), ctypes.byref(o), gen,
                                        pop_cur, fit_cur, pop_next, fit_next,
                                        ldx, None)


@pytest.mark.parametrize("kw", [
    dict(gen=-1), dict(gen=(1 << 32) - 1), dict(pop_cur=None),
    dict(pop_next=(2 << 20) + 4), dict(pop_next=1 << 20), dict(fit_next=3 << 20),
    dict(fit_cur=None), dict(ldx=999), dict(ldx=1002)])
def test_noalloc_step_rejects_bad_arguments(kw):
    # checked on the host before any device work (no GPU needed)
    assert _noalloc(P(), O(), **kw) == d.DE_E_INVAL
    assert _noalloc(P(F=0.0), O()) == d.DE_E_INVAL
    assert _noalloc(P(), O(R=None)) == d.DE_E_INVAL


def test_noalloc_step_scratch_limit():
    # the static scratch holds 8 MiB: statistics (3 x 8 runs), a flag byte
    # per row, the padded shift and, rotated, R in the operand layout; a
    # separable problem of 10 M rows needs 10 MB of row flags
    assert _noalloc(P(runs=512, NP=20000, D=8), O(kind=0), ldx=8) == \
        d.DE_E_UNSUPPORTED
    assert _noalloc(P(runs=64, NP=131072, D=8), O(kind=0), ldx=8) == \
        d.DE_E_UNSUPPORTED
