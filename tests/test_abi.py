"""CPU checks of the C-ABI library: it loads, exports every function that
include/hz.h declares, the binding resolves them all, and the host-only
V-cycle plan agrees with the oracle's plan (no device work)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hz.h")
LIB = os.path.join(ROOT, "paper_1712_08743_amd", "libhz.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|size_t|const\s+char)\s*\*?\s*(hz_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_path():
    names = declared_functions()
    for required in ("hz_create", "hz_destroy", "hz_set_model", "hz_point_rhs", "hz_solve",
                     "hz_misfit", "hz_plan", "hz_apply", "hz_smooth", "hz_restrict", "hz_prolong",
                     "hz_precond", "hz_status_str", "hz_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python -m paper_1712_08743_amd.build)"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    import paper_1712_08743_amd as hz
    assert set(hz.exported_symbols()) == set(declared_functions())


def test_status_strings_and_defaults():
    import paper_1712_08743_amd as hz
    lib = ctypes.CDLL(LIB)
    lib.hz_status_str.restype = ctypes.c_char_p
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert lib.hz_status_str(code)
    o = hz.default_opts()
    assert o.krylov == hz.HZ_BICGSTAB and o.tol == 1e-8 and o.nu1 == 2 and o.nu2 == 2
    assert (o.beta1, o.beta2) == (1.0, 0.5) and o.jacobi_w == 0.8 and o.gmres_m == 30
    assert o.autotune == 1 and o.chunk_rows == 0 and o.graphs == 0 and o.restart_at == 0
    assert o.coarse == hz.HZ_COARSE_AUTO and o.coarse_sweeps == 2


@pytest.mark.parametrize("shape,h,f,cmin,cmax", [
    ((201, 201), 10.0, 5.0, 1200.0, 2800.0),
    ((401, 801), 10.0, 3.0, 1275.0, 5175.0),
    ((401, 801), 10.0, 5.0, 1275.0, 5175.0),
    ((401, 801), 10.0, 8.0, 1275.0, 5175.0),
    ((401, 801), 10.0, 12.0, 1275.0, 5175.0),
    ((301, 601), 10.0, 10.0, 1500.0, 3500.0),
    ((129, 129), 10.0, 15.0, 1500.0, 3000.0),
    ((513, 513), 10.0, 2.0, 1500.0, 3000.0),
    ((1001,), 5.0, 10.0, 1500.0, 3000.0),
    ((257,), 20.0, 25.0, 1400.0, 3000.0),
])
def test_host_plan_matches_oracle_plan(shape, h, f, cmin, cmax):
    import paper_1712_08743_amd as hz
    from oracle import lfa
    om = 2 * np.pi * f
    for beta in ((1.0, 0.5), (1.0, 1.0)):
        for wdef in (0.8, 0.6):
            L0, w0 = lfa.plan(shape, h, om, 1 / cmax, 1 / cmin, beta[0], beta[1], w_default=wdef)
            L1, w1 = hz.plan_grid(shape, h, 1 / cmax, 1 / cmin, f, beta=beta, jacobi_w=wdef)
            assert L0 == L1 and np.allclose(w0, w1, rtol=0, atol=1e-15), (w0, w1)


def test_host_plan_rejects_bad_input():
    import paper_1712_08743_amd as hz
    with pytest.raises(hz.HzError):
        hz.plan_grid((201, 201), 10.0, 1e-3, 5e-4, 5.0)  # m_max < m_min
    with pytest.raises(hz.HzError):
        hz.plan_grid((201, 201), 10.0, 1 / 3000, 1 / 1500, 5.0, levels=9)


def test_host_plan_refuses_a_large_exact_coarsest_level():
    """An exactly solved coarsest level is inverted densely (one launch per
    pivot, n^3 work), so more than 4096 unknowns there is refused by the
    host plan; the same level smoothed instead of solved is accepted."""
    import paper_1712_08743_amd as hz
    mmin, mmax = 1 / 3500, 1 / 1500
    # 301 x 601 with three levels: 76 x 151 = 11 476 unknowns on the coarsest level
    for coarse in ("exact", "auto"):
        with pytest.raises(hz.HzError) as ei:
            hz.plan_grid((301, 601), 10.0, mmin, mmax, 3.0, levels=3, coarse=coarse)
        assert ei.value.code == hz.HZ_ERR_SHAPE
    L, w = hz.plan_grid((301, 601), 10.0, mmin, mmax, 3.0, levels=3, coarse="jacobi")
    assert L == 3 and len(w) == 2
    # auto smooths that level where its smallest kh reaches 2.5 (12 Hz: 2 pi 12 * 40 / 3500 = 0.86; not here)
    # 64 x 64 with one level: 4096 unknowns, the largest accepted
    assert hz.plan_grid((64, 64), 10.0, mmin, mmax, 3.0, levels=1)[0] == 1
    with pytest.raises(hz.HzError):
        hz.plan_grid((65, 65), 10.0, mmin, mmax, 3.0, levels=1)
    # the default plan stays far below the limit
    assert hz.plan_grid((301, 601), 10.0, mmin, mmax, 3.0)[0] == 6


def test_footprint_grows_with_the_work():
    import paper_1712_08743_amd as hz
    f1 = hz.footprint((257, 257), 1, 1)
    f8 = hz.footprint((257, 257), 1, 8)
    f8x2 = hz.footprint((257, 257), 2, 8)
    big = hz.footprint((513, 513), 1, 8)
    assert 0 < f1 < f8 < f8x2 < big
    # about 11 fine complex vectors per right-hand side dominate
    assert 11 * 16 * 257 * 257 * 8 <= f8 <= 20 * 16 * 257 * 257 * 8
    assert hz.footprint((257, 257), 1, 8, krylov="gmres", gmres_m=30) > f8 + 30 * 16 * 257 * 257 * 8


def test_every_context_call_refuses_a_null_context():
    """Each call that takes a context returns HZ_ERR_ARG for NULL (host-side
    check; zero sizes and NULL pointers everywhere else, no device work)."""
    import paper_1712_08743_amd as hz
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    lib = ctypes.CDLL(LIB)
    calls = re.findall(r"^\s*int\s+(hz_\w+)\s*\(\s*(?:const\s+)?hz_ctx\s*\*\s*\w+([^;]*)\);", text, flags=re.M | re.S)
    assert len(calls) >= 19
    for name, rest in calls:
        argtypes, args = [ctypes.c_void_p], [None]
        for p in (q.strip() for q in rest.split(",") if q.strip()):
            if "*" in p:
                argtypes.append(ctypes.c_void_p); args.append(None)
            elif p.startswith("double"):
                argtypes.append(ctypes.c_double); args.append(0.0)
            elif p.startswith("unsigned"):
                argtypes.append(ctypes.c_uint); args.append(0)
            else:
                argtypes.append(ctypes.c_int); args.append(0)
        f = getattr(lib, name)
        f.argtypes, f.restype = argtypes, ctypes.c_int
        assert f(*args) == hz.HZ_ERR_ARG, name


def test_traffic_hash_follows_the_code_not_its_comments():
    """A stored HBM-traffic measurement stays valid across comment and layout
    edits of the kernel sources, and not across a change of the code."""
    from paper_1712_08743_amd import profiling
    code = "__global__ void k(double* a) {\n  a[0] = 1.0;  // one\n}\n"
    commented = "/* the kernel\n   sets one value */\n__global__ void k(double* a) {\n    a[0] = 1.0;\n}\n"
    changed = "__global__ void k(double* a) {\n  a[0] = 2.0;  // one\n}\n"
    assert profiling._code_only(code) == profiling._code_only(commented)
    assert profiling._code_only(code) != profiling._code_only(changed)
    assert len(profiling.kernel_source_hash()) == 16
