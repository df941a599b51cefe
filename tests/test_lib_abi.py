"""CPU checks of the C-ABI library: it loads, exports every function that
include/dg.h declares, and validates configurations on the host before any
device work.  No compute call is made (no GPU here)."""
import os
import re

import pytest

import paper_1506_06140_amd as dg
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?(dg_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_function():
    lib = dg.load_library()
    names = _declared()
    assert "dg_init" in names and "dg_rk_stage" in names and "dg_adjoint_rhs" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(dg.EXPORTS)


def test_rate_state_size_matches_header():
    # the binding allocates and reads the carried rate state with the layout
    # the header states (8 slots, 16 doubles apart)
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    m = re.search(r"#define\s+DG_RATE_STATE\s+(\d+)", src)
    assert m and int(m.group(1)) == dg.DG_RATE_STATE
    assert dg.RATE_SLOTS * dg.RATE_STRIDE == dg.DG_RATE_STATE
    kern = open(os.path.join(ROOT, "paper_1506_06140_amd", "csrc", "dg_kernels.hip")).read()
    k = re.search(r"RATE_SLOTS\s*=\s*(\d+),\s*RATE_STRIDE\s*=\s*(\d+)", kern)
    assert k and (int(k.group(1)), int(k.group(2))) == (dg.RATE_SLOTS, dg.RATE_STRIDE)


def test_limiter_codes_match_header():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    m = re.search(r"enum\s*\{\s*DG_LIM_NONE\s*=\s*(\d+),\s*DG_LIM_MINMOD\s*=\s*(\d+),\s*DG_LIM_CHAR\s*=\s*(\d+)", src)
    assert m and tuple(int(x) for x in m.groups()) == (dg.DG_LIM_NONE, dg.DG_LIM_MINMOD, dg.DG_LIM_CHAR)


def test_static_scratch_size_matches_header():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    m = re.search(r"#define\s+DG_STATIC_SCRATCH_FLOATS\s+\((\d+)\s*\*\s*(\d+)\s*\*\s*(\d+)\)", src)
    assert m and int(m.group(1)) * int(m.group(2)) * int(m.group(3)) == dg.DG_STATIC_SCRATCH_FLOATS
    assert re.search(r"DG_ESCRATCH\s*=\s*-7", src) and dg.DG_ESCRATCH == -7


def test_strerror_covers_codes():
    for code in range(0, -8, -1):
        assert dg.strerror(code) != "unknown error"
    assert dg.strerror(-99) == "unknown error"


@pytest.mark.parametrize("field,value,code", [
    ("dim", 4, dg.DG_EUNSUPPORTED),
    ("k", 0, dg.DG_EUNSUPPORTED),
    ("k", 5, dg.DG_EUNSUPPORTED),
    ("gamma", 1.0, dg.DG_EINVAL),
    ("cfl", 0.0, dg.DG_EINVAL),
    ("flux", 7, dg.DG_EINVAL),
    ("slope_limiter", 3, dg.DG_EUNSUPPORTED),
])
def test_init_rejects_bad_configs_on_the_host(field, value, code):
    import ctypes as C
    lib = dg.load_library()
    cfg = dg.make_config(workloads.workload("density_wave"))
    setattr(cfg, field, value)
    ctx = C.c_void_p()
    assert lib.dg_init(C.byref(cfg), C.byref(ctx)) == code
    assert not ctx.value


@pytest.mark.parametrize("over,precision", [
    (dict(dim=3, n=(8, 8, 8), length=(1.0, 1.0, 1.0)), "fp64"),   # k = 4 is 2D only
    ({}, "bf16"),                                                  # no BF16 tables at k = 4
    (dict(refine_lo=(2, 2, 0), refine_hi=(4, 4, 0)), "fp64"),     # nor a refined box
])
def test_init_rejects_unsupported_k4(over, precision):
    import ctypes as C
    lib = dg.load_library()
    cfg = dg.make_config(workloads.workload("density_wave", k=4, **over), precision)
    ctx = C.c_void_p()
    assert lib.dg_init(C.byref(cfg), C.byref(ctx)) == dg.DG_EUNSUPPORTED
    assert not ctx.value


def test_init_rejects_non_cubic_cells():
    import ctypes as C
    lib = dg.load_library()
    cfg = dg.make_config(workloads.workload("density_wave", n=(32, 16, 1)))
    ctx = C.c_void_p()
    assert lib.dg_init(C.byref(cfg), C.byref(ctx)) == dg.DG_EINVAL


def test_null_arguments_are_rejected():
    lib = dg.load_library()
    assert lib.dg_init(None, None) == dg.DG_EINVAL
    assert lib.dg_rhs(None, None, None, None) == dg.DG_EINVAL
    assert lib.dg_status(None, None) == dg.DG_EINVAL
    lib.dg_destroy(None)
