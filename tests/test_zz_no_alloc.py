"""GPU: dg_rhs_noalloc (the BF16 right-hand side with the library's static
device scratch instead of the context's) against dg_rhs on the same context,
through the C ABI: equal bit for bit (same kernels, same inputs), on two
calls in a row, the second with a smaller input, then a state too large for
the static scratch, which is refused."""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _call(s, name, w):
    import torch
    out = s.empty()
    st = getattr(s.lib, name)(s.ctx, w.data_ptr(), out.data_ptr(), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, out


def _case(wl):
    import paper_1506_06140_amd as dg
    o = oracle.make(wl)
    w0 = o.initial_state()
    if wl["limiter"] or wl["positivity"]:
        w0, st = o.limit(w0)
        assert st == 0
    s = dg.Solver(wl, "bf16")
    return s, _dev(w0)


def test_rhs_noalloc_matches_rhs():
    import torch
    import paper_1506_06140_amd as dg
    big = workloads.workload("vortex", n=(160, 120, 1), length=(10.0, 7.5, 1.0))  # 2.7 M floats of scratch
    small = workloads.workload("blast_amr", k=2, n=(8, 7, 6), length=(1.0, 7 / 8, 6 / 8), refine_lo=(2, 2, 1),
                               refine_hi=(6, 5, 4), eps=1e-3, ic="kh3d", noise=1e-2, seed=6140)
    for wl in (big, small):
        s, w = _case(wl)
        assert s.nvar * s.N * s.ncell <= dg.DG_STATIC_SCRATCH_FLOATS
        st, ref = _call(s, "dg_rhs", w)
        assert st == dg.DG_OK
        st, got = _call(s, "dg_rhs_noalloc", w)
        assert st == dg.DG_OK
        torch.cuda.synchronize()
        assert s.status() == dg.DG_OK
        assert torch.equal(got, ref), (wl["name"], float((got - ref).abs().max()))
        print(wl["name"], s.ncell, "cells: dg_rhs_noalloc equals dg_rhs", flush=True)


def test_rhs_noalloc_refuses_large_states_and_other_precisions():
    import paper_1506_06140_amd as dg
    # the vector-ALU 3D path stages the BF16 volume term (the fused MFMA
    # kernel at k = 2, 3 stages nothing and has no size limit)
    wl = workloads.workload("kh3d", n=(128, 128, 16), length=(1.0, 1.0, 0.125), path3d=1)  # 13 M floats
    s = dg.Solver(wl, "bf16")
    assert s.nvar * s.N * s.ncell > dg.DG_STATIC_SCRATCH_FLOATS
    w = s.empty()
    st, _ = _call(s, "dg_rhs_noalloc", w)
    assert st == dg.DG_ESCRATCH
    assert "static scratch" in dg.strerror(st)
    s64 = dg.Solver(workloads.workload("vortex", n=(16, 16, 1), length=(10.0, 10.0, 1.0)))
    st, _ = _call(s64, "dg_rhs_noalloc", s64.empty())
    assert st == dg.DG_EINVAL
