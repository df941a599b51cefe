"""GPU: the one-call SSP-RK3 step (dg_max_rate + dg_rk_step) against the
composed calls (dg_max_dt, three dg_rk_stage, dg_limit) and the FP64 oracle.

The fused step computes the same quantities in the same precision and order
(the time step from the same per-cell rates, the stages from the same
kernels), so it must equal the composed path bit for bit: dt, every state and
the carried rate.  Against the oracle the state bounds are those of
tests/parity.py (relative L1 and per element 1e-12) and dt agrees to 1e-14.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from parity import check_state

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _active(o, x):
    """[nvar][...] view of a state without the ignored hole cells of a refined box."""
    x = np.asarray(x)
    if not isinstance(o, oracle.AmrOracle):
        return x.reshape(o.nvar, -1)
    c, f = o.blocks(x)
    return np.concatenate([c[:, :, ~o.hole].reshape(o.nvar, -1), f.reshape(o.nvar, -1)], axis=1)


def _amr(dim, k, n, lo, hi, **kw):
    h = 1.0 / 8.0
    return workloads.workload("blast_amr", dim=dim, k=k, n=n, length=tuple(h * m for m in n), refine_lo=lo,
                              refine_hi=hi, eps=1e-3, **kw)


CASES = [
    # 2D grids take the fused path (time-step work inside the tile kernel);
    # ragged with respect to the 8x8 and 16-wide tiles
    ("vortex_k2_40x24", dict(name="vortex", n=(40, 24, 1), length=(10.0, 6.0, 1.0)), "fp64"),
    ("vortex_k1_33x17", dict(name="vortex", k=1, n=(33, 17, 1), length=(11.0, 17 / 3, 1.0)), "fp64"),
    ("vortex_k3_20x18", dict(name="vortex", k=3, n=(20, 18, 1), length=(10.0, 9.0, 1.0), noise=0.0), "fp64"),
    ("sod_limited_davis", dict(name="sod", n=(40, 4, 1), length=(1.0, 0.1, 1.0), flux=1, eps=1e-3), "fp64"),
    ("vortex_k2_fp32", dict(name="vortex", n=(40, 24, 1), length=(10.0, 6.0, 1.0)), "fp32"),
    ("vortex_k2_bf16", dict(name="vortex", n=(40, 24, 1), length=(10.0, 6.0, 1.0)), "bf16"),
    # 3D and the refined box: the two-kernel time step
    ("kh3d_k2_limited", dict(name="kh3d", k=2, n=(12, 10, 9), length=(1.2, 1.0, 0.9)), "fp64"),
    # uniform 3D at k = 3 runs the four-lanes-per-cell kernel
    ("kh3d_k3_limited", dict(name="kh3d", k=3, n=(9, 8, 7), length=(0.9, 0.8, 0.7)), "fp64"),
    ("blast_amr_2d_k2", dict(amr=(2, 2, (10, 9, 1), (2, 3, 0), (7, 6, 0))), "fp64"),
    ("blast_amr_3d_k1", dict(amr=(3, 1, (8, 7, 6), (2, 2, 1), (6, 5, 4))), "fp64"),
]


def _setup(spec, precision):
    import paper_1506_06140_amd as dg
    spec = dict(spec)
    if "amr" in spec:
        wl = _amr(*spec["amr"])
        o = oracle.AmrOracle(wl)
        w0 = o.initial_state()
        w0, st = o.limit(w0)
        assert st == 0
    else:
        name = spec.pop("name")
        wl = workloads.workload(name, **spec)
        o = oracle.Oracle(wl)
        w0 = o.initial_state()
        if wl["ic"] in ("blast", "sod"):
            w0, st = oracle.Oracle(dict(wl, limiter=1, positivity=1, eps=1e-3)).limit(w0)
            assert st == 0
    return wl, o, dg.Solver(wl, precision=precision), w0


@pytest.mark.parametrize("case,spec,precision", CASES, ids=[c[0] for c in CASES])
def test_step_equals_composed_calls(case, spec, precision):
    _say("case", case, precision)
    wl, o, s, w0 = _setup(spec, precision)
    steps = 3
    # composed: dg_max_dt, then stages and limiters
    bufs = [s.empty() for _ in range(3)] + [s.scalar()]
    w = _dev(w0)
    ref_states, ref_dts = [], []
    for _ in range(steps):
        w = s.step(w, bufs).clone()
        ref_states.append(_active(o, _host(w)))
        ref_dts.append(_host(bufs[3])[0])
    assert s.status() == 0
    # fused: rate carried from step to step
    fb = [s.empty() for _ in range(3)]
    dt, rate = s.scalar(), s.rate_state()
    w = _dev(w0)
    s.max_rate(w, rate)
    for i in range(steps):
        w = s.rk_step(w, fb, dt, rate).clone()
        got = _active(o, _host(w))
        _say(case, "step", i, "dt", _host(dt)[0], ref_dts[i])
        assert _host(dt)[0] == ref_dts[i], (i, _host(dt)[0], ref_dts[i])
        assert np.array_equal(got, ref_states[i]), (i, np.abs(got - ref_states[i]).max())
        fresh = s.rate_value(s.max_rate(w))
        assert s.rate_value(rate) == fresh, (i, s.rate_value(rate), fresh)
    assert s.status() == 0


@pytest.mark.parametrize("case,spec,precision", [CASES[0], CASES[3], CASES[6], CASES[7], CASES[8]],
                         ids=[CASES[i][0] for i in (0, 3, 6, 7, 8)])
def test_step_matches_oracle(case, spec, precision):
    _say("case", case)
    wl, o, s, w0 = _setup(spec, precision)
    fb = [s.empty() for _ in range(3)]
    dt, rate = s.scalar(), s.rate_state()
    w = _dev(w0)
    s.max_rate(w, rate)
    ref = w0
    for i in range(3):
        ref, dt_ref = o.step(ref)
        w = s.rk_step(w, fb, dt, rate).clone()
        assert _host(dt)[0] == pytest.approx(dt_ref, rel=1e-14)
        check_state(o, _host(w), ref, f"{case} step {i}")
    # the carried rate gives the oracle's next time step
    dt_next = o.max_dt(ref)
    s.rk_step(w, fb, dt, rate)
    assert _host(dt)[0] == pytest.approx(dt_next, rel=1e-14)
    assert s.status() == 0


GRAPH_CASES = [
    ("vortex", dict(name="vortex", n=(48, 40, 1), length=(12.0, 10.0, 1.0))),
    # limiters with many cells in the positivity point-loop pass (its list
    # count is cleared by a kernel inside the graph) on the refined box
    ("blast_box_k3", dict(name="blast_amr", k=3, n=(8, 8, 8), length=(1.0, 1.0, 1.0), refine_lo=(2, 2, 2),
                          refine_hi=(6, 6, 6), eps=1e-3)),
]


@pytest.mark.parametrize("case,spec", GRAPH_CASES, ids=[c[0] for c in GRAPH_CASES])
def test_step_graph_replays(case, spec):
    # two chained steps captured into a graph (ping-pong A -> B -> A) and
    # replayed three times, with eager work and synchronisation in between;
    # every replay equals the eager chain bit for bit
    import torch
    spec = dict(spec)
    wl = workloads.workload(spec.pop("name"), **spec)
    o = oracle.make(wl)
    s = __import__("paper_1506_06140_amd").Solver(wl)
    w0 = o.initial_state()
    if wl["limiter"] or wl["positivity"]:
        w0, st = o.limit(w0)
        assert st == 0
    # eager reference: 8 steps
    fb = [s.empty() for _ in range(3)]
    dt, rate = s.scalar(), s.rate_state()
    w = _dev(w0)
    s.max_rate(w, rate)
    eager = []
    for _ in range(8):
        w = s.rk_step(w, fb, dt, rate).clone()
        eager.append(_host(w))
    A, B = _dev(w0), s.empty()
    u1, u2 = s.empty(), s.empty()
    dtb, rb = s.scalar(), s.rate_state()

    def two():
        s.rk_step(A, [u1, u2, B], dtb, rb)
        s.rk_step(B, [u1, u2, A], dtb, rb)

    s.max_rate(A, rb)
    two()  # warm-up on the capture stream's pattern: steps 1, 2
    torch.cuda.synchronize()
    assert np.array_equal(_host(A), eager[1])
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    A_saved, r_saved = A.clone(), rb.clone()
    with torch.cuda.stream(side):
        two()  # steps 3, 4 eagerly on the side stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert np.array_equal(_host(A), eager[3])
    # restore the state after step 2 and capture (capture does not execute)
    A.copy_(A_saved)
    rb.copy_(r_saved)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        two()
    torch.cuda.synchronize()
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = _host(A)
        _say("replay", r, "max diff", np.abs(got - eager[3 + 2 * r]).max())
        assert np.array_equal(got, eager[3 + 2 * r]), r
        x = _dev(np.ones(16)) * 2.0  # eager work between replays
        torch.cuda.synchronize()
        assert float(x.sum()) == 32.0
    assert s.status() == 0


def test_step_argument_errors():
    import torch
    import paper_1506_06140_amd as dg
    wl = workloads.workload("vortex", n=(16, 16, 1), length=(4.0, 4.0, 1.0))
    s = dg.Solver(wl)
    a, b, c, d = (s.empty() for _ in range(4))
    dt, rate = s.scalar(), s.rate_state()
    with pytest.raises(dg.DGError) as e:
        s.rk_step(a, [b, b, c], dt, rate)  # u1 == u2
    assert e.value.code == dg.DG_EINVAL
    with pytest.raises(dg.DGError) as e:
        s.rk_step(a, [b, c, a], dt, rate)  # out == w
    assert e.value.code == dg.DG_EINVAL
    # dt inside the rate state: rejected before anything is launched
    st = s.lib.dg_rk_step(s.ctx, a.data_ptr(), b.data_ptr(), c.data_ptr(), d.data_ptr(), rate.data_ptr() + 8 * 5,
                          rate.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == dg.DG_EINVAL
    with pytest.raises(ValueError):  # a one-element rate buffer is too small
        s.rk_step(a, [b, c, d], dt, s.scalar())
