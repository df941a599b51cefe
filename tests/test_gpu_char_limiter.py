"""GPU: the characteristic TVB limiter (Sec. 3.2 eq. char_limiter, App. E)
against the FP64 oracle.

The kernel applies the eigenvector matrices in factored form and the oracle
as dense matrices, so the two round differently (about 1e-16 relative); the
state bounds are those of tests/parity.py (relative L1 and per element 1e-12),
and which cells are limited (an integer decision) must agree exactly on
states without near-ties.  The shock tube of Sec. 5.2 is run to the end on
the GPU with each limiter and checked against the oracle's run and the
paper's comparison."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from parity import check_state, rel_l1
from test_gpu_amr import _per_var, _wl, rough_amr_state
from test_gpu_parity import _rough
from test_oracle_limiters import _exact_riemann

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _touched(w, x, nvar):
    """Cells whose modes differ between w and x."""
    return (np.asarray(x).reshape(nvar, w.shape[1], -1) != w.reshape(nvar, w.shape[1], -1)).any(axis=(0, 1))


# amplitude 0.03 of the higher modes leaves 10-60 % of the cells limited (a
# mix, so that the decision is tested both ways), 0.4 limits every cell
@pytest.mark.parametrize("amp", [0.03, 0.4])
@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3)])
def test_char_limiter_matches_oracle(dim, k, amp):
    import paper_1506_06140_amd as dg
    n = (9, 7, 5) if dim == 3 else (13, 11, 1)
    h = 0.1
    wl = workloads.workload("kh3d", dim=dim, k=k, n=n, length=tuple(h * m for m in n), limiter=2, positivity=1)
    _say("char limiter", dim, k, "amp", amp)
    o = oracle.Oracle(wl)
    s = dg.Solver(wl)
    w = _rough(o, seed=100 + dim * 10 + k, amp=amp)
    ref, st = o.limit(w)
    assert st == 0
    d = _dev(w)
    s.limit(d)
    got = _host(d)
    assert np.array_equal(got[:, 0], w[:, 0])  # means untouched, bitwise
    t_ref, t_got = _touched(w, ref, o.nvar), _touched(w, got, o.nvar)
    _say("cells changed", int(t_ref.sum()), "of", t_ref.size)
    if amp < 0.1:
        assert 0 < t_ref.sum() < t_ref.size
    assert np.array_equal(t_ref, t_got)
    check_state(o, got, ref, f"char limiter {dim}D k={k}")
    assert s.status() == 0


def test_char_limiter_keeps_smooth_states_and_skips_bad_means():
    import paper_1506_06140_amd as dg
    wl = workloads.workload("kh3d", dim=3, k=2, n=(6, 5, 4), length=(0.6, 0.5, 0.4), limiter=2, positivity=0)
    o = oracle.Oracle(wl)
    s = dg.Solver(wl)
    w = _rough(o, seed=7, amp=1e-6)  # every slope under the TVB bound
    d = _dev(w)
    s.limit(d)
    assert np.array_equal(_host(d), w)
    # a cell with negative mean pressure is left as it is, like the oracle
    bad = _rough(o, seed=8, amp=0.4)
    bad[4, 0, 2, 2, 3] = 0.1 * bad[0, 0, 2, 2, 3]
    ref, _ = o.limit(bad)
    d = _dev(bad)
    s.limit(d)
    got = _host(d)
    assert np.array_equal(got[:, :, 2, 2, 3], bad[:, :, 2, 2, 3])
    check_state(o, got, ref, "char limiter, bad mean")
    assert s.status() == dg.DG_OK  # no positivity pass configured: no flag


AMR_CASES = [
    ("2d_k2", dict(dim=2, k=2, n=(10, 9, 1), lo=(2, 3, 0), hi=(7, 6, 0))),
    ("3d_k1", dict(dim=3, k=1, n=(8, 7, 6), lo=(2, 2, 1), hi=(6, 5, 4))),
    ("3d_k3", dict(dim=3, k=3, n=(8, 8, 8), lo=(2, 2, 2), hi=(6, 6, 6))),
]


@pytest.mark.parametrize("ic", ["blast", "kh3d_rough"])
@pytest.mark.parametrize("case,spec", AMR_CASES, ids=[c[0] for c in AMR_CASES])
def test_char_limiter_on_refined_box(case, spec, ic):
    import paper_1506_06140_amd as dg
    _say("AMR char limiter", case, ic)
    if ic == "blast":
        wl = _wl(**spec, limiter=2)
        o = oracle.AmrOracle(wl)
        w = o.initial_state()  # discontinuous blast projection (3D: many cells limited)
    else:
        wl = _wl(**spec, limiter=2, ic="kh3d")
        o = oracle.AmrOracle(wl)
        w = rough_amr_state(o, seed=31 + spec["dim"] * 4 + spec["k"])
    s = dg.Solver(wl)
    ref, st = o.limit(w)
    assert st == 0
    d = _dev(w)
    s.limit(d)
    got = _host(d)
    _say(case, ic, "modes changed", int((_per_var(o, ref) != _per_var(o, w)).sum()))
    check_state(o, got, ref, f"{case} {ic} AMR char limiter")
    assert s.status() == 0


STEP_CASES = [
    ("sod_k2", dict(name="sod", n=(40, 4, 1), length=(1.0, 0.1, 1.0), limiter=2, eps=1e-3)),
    ("kh3d_k2", dict(name="kh3d", k=2, n=(12, 10, 9), length=(1.2, 1.0, 0.9), limiter=2)),
    ("amr_3d_k2", dict(amr=dict(dim=3, k=2, n=(8, 7, 6), lo=(2, 2, 1), hi=(6, 5, 4), limiter=2))),
]


@pytest.mark.parametrize("case,spec", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_char_limited_steps_match_oracle(case, spec):
    # three SSP-RK3 steps, limiters after every stage, through the one-call step
    import paper_1506_06140_amd as dg
    spec = dict(spec)
    _say("char limited steps", case)
    if "amr" in spec:
        wl = _wl(**spec["amr"])
        o = oracle.AmrOracle(wl)
    else:
        wl = workloads.workload(spec.pop("name"), **spec)
        o = oracle.Oracle(wl)
    s = dg.Solver(wl)
    w0, st = o.limit(o.initial_state())
    assert st == 0
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
    assert s.status() == 0


def _gpu_sod(limiter, nx=64):
    import paper_1506_06140_amd as dg
    wl = workloads.workload("sod", n=(nx, 2, 1), length=(1.0, 2.0 / nx, 1.0), limiter=limiter)
    o = oracle.Oracle(wl)
    s = dg.Solver(wl)
    w0, st = o.limit(o.initial_state())
    assert st == 0
    bufs = [s.empty() for _ in range(3)] + [s.scalar()]
    w = _dev(w0)
    dt = s.scalar()
    t, t_end, steps = 0.0, wl["t_end"], 0
    while t < t_end - 1e-14:
        s.max_dt(w, dt)
        h = float(_host(dt)[0])
        if t + h > t_end:
            h = t_end - t
            dt.fill_(h)
        w = s.step(w, bufs, dt).clone()
        t += h
        steps += 1
    assert s.status() == 0
    return o, _host(w), t, steps


@pytest.mark.slow
def test_sod_limiter_comparison_on_gpu():
    # DG-3, 64 cells, t = 0.228: every limiter's GPU run against the oracle's
    # run, then the comparison of Sec. 5.2 on the GPU results
    res = {}
    for lim in (0, 1, 2):
        res[lim] = _gpu_sod(lim)
    stats = {}
    for lim, (o, w, t, steps) in res.items():
        ref = _oracle_sod(o)
        err = rel_l1(o, w, ref)
        rho = w[0, 0, 0].mean(axis=0)
        nx = rho.size
        xs = (np.arange(nx * 64) + 0.5) / (nx * 64)
        ex, _ = _exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4, (xs - 0.5) / t)
        ex = ex.reshape(nx, 64).mean(axis=1)
        stats[lim] = dict(l1=np.abs(rho - ex).mean(), tv=np.abs(np.diff(rho)).sum(), lo=rho.min(), hi=rho.max())
        _say("limiter", lim, steps, "steps, rel-L1 vs oracle run", err, stats[lim])
        assert np.all(err <= 1e-10), err
    none, comp, char = stats[0], stats[1], stats[2]
    assert none["l1"] < char["l1"] < 0.5 * comp["l1"]
    assert none["hi"] > 1.0 + 1e-3
    assert char["tv"] < (1.0 - 0.125) * 1.01 < comp["tv"]


def _sod_start(o):
    w, st = o.limit(o.initial_state())
    assert st == 0
    return (w,)


def _oracle_sod(o):
    (w,) = _sod_start(o)
    t, t_end = 0.0, o.wl["t_end"]
    while t < t_end - 1e-14:
        dt = min(o.max_dt(w), t_end - t)
        w, _ = o.step(w, dt)
        t += dt
    return w
