"""GPU: adaptive refinement of the one-box mesh (Sec. 4.1-4.3) through
dg_amr_flags and dg_amr_regrid, against the FP64 oracle: the flags are an
integer decision and must agree exactly (seeded states, no ties); moved
states to relative L1 <= 1e-12 per variable; the totals are kept to
rounding; and a short adaptive KH run follows the oracle's boxes and states."""
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


def _kh(k, n=26):
    return workloads.workload("kh2d", n=(n, n, 1), k=k)


def _blast3d(k):
    h = 1.0 / 8.0
    n = (8, 8, 8)
    return workloads.workload("blast_amr", dim=3, k=k, n=n, length=tuple(h * m for m in n), refine_lo=(0, 0, 0),
                              refine_hi=(0, 0, 0))


def _with_box(wl, box):
    return dict(wl, refine_lo=box[0], refine_hi=box[1]) if box else dict(wl, refine_lo=(0, 0, 0),
                                                                         refine_hi=(0, 0, 0))


CASES = [("kh_k1", _kh, 1), ("kh_k2", _kh, 2), ("kh_k3", _kh, 3), ("blast3d_k1", _blast3d, 1),
         ("blast3d_k2", _blast3d, 2)]


@pytest.mark.parametrize("case,make,k", CASES, ids=[c[0] for c in CASES])
def test_flags_and_regrid_match_oracle(case, make, k):
    import paper_1506_06140_amd as dg
    _say("adapt", case)
    wl = make(k)
    o = oracle.make(wl)
    w, st = o.limit(o.initial_state())
    assert st == 0
    s = dg.Solver(wl)
    d = _dev(w)
    # flags on the base grid
    ref = oracle.amr_flags(wl, w)
    flags, gbox = s.amr_flags(d)
    got = _host(flags)
    _say(case, "flagged", int(ref.sum()), "of", ref.size)
    assert 0 < ref.sum() < ref.size
    assert np.array_equal(got, ref)
    box = oracle.box_from_flags(wl, ref)
    assert gbox == box
    # refine into the box
    wlb = _with_box(wl, box)
    refw = oracle.regrid(wl, w, wlb)
    sb, db = s.regrid(d, box)
    ob = oracle.make(wlb)
    check_state(ob, _host(db), refw, f"{case} refine")
    np.testing.assert_allclose(ob.totals(_host(db)), o.totals(w), rtol=0, atol=1e-14 * np.abs(o.totals(w)).max())
    # flags on the boxed mesh (node weights inside the box)
    refb = oracle.amr_flags(wlb, refw)
    fb, _ = sb.amr_flags(db)
    assert np.array_equal(_host(fb), refb)
    # move the box by one cell along x (part refined, part derefined), then back to no box
    lo, hi = box
    moved = ((min(lo[0] + 1, hi[0] - 1),) + tuple(lo[1:]), tuple(hi))
    wlm = _with_box(wl, moved)
    refm = oracle.regrid(wlb, refw, wlm)
    sm, dm = sb.regrid(db, moved)
    check_state(oracle.make(wlm), _host(dm), refm, f"{case} move")
    s0, d0 = sm.regrid(dm, None)
    ref0 = oracle.regrid(wlm, refm, wl)
    check_state(o, _host(d0), ref0, f"{case} derefine")
    np.testing.assert_allclose(o.totals(_host(d0)), o.totals(w), rtol=0, atol=1e-14 * np.abs(o.totals(w)).max())
    assert s0.status() == 0


def test_regrid_argument_errors():
    import paper_1506_06140_amd as dg
    a = dg.Solver(_kh(2))
    b = dg.Solver(_kh(2, n=24))
    wa, wb = a.empty(), b.empty()
    assert a.lib.dg_amr_regrid(a.ctx, wa.data_ptr(), b.ctx, wb.data_ptr(), None) == dg.DG_EINVAL
    assert a.lib.dg_amr_regrid(a.ctx, wa.data_ptr(), a.ctx, wa.data_ptr(), None) == dg.DG_EINVAL
    flags, box = a.empty(), a.empty()
    assert a.lib.dg_amr_flags(a.ctx, wa.data_ptr(), 0.0, 1.1, flags.data_ptr(), box.data_ptr(), None) == dg.DG_EINVAL
    assert a.lib.dg_amr_flags(a.ctx, wa.data_ptr(), 0.01, 0.9, flags.data_ptr(), box.data_ptr(), None) == dg.DG_EINVAL


def test_adaptive_kh_steps_follow_the_oracle():
    # each step: flags, the box around them with one buffer layer, regrid,
    # then one RK_3 step with the limiters; boxes equal, states to 1e-12
    import paper_1506_06140_amd as dg
    wl = dict(_kh(2), rk="rk3")
    o = oracle.make(wl)
    w0, _ = o.limit(o.initial_state())
    cur, ref = wl, w0
    s, d = dg.Solver(wl), _dev(w0)
    for i in range(4):
        box = oracle.box_from_flags(cur, oracle.amr_flags(cur, ref, wl["wt"], wl["alpha"]))
        new = _with_box(wl, box)
        ref = oracle.regrid(cur, ref, new)
        cur = new
        oc = oracle.make(cur)
        ref, dt_ref = oc.step(ref)
        _, gbox = s.amr_flags(d, wl["wt"], wl["alpha"])
        assert gbox == box, (i, gbox, box)
        s, d = s.regrid(d, gbox)
        bufs = [s.empty() for _ in range(3)]
        dt, rate = s.scalar(), s.rate_state()
        s.max_rate(d, rate)
        d = s.rk_step(d, bufs, dt, rate).clone()
        assert float(_host(dt)[0]) == pytest.approx(dt_ref, rel=1e-14)
        check_state(oc, _host(d), ref, f"adaptive KH step {i} box {box}")
    assert s.status() == 0
