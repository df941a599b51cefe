"""GPU parity on the static 2:1 refined box (hanging faces, AMR limiting)
against the FP64 oracle; comparison rules of tests/parity.py (states: relative
L1 and per-element bounds of 1e-12; the RHS against fac(|V| + |S|))."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from parity import check_rhs, check_state

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _per_var(o, x):
    """Flat AMR state -> [nvar][...] (both blocks, hole cells removed)."""
    c, f = o.blocks(x)
    return np.concatenate([c[:, :, ~o.hole].reshape(o.nvar, -1), f.reshape(o.nvar, -1)], axis=1)


def _wl(dim, k, n, lo, hi, **kw):
    h = 1.0 / 8.0
    base = dict(limiter=1, positivity=1, ic="blast")
    base.update(kw)
    if base["ic"] == "kh3d":
        # shear layer: density and velocity jumps at y = 1/4 and 3/4 (on
        # hanging faces of the boxes below) plus cell-wise velocity noise,
        # so that the two traces differ on every hanging face
        base.setdefault("noise", 1e-2)
        base.setdefault("seed", 6140)
    return workloads.workload("blast_amr", dim=dim, k=k, n=n, length=tuple(h * m for m in n),
                              refine_lo=lo, refine_hi=hi, **base)


CASES = [
    ("2d_k2", dict(dim=2, k=2, n=(10, 9, 1), lo=(2, 3, 0), hi=(7, 6, 0))),
    ("3d_k1", dict(dim=3, k=1, n=(8, 7, 6), lo=(2, 2, 1), hi=(6, 5, 4))),
    ("3d_k2", dict(dim=3, k=2, n=(8, 7, 6), lo=(2, 2, 1), hi=(6, 5, 4))),
    ("3d_k3", dict(dim=3, k=3, n=(8, 8, 8), lo=(2, 2, 2), hi=(6, 6, 6))),
]
# right-hand side cases: every box with the shear layer (jumps across hanging
# faces), the 3D boxes with the blast, and both HLLC wave-speed bounds
RHS_CASES = ([(c + "_kh", dict(s, ic="kh3d")) for c, s in CASES]
             + [(c + "_blast", s) for c, s in CASES if s["dim"] == 3]
             + [("3d_k2_kh_davis", dict(CASES[2][1], ic="kh3d", flux=1)),
                ("2d_k2_kh_davis", dict(CASES[0][1], ic="kh3d", flux=1)),
                # 3D FP64 runs the MFMA kernel by default; the vector-ALU
                # kernels (path3d = DG_PATH3D_VALU) on the same boxes
                ("3d_k2_kh_valu", dict(CASES[2][1], ic="kh3d", path3d=1)),
                ("3d_k3_kh_valu", dict(CASES[3][1], ic="kh3d", path3d=1)),
                ("3d_k3_blast_valu", dict(CASES[3][1], path3d=1)),
                # a box touching the periodic wrap of the base grid's x axis
                # and a box one cell wide along z
                ("3d_k3_kh_edges", dict(dim=3, k=3, n=(8, 7, 6), lo=(1, 2, 2), hi=(7, 5, 3), ic="kh3d"))])


def rough_amr_state(o, seed, amp=0.02):
    """The projected initial state plus seeded random higher modes in both
    blocks: a mix of limited and untouched cells on either side of the
    refinement boundary."""
    rng = np.random.default_rng(seed)
    w = o.initial_state()
    for b in o.blocks(w):  # views into w
        b[:, 1:] += amp * rng.uniform(-1, 1, size=b[:, 1:].shape)
    return w


def _limited_state(o):
    w = o.initial_state()
    lim = oracle.AmrOracle(dict(o.wl, eps=1e-3))
    w, st = lim.limit(w)
    assert st == 0
    return w


@pytest.mark.parametrize("case,spec", RHS_CASES, ids=[c[0] for c in RHS_CASES])
def test_amr_rhs_stage_dt_match_oracle(case, spec):
    import paper_1506_06140_amd as dg
    wl = _wl(**spec)
    o = oracle.AmrOracle(wl)
    s = dg.Solver(wl)
    assert s.amr and s.ncoarse == o.ncoarse and s.nfine == o.nfine
    w = _limited_state(o)
    d = _dev(w)
    V, S, A = o.terms_cells(w, with_abs=True)
    L = _host(s.rhs(d))
    check_rhs(o, L, V, S, A, f"{case} AMR rhs")
    dt = o.max_dt(w)
    dtd = s.max_dt(d)
    assert float(_host(dtd)[0]) == pytest.approx(dt, rel=1e-14)
    ref = o.rk3_stage(1, dt, w, w)
    got = _host(s.rk_stage(1, dtd, None, d))
    check_state(o, got, ref, f"{case} AMR stage-1")
    # conservation of the GPU right-hand side across the interface
    Lc, Lf = o.blocks(L)
    tot = Lc[:, 0, ~o.hole].sum(axis=1) * o.dx ** o.dim + Lf[:, 0, :].sum(axis=1) * o.dxf ** o.dim
    scale = np.abs(Lc[:, 0, ~o.hole]).sum(axis=1) * o.dx ** o.dim + np.abs(Lf[:, 0, :]).sum(axis=1) * o.dxf ** o.dim
    assert np.all(np.abs(tot) <= 1e-13 * scale)
    assert s.status() == 0


@pytest.mark.parametrize("ic", ["blast", "kh3d_rough"])
@pytest.mark.parametrize("case,spec", CASES, ids=[c[0] for c in CASES])
def test_amr_limiter_matches_oracle(case, spec, ic):
    import paper_1506_06140_amd as dg
    if ic == "blast":
        wl = _wl(**spec)
        o = oracle.AmrOracle(wl)
        w = o.initial_state()  # discontinuous blast projection (3D: many cells limited)
    else:
        wl = _wl(**spec, ic="kh3d")
        o = oracle.AmrOracle(wl)
        w = rough_amr_state(o, seed=17 + spec["dim"] * 4 + spec["k"])
    s = dg.Solver(wl)
    ref, st = o.limit(w)
    assert st == 0
    d = _dev(w)
    s.limit(d)
    got = _host(d)
    _say(case, "cells changed by the limiter", int((np.abs(_per_var(o, ref) - _per_var(o, w)) > 0).any(axis=0).sum()))
    check_state(o, got, ref, f"{case} AMR limiter")
    assert s.status() == 0


@pytest.mark.parametrize("case,spec", [
    ("3d_k3_blast", dict(dim=3, k=3, n=(8, 8, 8), lo=(2, 2, 2), hi=(6, 6, 6))),
    ("3d_k2_kh", dict(dim=3, k=2, n=(8, 7, 6), lo=(2, 2, 1), hi=(6, 5, 4), ic="kh3d")),
], ids=["3d_k3_blast", "3d_k2_kh"])
def test_amr_limited_steps_match_oracle(case, spec):
    # limit the initial state, then two full limited SSP-RK3 steps
    import paper_1506_06140_amd as dg
    wl = _wl(**spec)
    o = oracle.AmrOracle(wl)
    s = dg.Solver(wl)
    w0, st = o.limit(o.initial_state())
    assert st == 0
    ref, _ = o.run(w0, 2)
    bufs = [s.empty() for _ in range(3)] + [s.scalar()]
    w = _dev(w0)
    for _ in range(2):
        w = s.step(w, bufs).clone()
    check_state(o, _host(w), ref, f"{case} AMR 2 limited steps")
    np.testing.assert_allclose(o.totals(_host(w)), o.totals(w0), rtol=1e-12, atol=1e-14)


def test_amr_projection_matches_oracle():
    import paper_1506_06140_amd as dg
    wl = _wl(dim=3, k=2, n=(8, 7, 6), lo=(2, 2, 1), hi=(6, 5, 4))
    o = oracle.AmrOracle(wl)
    s = dg.Solver(wl)
    x = o.node_coords()
    nct = o.ncoarse + o.nfine
    cell = np.repeat(np.arange(nct), o.Q).reshape(nct, o.Q)
    node = np.tile(np.arange(o.Q), nct).reshape(nct, o.Q)
    wlq = dict(wl); wlq["nq"] = o.Q
    prim = np.stack(workloads.primitives(wlq, x[..., 0], x[..., 1], x[..., 2], cell=cell, node=node), axis=-1)
    import oracle as _o
    lib, _ = _o._load()
    import ctypes as C
    ref = np.zeros(o.size)
    assert lib.orc_amr_project(C.byref(o.c), np.ascontiguousarray(prim), ref) == 0
    got = _host(s.project(_dev(np.transpose(prim, (2, 1, 0)))))
    check_state(o, got, ref, "AMR projection", tol=1e-14)
    # the library's own node coordinates agree with the oracle's
    xs = s.node_coords()
    np.testing.assert_allclose(np.transpose(xs, (2, 1, 0)), x, atol=1e-15)
