"""Pins of the oracle's adaptive refinement on the one-box mesh: the
refinement criterion (Sec. 4.1, eqs. cell_ref and node_ref), refinement and
derefinement by L2 projection (Sec. 4.2 eq. ref_weights, Sec. 4.3 eq.
deref_weights) and the box around the flagged cells with one buffer layer
(Sec. 4), against what the paper states and the mathematics fixes:
refine-then-derefine is the identity (the text's P_A P_A^T = I; what holds,
and is pinned in test_oracle_amr, is 2^-d sum_c P_c^T P_c = I), projections
keep the conserved totals, a linear density is flagged exactly where its
slope coefficient passes the thresholds, with the alpha hysteresis band."""
import math

import numpy as np
import pytest

import oracle
import workloads


def _kh(n=26, k=2, **kw):
    return workloads.workload("kh2d", n=(n, n, 1), k=k, **kw)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_refine_then_derefine_restores_and_conserves(k):
    wl = _kh(k=k)
    o = oracle.make(wl)
    w, _ = o.limit(o.initial_state())
    box = ((3, 4, 0), (20, 17, 0))
    wlb = dict(wl, refine_lo=box[0], refine_hi=box[1])
    wb = oracle.regrid(wl, w, wlb)
    ob = oracle.make(wlb)
    np.testing.assert_allclose(ob.totals(wb), o.totals(w), rtol=0, atol=1e-14 * np.abs(o.totals(w)).max())
    back = oracle.regrid(wlb, wb, wl)
    np.testing.assert_allclose(back, w, rtol=0, atol=1e-14 * np.abs(w).max())


def test_moving_box_conserves_and_keeps_the_overlap():
    wl = _kh()
    o = oracle.make(wl)
    w, _ = o.limit(o.initial_state())
    A = dict(wl, refine_lo=(2, 4, 0), refine_hi=(14, 20, 0))
    B = dict(wl, refine_lo=(8, 2, 0), refine_hi=(24, 12, 0))
    wa = oracle.regrid(wl, w, A)
    wb = oracle.regrid(A, wa, B)
    oa, ob = oracle.make(A), oracle.make(B)
    scale = np.abs(o.totals(w)).max()
    np.testing.assert_allclose(ob.totals(wb), oa.totals(wa), rtol=0, atol=1e-14 * scale)
    # children of base cells refined in both boxes are carried over bit for bit
    ca, fa = oa.blocks(wa)
    cb, fb = ob.blocks(wb)
    fa = fa.reshape(oa.nvar, oa.N, oa.nf[1], oa.nf[0])
    fb = fb.reshape(ob.nvar, ob.N, ob.nf[1], ob.nf[0])
    # overlap of the boxes: base cells x 8..13, y 4..11
    sa = fa[:, :, 2 * (4 - 4):2 * (12 - 4), 2 * (8 - 2):2 * (14 - 2)]
    sb = fb[:, :, 2 * (4 - 2):2 * (12 - 2), 2 * (8 - 8):2 * (14 - 8)]
    assert np.array_equal(sa, sb)


def _linear_density(wl, slope):
    """Uniform-pressure state at rest with rho = 1 + slope (x - 1/2), exactly."""
    o = oracle.make(wl)
    w = np.zeros(o.shape)
    if isinstance(o, oracle.AmrOracle):
        raise AssertionError("build on the base grid")
    h = o.dx
    xc = (np.arange(wl["n"][0]) + 0.5) * h
    w[0, 0] = 1.0 + slope * (xc[None, None, :] - 0.5)
    w[0, 1] = slope * h / 2 / math.sqrt(3.0)   # mode 1 is sqrt(3) xi, xi = 2 (x - xc) / h
    w[3, 0] = 2.5 / 0.4
    return w


@pytest.mark.parametrize("factor,cell_flag,node_flag", [
    (1.2, True, True),     # above alpha w_t: refine, and keep refined
    (1.0, False, True),    # inside the band (w_t/alpha, alpha w_t): no change either way
    (0.85, False, False),  # below w_t/alpha: derefine
])
def test_flags_of_a_linear_density(factor, cell_flag, node_flag):
    wt, alpha = 0.01, 1.1
    wl = _kh(n=20, k=1)
    h = 1.0 / 20
    slope = factor * wt * math.sqrt(3.0) * 2 / h  # slope coefficient = factor * w_t
    w = _linear_density(wl, slope)
    f = oracle.amr_flags(wl, w, wt, alpha)
    assert np.all(f == cell_flag)
    wlb = dict(wl, refine_lo=(2, 3, 0), refine_hi=(9, 12, 0))
    wb = oracle.regrid(wl, w, wlb)  # exact for a linear density
    fb = oracle.amr_flags(wlb, wb, wt, alpha).reshape(20, 20)
    hole = np.zeros((20, 20), dtype=bool)
    hole[3:12, 2:9] = True
    assert np.all(fb[hole] == node_flag)
    assert np.all(fb[~hole] == cell_flag)


def test_box_from_flags_adds_one_layer_and_stays_inside():
    wl = _kh(n=20, k=1)
    f = np.zeros((20, 20), dtype=np.int32)
    f[5, 7] = 1
    f[9, 12] = 1
    assert oracle.box_from_flags(wl, f) == ((6, 4, 0), (14, 11, 0))
    f[0, 19] = 1  # at the edges the box stops at 1 and n - 1
    assert oracle.box_from_flags(wl, f) == ((6, 1, 0), (19, 11, 0))
    assert oracle.box_from_flags(wl, np.zeros((20, 20))) is None


def test_adaptive_kh_steps_stay_conservative():
    # a few steps of KH with the box following the flags every step
    wl = _kh(n=26, k=2)
    o = oracle.make(wl)
    w, _ = o.limit(o.initial_state())
    tot0 = o.totals(w)
    cur = wl
    for _ in range(3):
        box = oracle.box_from_flags(cur, oracle.amr_flags(cur, w, wl["wt"], wl["alpha"]))
        new = dict(wl, refine_lo=box[0], refine_hi=box[1]) if box else dict(wl, refine_lo=(0, 0, 0),
                                                                            refine_hi=(0, 0, 0))
        w = oracle.regrid(cur, w, new)
        cur = new
        oc = oracle.make(cur)
        w, _ = oc.step(w)
    np.testing.assert_allclose(oc.totals(w)[[0, 3]], tot0[[0, 3]], rtol=1e-13)
    assert np.isfinite(w).all()
