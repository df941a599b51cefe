"""The comparison rules of the GPU parity tests (HIP path against the FP64
oracle on the same seeded inputs).

States (after a stage, a step, a trajectory, the limiters), per conserved
variable v, both of:
  * relative L1: sum |w_gpu - w_orc| / sum |w_orc| over all modes and cells
    <= tol;
  * per element: |w_gpu - w_orc| <= tol * max(|w_orc|, s_v), with s_v the mean
    |mode 0| of variable v (a higher mode is compared against the size of its
    variable, not against itself: a slope that is zero in exact arithmetic
    still carries rounding of the order of the mean).
A state produced by one Runge-Kutta stage from inputs checked on the same
cells may instead be held per element to its propagated rounding scale
(stage_scale) where that is larger.
A variable whose oracle norm is below 1e-10 of the largest variable's norm
vanishes in exact arithmetic (the normal momenta of a one-dimensional shock
tube, the transverse momentum of a planar shear): its rounding noise has no
scale of its own, so both bounds use the largest variable's norm and mean
instead.  No other floor is applied.

The right-hand side L = fac (V - S) alone, per variable:
  * sum |L_gpu - L_orc| <= tol * sum (|V| + |S|): L is a difference of the
    volume and face integrals, nearly equal in smooth flow, so its rounding
    scales with |V| + |S|, not with |L|;
  * per element, |L_gpu - L_orc| <= tol * max(A, mean_v A), with A = fac
    times the sum of the magnitudes of every summand of V and S (the
    oracle's with_abs output) and mean_v A its mean over the variable's
    elements.  A single element of V or S can itself be a near-cancelling
    sum (a mode that is odd in a symmetric state, or a constant state whose
    flux integrates to zero against a gradient), so its rounding scale is
    the magnitude of its summands, as in the standard bound on a computed
    sum, not |V| + |S|.  The summands are themselves computed fluxes: a flux
    that is exactly zero in the oracle (the mass flux through gas at rest)
    is a cancelling expression (the HLLC star-state correction) that rounds
    to a few ulps of the variable's typical flux in another evaluation order,
    so an element's scale is never taken below the variable's mean A, as a
    state element's is never taken below the variable's mean |mode 0|;
  * relative L1 of L itself, sum |dL| / sum |L|, is printed and asserted
    <= tol for every variable whose conditioning sum(|V| + |S|) / sum |L| is at
    most 10 (no near-cancellation between the two integrals).
"""
from __future__ import annotations

import sys

import numpy as np

import oracle

TOL = 1e-12
VANISH = 1e-10
COND_MAX = 10.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def modes(o, x):
    """[nvar][N][cells] view of a state of `o`'s grid (a refined box: both
    blocks, the ignored hole cells of the coarse block removed)."""
    x = np.asarray(x)
    if isinstance(o, oracle.AmrOracle):
        c, f = o.blocks(x)
        return np.concatenate([c[:, :, ~o.hole], f], axis=2)
    return x.reshape(o.nvar, o.N, -1)


def _scales(ref):
    """Per-variable (L1 norm, mean |mode 0|), vanishing variables lifted to the
    largest variable's values."""
    norm = np.abs(ref).reshape(ref.shape[0], -1).sum(axis=1)
    mean0 = np.abs(ref[:, 0]).reshape(ref.shape[0], -1).mean(axis=1)
    vanish = norm < VANISH * norm.max()
    norm = np.where(vanish, norm.max(), norm)
    mean0 = np.where(vanish, mean0.max(), mean0)
    return norm, mean0


def state_errors(o, got, ref):
    """(relative L1, largest per-element ratio) per variable."""
    g, r = modes(o, got), modes(o, ref)
    return state_errors_modes(g, r)


def state_errors_modes(g, r, scale=None):
    """The same for arrays already shaped [nvar][N][cells]; `scale` (same
    shape, optional) is a per-element rounding scale propagated from the
    inputs of the operation that produced r (see stage_scale)."""
    g = np.asarray(g, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    nv = r.shape[0]
    norm, mean0 = _scales(r)
    d = np.abs(g - r).reshape(nv, -1)
    rel = d.sum(axis=1) / norm
    bound = np.maximum(np.abs(r).reshape(nv, -1), mean0[:, None])
    if scale is not None:
        bound = np.maximum(bound, np.asarray(scale).reshape(nv, -1))
    elem = (d / bound).max(axis=1)
    return rel, elem


def stage_scale(a, b, dt, wn, wp, A):
    """Per-element rounding scale of a Runge-Kutta stage u = a wn + b (wp +
    dt L) (a = 0 for the first stage): |a wn| + |b| (|wp| + dt max(A, mean_v
    A)), with A the right-hand side's summand scale of the rule above.  A
    field that the stage creates from zero (the momentum of gas starting at
    rest) has a mean over the mesh far below its values where it is not
    zero; its elements are measured against what produced them."""
    nv = A.shape[0]
    A = np.asarray(A).reshape(nv, -1)
    As = np.maximum(A, A.mean(axis=1, keepdims=True)).reshape(np.shape(wp))
    return np.abs(a * np.asarray(wn)) + abs(b) * (np.abs(wp) + dt * As)


def check_state(o, got, ref, what="", tol=TOL):
    rel, elem = state_errors(o, got, ref)
    say(what, "rel-L1", rel, "max per-element", elem)
    assert np.all(rel <= tol), (what, "rel-L1", rel)
    assert np.all(elem <= tol), (what, "per-element", elem)
    return rel, elem


def check_state_modes(g, r, what="", tol=TOL, scale=None):
    rel, elem = state_errors_modes(g, r, scale)
    say(what, "rel-L1", rel, "max per-element", elem)
    assert np.all(rel <= tol), (what, "rel-L1", rel)
    assert np.all(elem <= tol), (what, "per-element", elem)
    return rel, elem


def rhs_errors_modes(L, V, S, A):
    """(sum-bound ratio, largest per-element ratio, relative L1 of L,
    conditioning sum(|V|+|S|)/sum|L|) per variable, arrays [nvar][...]."""
    nv = V.shape[0]
    L = np.asarray(L).reshape(nv, -1)
    V = np.asarray(V).reshape(nv, -1)
    S = np.asarray(S).reshape(nv, -1)
    A = np.asarray(A).reshape(nv, -1)
    ref = V - S
    d = np.abs(L - ref)
    a = np.abs(V) + np.abs(S)
    asum = a.sum(axis=1)
    lsum = np.abs(ref).sum(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        elem = (d / np.maximum(A, A.mean(axis=1, keepdims=True))).max(axis=1)
        rell = d.sum(axis=1) / lsum
        cond = asum / lsum
    return d.sum(axis=1) / asum, elem, rell, cond


def check_rhs(o, L, V, S, A, what="", tol=TOL):
    """L from the GPU; (V, S, A) from the oracle's terms_cells(with_abs=True)."""
    return check_rhs_modes(modes(o, L), modes(o, V), modes(o, S), modes(o, A), what, tol)


def check_rhs_modes(L, V, S, A, what="", tol=TOL):
    err, elem, rell, cond = rhs_errors_modes(L, V, S, A)
    say(what, "rhs error / (|V|+|S|)", err, "max per-element", elem, "rel-L1 of L", rell, "conditioning", cond)
    assert np.all(err <= tol), (what, "rhs L1", err)
    assert np.all(elem <= tol), (what, "rhs per-element", elem)
    wellcond = cond <= COND_MAX
    assert np.all(rell[wellcond] <= tol), (what, "rel-L1 of L", rell, cond)
    return err, elem, rell


def rel_l1(o, got, ref):
    """Relative L1 per variable alone (the mixed-precision bounds, stated as
    relative L1 after a number of steps)."""
    return state_errors(o, got, ref)[0]
