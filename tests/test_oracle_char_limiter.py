"""Pins of the oracle's characteristic limiter (Sec. 3.2, eq. char_limiter,
with the bounded minmod of Sec. 3.3) and of the eigenvector matrices it uses
(App. E), against what the mathematics fixes: L R = I, L A R = diag of the
wave speeds with A the flux Jacobian taken by finite differences of the flux,
and a single acoustic wave, for which the limiter reduces to the scalar minmod
of its amplitude whatever the eigenvector's scaling.  Then the paper's
shock-tube comparison of the limiters (Sec. 5.2 and its figure): no slope
limiter gives the smallest L1 error but over- and undershoots, the
characteristic limiter a far better profile than the component-wise one."""
import math

import numpy as np
import pytest

import oracle
import workloads
from test_oracle_limiters import _exact_riemann

R3 = math.sqrt(3.0)
GAMMA = 1.4


def _oracle(dim, n, **kw):
    h = 1.0 / 3.0
    n = tuple(n) + (1,) * (3 - len(n))
    wl = workloads.workload("density_wave", dim=dim, k=2, n=n, length=tuple(h * m for m in n), gamma=GAMMA, **kw)
    return oracle.Oracle(wl)


def _cons(rho, v, p):
    v = np.asarray(v, dtype=float)
    return np.r_[rho, rho * v, p / (GAMMA - 1) + 0.5 * rho * v @ v]


def _random_states(dim, count, seed):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        rho, p = rng.uniform(0.2, 3.0), rng.uniform(0.1, 4.0)
        v = rng.normal(scale=1.5, size=dim)
        yield rho, v, p


def _fd_jacobian(o, U, axis):
    nv = U.size
    A = np.zeros((nv, nv))
    for j in range(nv):
        h = 1e-6 * max(1.0, abs(U[j]))
        e = np.zeros(nv)
        e[j] = h
        A[:, j] = (o.euler_flux(U + e, axis) - o.euler_flux(U - e, axis)) / (2 * h)
    return A


@pytest.mark.parametrize("dim", [2, 3])
def test_left_and_right_eigenvectors_are_inverse(dim):
    o = _oracle(dim, (3,) * dim)
    for rho, v, p in _random_states(dim, 20, 11 + dim):
        U = _cons(rho, v, p)
        for a in range(dim):
            R, L = o.eigvecs(U, a)
            np.testing.assert_allclose(L @ R, np.eye(o.nvar), atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_eigenvectors_diagonalise_the_flux_jacobian(dim):
    # columns of R: waves v_a - c, v_a, v_a + c, then the shear waves at v_a
    o = _oracle(dim, (3,) * dim)
    for rho, v, p in _random_states(dim, 8, 23 + dim):
        U = _cons(rho, v, p)
        c = math.sqrt(GAMMA * p / rho)
        for a in range(dim):
            R, L = o.eigvecs(U, a)
            lam = np.diag([v[a] - c, v[a], v[a] + c] + [v[a]] * (dim - 1))
            got = L @ _fd_jacobian(o, U, a) @ R
            np.testing.assert_allclose(got, lam, atol=1e-8 * (1 + np.abs(U).max()))


def test_eigenvectors_reject_unphysical_states():
    o = _oracle(2, (3, 3))
    with pytest.raises(RuntimeError):
        o.eigvecs(np.array([1.0, 0.0, 0.0, -1.0]), 0)  # negative pressure
    with pytest.raises(RuntimeError):
        o.eigvecs(np.array([-1.0, 0.0, 0.0, 1.0]), 1)  # negative density


def _minmod(a, b, c):
    if a > 0 and b > 0 and c > 0:
        return min(a, b, c)
    if a < 0 and b < 0 and c < 0:
        return max(a, b, c)
    return 0.0


def _acoustic_eigvec(o, U, axis, sign):
    """Eigenvector of the finite-difference flux Jacobian for v_a + sign c,
    scaled to unit density component (independent of App. E)."""
    lam, vec = np.linalg.eig(_fd_jacobian(o, U, axis))
    rho = U[0]
    v = U[1 + axis] / rho
    p = (GAMMA - 1) * (U[-1] - 0.5 * (U[1:-1] @ U[1:-1]) / rho)
    j = np.argmin(np.abs(lam - (v + sign * math.sqrt(GAMMA * p / rho))))
    r = np.real(vec[:, j])
    return r / r[0]


# amplitude of the slope (sqrt(3) times the mode coefficient) against the
# backward and forward differences of the means, all along one eigenvector
@pytest.mark.parametrize("s,dw,de", [
    (0.30, 0.50, 0.40),    # smaller than both differences: kept
    (0.90, 0.50, 0.70),    # clipped to the backward difference
    (-0.80, -0.60, -0.35),  # clipped to the forward difference
    (0.60, -0.30, 0.45),   # the differences disagree in sign: slope removed
])
@pytest.mark.parametrize("dim,axis,sign", [(2, 0, -1), (2, 1, 1), (3, 0, 1), (3, 1, -1), (3, 2, -1)])
def test_single_acoustic_wave_reduces_to_scalar_minmod(dim, axis, sign, s, dw, de):
    o = _oracle(dim, (3,) * dim, limiter=2, beta=1.0, mtilde=0.5)
    U0 = _cons(1.0, [0.3, -0.2, 0.1][:dim], 1.0)
    r = _acoustic_eigvec(o, U0, axis, sign)
    w = np.zeros(o.shape)
    w[:, 0] = U0[:, None, None, None]
    # means along `axis` through the centre: U0 - dw r | U0 | U0 + de r
    idx = [slice(None)] * 3  # z, y, x of the state's cell axes
    for pos, off in ((0, -dw), (2, de)):
        sl = [1, 1, 1]
        sl[2 - axis] = pos
        if dim == 2:
            sl[0] = 0
        w[(slice(None), 0) + tuple(sl)] = U0 + off * r
    centre = (0, 1, 1) if dim == 2 else (1, 1, 1)
    w[(slice(None), 1 + axis) + centre] = s / R3 * r
    w[(slice(None), o.dim + 1) + centre] = 0.01 * np.arange(1, o.nvar + 1)  # a higher mode
    del idx
    out, st = o.limit(w)
    assert st == 0
    m = _minmod(s, dw, de)
    got = out[(slice(None), slice(None)) + centre]
    np.testing.assert_array_equal(got[:, 0], U0)  # means are kept
    np.testing.assert_allclose(got[:, 1 + axis], m / R3 * r, rtol=1e-7, atol=1e-9)
    for b in range(dim):
        if b != axis:
            np.testing.assert_allclose(got[:, 1 + b], 0.0, atol=1e-9)
    if m == s:
        np.testing.assert_array_equal(got, w[(slice(None), slice(None)) + centre])  # untouched
    else:
        np.testing.assert_array_equal(got[:, o.dim + 1:], 0.0)  # higher modes dropped


def _rough_state(o, seed, amp):
    rng = np.random.default_rng(seed)
    w = np.zeros(o.shape)
    w[0, 0] = 1.0 + 0.3 * rng.random(o.shape[2:])
    for a in range(o.dim):
        w[1 + a, 0] = 0.4 * rng.standard_normal(o.shape[2:])
    w[o.dim + 1, 0] = 2.5 + 0.5 * rng.random(o.shape[2:])
    w[:, 1:] = amp * rng.standard_normal(w[:, 1:].shape)
    return w


@pytest.mark.parametrize("dim", [2, 3])
def test_characteristic_limiter_keeps_means_and_bounded_slopes(dim):
    n = (5, 4, 3)[:dim]
    o = _oracle(dim, n, limiter=2, mtilde=0.5)
    w = _rough_state(o, 5 + dim, 0.05)
    out, st = o.limit(w)
    assert st == 0
    np.testing.assert_array_equal(out[:, 0], w[:, 0])
    assert not np.array_equal(out, w)
    # slopes below the TVB bound M~ dx in every characteristic field are kept:
    # scale the slopes down until no cell is touched
    small = w.copy()
    small[:, 1:] *= 1e-3
    out2, _ = o.limit(small)
    np.testing.assert_array_equal(out2, small)
    # idempotent up to round-off: a limited state is (nearly) a fixed point
    out3, _ = o.limit(out)
    np.testing.assert_allclose(out3, out, atol=1e-12)


def _sod(limiter, nx=64):
    wl = workloads.workload("sod", n=(nx, 2, 1), length=(1.0, 2.0 / nx, 1.0), limiter=limiter)
    o = oracle.Oracle(wl)
    w, st = o.limit(o.initial_state())
    assert st == 0
    t, t_end = 0.0, wl["t_end"]
    while t < t_end - 1e-14:
        dt = min(o.max_dt(w), t_end - t)
        w, _ = o.step(w, dt)
        t += dt
    rho = w[0, 0, 0].mean(axis=0)
    xs = (np.arange(nx * 64) + 0.5) / (nx * 64)
    ex, _ = _exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, GAMMA, (xs - 0.5) / t)
    ex = ex.reshape(nx, 64).mean(axis=1)
    return dict(l1=np.abs(rho - ex).mean(), tv=np.abs(np.diff(rho)).sum(), lo=rho.min(), hi=rho.max())


@pytest.mark.slow
def test_sod_limiter_comparison():
    # DG-3 (k = 2), 64 cells, t = 0.228, positivity limiter in all three runs
    none, comp, char = _sod(0), _sod(1), _sod(2)
    tv_exact = 1.0 - 0.125
    # no slope limiter: smallest L1 error, but over- and undershoots
    assert none["l1"] < char["l1"] < comp["l1"], (none, char, comp)
    assert none["hi"] > 1.0 + 1e-3 and none["lo"] < 0.125 - 1e-4
    # characteristic limiting: much closer to the exact profile than the
    # component-wise one (L1 and the variation of the means)
    assert char["l1"] < 0.5 * comp["l1"]
    assert char["tv"] < tv_exact * 1.01 < comp["tv"]
    assert 0.125 - 1e-5 < char["lo"] and char["hi"] < 1.0 + 1e-5
