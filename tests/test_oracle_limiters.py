"""Pins of the oracle's slope limiter (Sec. 3.1, 3.3) and positivity limiter
(Sec. 3.4) against hand-built cases and the properties the paper states, and
of the limited scheme against the exact Sod solution (Sec. 5.2)."""
import math

import numpy as np
import pytest

import oracle
import workloads
from conftest import read_golden

R3 = math.sqrt(3.0)


def _grid(dim=2, k=2, n=(3, 3, 1), **kw):
    h = 1.0 / 3.0
    wl = workloads.workload("density_wave", dim=dim, k=k, n=n,
                            length=tuple(h * m for m in n), **kw)
    return oracle.Oracle(wl)


def _positive_means(o, rho=1.0, p=1.0):
    w = np.zeros(o.shape)
    w[0, 0] = rho
    w[o.dim + 1, 0] = p / 0.4
    return w


@pytest.mark.parametrize("a,expect_slope,expect_limited", [
    (0.1, 0.1, False),    # |a| below both differences, same sign: kept
    (0.5, 0.2, True),     # clipped to beta * backward difference
    (0.25, 0.2, True),    # between the differences: clipped to the smaller
    (-0.1, 0.0, True),    # sign disagrees: slope removed
])
def test_minmod_cases(a, expect_slope, expect_limited):
    o = _grid(limiter=1, mtilde=0.0, beta=1.0)
    w = _positive_means(o)
    # x-row through the centre cell: means 1.0 | 1.2 | 1.5 of the density
    w[0, 0, 0, 1, :] = [1.0, 1.2, 1.5]
    w[0, 1, 0, 1, 1] = a / R3           # x-slope of the centre cell
    w[0, 3:, 0, 1, 1] = [0.01, -0.02, 0.03]  # second-degree modes
    out, st = o.limit(w)
    assert st == 0
    c = out[0, :, 0, 1, 1]
    if expect_limited:
        assert c[1] == pytest.approx(expect_slope / R3, abs=1e-16)
        assert np.all(c[3:] == 0.0)
    else:
        assert np.array_equal(c, w[0, :, 0, 1, 1])
    # other components: no slopes, unchanged; all means unchanged
    assert np.array_equal(out[1:, :, 0, 1, 1], w[1:, :, 0, 1, 1])
    assert np.array_equal(out[:, 0], w[:, 0])


def test_tvb_bound_keeps_small_slopes():
    # minmodB: a is kept when |a| <= Mtilde dx (Sec. 3.3); here dx = 1/3.
    o = _grid(limiter=1, mtilde=0.9, beta=1.0)
    w = _positive_means(o)
    w[0, 0, 0, 1, :] = [1.0, 1.2, 1.5]
    w[0, 1, 0, 1, 1] = -0.29 / R3  # |a| = 0.29 <= 0.3: kept although signs differ
    w[0, 3, 0, 1, 1] = 0.01
    out, _ = o.limit(w)
    assert np.array_equal(out[0, :, 0, 1, 1], w[0, :, 0, 1, 1])
    w[0, 1, 0, 1, 1] = -0.31 / R3  # above the bound: minmod applies
    out, _ = o.limit(w)
    assert out[0, 1, 0, 1, 1] == 0.0 and out[0, 3, 0, 1, 1] == 0.0


def test_limiting_one_direction_sets_all_slopes_of_the_component():
    # If any direction is limited the component becomes w1 + limited linear
    # part (eq. comp_limiter_applied): the y-slope passes through 1/sqrt(3) *
    # minmod, and degree >= 2 modes vanish.
    o = _grid(limiter=1, mtilde=0.0, beta=1.0)
    w = _positive_means(o)
    w[0, 0, 0, 1, :] = [1.0, 1.2, 1.5]
    w[0, 0, 0, :, 1] = [1.1, 1.2, 1.4]
    w[0, 1, 0, 1, 1] = 0.5 / R3   # limited in x
    w[0, 2, 0, 1, 1] = 0.05 / R3  # fine in y (0.05 < 0.1, 0.2)
    out, _ = o.limit(w)
    assert out[0, 1, 0, 1, 1] == pytest.approx(0.2 / R3, abs=1e-16)
    assert out[0, 2, 0, 1, 1] == pytest.approx(0.05 / R3, rel=1e-15)


def test_limiter_on_smooth_linear_data_is_identity():
    # A linear field whose slopes equal the mean differences divided by sqrt(3)
    # is not clipped with beta = 1.
    o = _grid(n=(5, 5, 1), limiter=1, mtilde=0.0, beta=1.0)
    w = _positive_means(o)
    ix = np.arange(5)
    w[0, 0, 0] = 1.0 + 0.1 * ix[None, :] + 0.05 * ix[:, None]
    w[0, 1, 0, 1:-1, 1:-1] = 0.1 / R3 * 0.999
    w[0, 2, 0, 1:-1, 1:-1] = 0.05 / R3 * 0.999
    out, _ = o.limit(w)
    np.testing.assert_array_equal(out[:, :, 0, 1:-1, 1:-1], w[:, :, 0, 1:-1, 1:-1])


def _rough_state(o, seed, amp):
    rng = np.random.default_rng(seed)
    w = np.zeros(o.shape)
    w[0, 0] = 1.0 + 0.5 * rng.uniform(0, 1, size=w.shape[2:])
    w[1, 0] = 0.3 * rng.uniform(-1, 1, size=w.shape[2:])
    pbar = 0.02 + 0.2 * rng.uniform(0, 1, size=w.shape[2:])
    w[o.dim + 1, 0] = 0.5 * w[1, 0] ** 2 / w[0, 0] + pbar / 0.4
    w[:, 1:] = amp * rng.uniform(-1, 1, size=w[:, 1:].shape)
    return w


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (3, 2), (3, 3)])
def test_positivity_limiter_enforces_floor(dim, k):
    n = (4, 4, 3)
    o = _grid(dim=dim, k=k, n=n, positivity=1, limiter=0)
    w = _rough_state(o, seed=dim * 10 + k, amp=0.6)
    S = o.positivity_points()
    def prims(ww):
        u = o.eval_points(ww, S)
        rho = u[..., 0]
        ke = 0.5 * (u[..., 1:dim + 1] ** 2).sum(-1) / rho
        return rho, 0.4 * (u[..., dim + 1] - ke)
    r0, p0 = prims(w)
    assert r0.min() < 0 or p0.min() < 0  # the test state needs limiting
    out, st = o.limit(w)
    assert st == 0
    r1, p1 = prims(out)
    eps = 1e-10
    assert r1.min() >= eps - 1e-13
    assert p1.min() >= eps - 1e-12
    np.testing.assert_array_equal(out[:, 0], w[:, 0])  # means untouched


def test_positivity_limiter_is_identity_on_positive_states():
    o = _grid(dim=3, k=2, n=(4, 4, 3), positivity=1)
    w = _rough_state(o, seed=1, amp=1e-4)
    w[o.dim + 1, 0] += 1.0
    out, st = o.limit(w)
    assert st == 0
    np.testing.assert_array_equal(out, w)


def test_negative_mean_is_reported():
    o = _grid(dim=2, k=1, n=(3, 3, 1), positivity=1)
    w = _positive_means(o)
    w[0, 0, 0, 1, 1] = -0.5
    _, st = o.limit(w)
    assert st == oracle.ORC_ENEGATIVE


# --- Sod shock tube against the exact Riemann solution (Sec. 5.2) ----------------------

def _exact_riemann(rl, ul, pl, rr, ur, pr, g, xi):
    """Exact solution of the 1D Riemann problem at similarity coordinates xi = x/t
    (Toro, ch. 4: Newton iteration on the pressure function, then sampling)."""
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

    def fK(p, rK, pK, cK):
        if p > pK:
            A, B = 2 / ((g + 1) * rK), (g - 1) / (g + 1) * pK
            return (p - pK) * math.sqrt(A / (p + B)), math.sqrt(A / (B + p)) * (1 - (p - pK) / (2 * (B + p)))
        pr_ = p / pK
        return 2 * cK / (g - 1) * (pr_ ** ((g - 1) / (2 * g)) - 1), pr_ ** (-(g + 1) / (2 * g)) / (rK * cK)

    p = 0.5 * (pl + pr)
    for _ in range(100):
        f1, d1 = fK(p, rl, pl, cl)
        f2, d2 = fK(p, rr, pr, cr)
        dp = (f1 + f2 + ur - ul) / (d1 + d2)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-15 * p:
            break
    u = 0.5 * (ul + ur) + 0.5 * (fK(p, rr, pr, cr)[0] - fK(p, rl, pl, cl)[0])
    rsl = rl * (p / pl) ** (1 / g) if p <= pl else rl * ((p / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pl + 1))
    rsr = rr * ((p / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pr + 1)) if p > pr else rr * (p / pr) ** (1 / g)
    sr = ur + cr * math.sqrt((g + 1) / (2 * g) * p / pr + (g - 1) / (2 * g))
    csl = cl * (p / pl) ** ((g - 1) / (2 * g))
    out = np.empty_like(xi)
    for i, s in enumerate(xi):
        if s < u:
            if s < ul - cl:
                out[i] = rl
            elif s > u - csl:
                out[i] = rsl
            else:
                out[i] = rl * (2 / (g + 1) + (g - 1) / ((g + 1) * cl) * (ul - s)) ** (2 / (g - 1))
        else:
            out[i] = rsr if s < sr else rr
    return out, dict(p_star=p, u_star=u, rho_star_left=rsl, rho_star_right=rsr, shock_speed=sr)


def test_exact_riemann_solver_reproduces_textbook_star_state():
    _, star = _exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4, np.array([0.0]))
    for name, val in read_golden("sod_star_state.txt"):
        assert star[name] == pytest.approx(float(val), abs=6e-5)


def _sod_l1(nx):
    wl = workloads.workload("sod", n=(nx, 4, 1), length=(1.0, 4.0 / nx, 1.0))
    o = oracle.Oracle(wl)
    w = o.initial_state()
    w, st = o.limit(w)  # the main loop limits the initial state too (Sec. 4.5)
    assert st == 0
    t, t_end = 0.0, wl["t_end"]
    while t < t_end - 1e-14:
        dt = min(o.max_dt(w), t_end - t)
        w, _ = o.step(w, dt)
        t += dt
    rho = w[0, 0, 0].mean(axis=0)  # average the (identical) rows
    xs = (np.arange(nx * 64) + 0.5) / (nx * 64)
    ex, star = _exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4, (xs - 0.5) / t)
    ex = ex.reshape(nx, 64).mean(axis=1)
    # the waves have not reached the open ends, so (up to the exponentially
    # small numerical precursors reaching them) no mass has left the box
    np.testing.assert_allclose(o.totals(w)[0], 4.0 / nx * (0.5 + 0.5 * 0.125), rtol=1e-8)
    assert rho.min() > 0.125 - 0.01 and rho.max() < 1.0 + 0.01
    # shock position: the density crosses the mid value between the
    # post-shock and pre-shock states within two cells of 0.5 + S t
    mid = 0.5 * (star["rho_star_right"] + 0.125)
    xc = (np.arange(nx) + 0.5) / nx
    i = np.where((rho[:-1] > mid) & (rho[1:] <= mid))[0][-1]
    assert abs(xc[i] - (0.5 + star["shock_speed"] * t)) < 2.0 / nx
    return np.abs(rho - ex).mean()


@pytest.mark.slow
def test_sod_cell_means_converge_to_exact_solution():
    e64 = _sod_l1(64)
    e128 = _sod_l1(128)
    assert e64 < 0.015, e64
    assert e128 < 0.7 * e64, (e64, e128)
