"""Pins of the oracle's gravity source (Sec. 2.4, eq. gravity_term) and
gravity time step (Sec. 2.5), and of the angular momentum conservation of
DG (Sec. 2.6) on the cold Keplerian disc (Sec. 5, Keplerian disc), against
closed forms: the projection of rho a and m . a for a uniform field, free
fall of a uniform medium, the time-step minimum, and the total angular
momentum of the unlimited DG-2 scheme under a central force."""
import math

import numpy as np
import pytest

import oracle
import workloads

G = (0.3, -0.7, 0.45)


def _uniform(dim, k, gravity, state=(1.3, (0.4, -0.2, 0.1), 0.9)):
    n = (6, 5, 4) if dim == 3 else (6, 5, 1)
    h = 1.0 / 3.0
    return workloads.workload("density_wave", dim=dim, k=k, n=n, length=tuple(h * m for m in n), ic="uniform",
                              state=state, gravity=gravity)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 3), (3, 2)])
def test_uniform_field_on_uniform_state(dim, k):
    o = oracle.Oracle(_uniform(dim, k, ("uniform", G)))
    w = o.initial_state()
    L = o.rhs(w)
    rho, vel = 1.3, (0.4, -0.2, 0.1)
    expect = [0.0] + [rho * G[a] for a in range(dim)] + [rho * sum(vel[a] * G[a] for a in range(dim))]
    for v in range(o.nvar):
        np.testing.assert_allclose(L[v, 0], expect[v], atol=1e-14)
    assert np.abs(L[:, 1:]).max() < 1e-13  # the hydro terms of a constant state, to rounding


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 4), (3, 1), (3, 2)])
def test_uniform_field_projects_exactly(dim, k):
    # for a constant field the source of the momentum is g_a times the density
    # coefficients, and that of the energy g . (momentum coefficients): the
    # volume rule integrates (degree k) x (degree k) exactly
    rng = np.random.default_rng(3 + dim * 10 + k)
    base = oracle.Oracle(_uniform(dim, k, None))
    grav = oracle.Oracle(_uniform(dim, k, ("uniform", G)))
    w = base.initial_state()
    w[:, 1:] = 0.05 * rng.uniform(-1, 1, size=w[:, 1:].shape)  # polynomial state of degree k
    D = grav.rhs(w) - base.rhs(w)
    np.testing.assert_allclose(D[0], 0.0, atol=1e-15)
    for a in range(dim):
        np.testing.assert_allclose(D[1 + a], G[a] * w[0], atol=1e-13)
    np.testing.assert_allclose(D[dim + 1], sum(G[a] * w[1 + a] for a in range(dim)), atol=1e-13)


def test_free_fall_of_a_uniform_medium():
    # no pressure gradient: every element accelerates with g, so rho stays,
    # m = rho (v0 + g t) and E = E0 + rho (v0 . g t + |g|^2 t^2 / 2); SSP-RK3
    # integrates these polynomials in t exactly
    wl = _uniform(2, 2, ("uniform", G))
    o = oracle.Oracle(wl)
    w = o.initial_state()
    rho, v0 = 1.3, np.array([0.4, -0.2])
    g = np.array(G[:2])
    E0 = w[3, 0].copy()
    dt, steps = 0.01, 7
    w, t = o.run(w, steps, dt=dt)
    np.testing.assert_allclose(w[0, 0], rho, rtol=1e-14)
    for a in range(2):
        np.testing.assert_allclose(w[1 + a, 0], rho * (v0[a] + g[a] * t), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(w[3, 0], E0 + rho * (v0 @ g * t + g @ g * t * t / 2), rtol=1e-13)
    assert np.abs(w[:, 1:]).max() < 1e-13


@pytest.mark.parametrize("strength", [0.1, 500.0])
def test_time_step_is_the_smaller_of_hydro_and_gravity(strength):
    state = (1.3, (0.4, -0.2, 0.0), 0.9)
    gvec = tuple(strength * x for x in G)
    o = oracle.Oracle(_uniform(2, 2, ("uniform", gvec), state))
    w = o.initial_state()
    gam = o.wl["gamma"]
    c = math.sqrt(gam * 0.9 / 1.3)
    hydro = o.wl["cfl"] / 5.0 / ((0.4 + c) / o.dx + (0.2 + c) / o.dx)
    grav = c / (math.sqrt(2 * gam * (gam - 1)) * math.hypot(gvec[0], gvec[1]))
    assert o.max_dt(w) == pytest.approx(min(hydro, grav), rel=1e-14)
    assert (grav < hydro) == (strength > 100.0)


def _total_angular_momentum(o, w):
    """Integral of x m_y - y m_x over the domain from the DG polynomial
    (mode 1 is sqrt(3) xi, mode 2 sqrt(3) eta; (1/2) int xi sqrt(3) xi = 1/sqrt(3))."""
    nx, ny = o.wl["n"][0], o.wl["n"][1]
    h = o.dx
    xc = o.wl["x0"][0] + (np.arange(nx) + 0.5) * h
    yc = o.wl["x0"][1] + (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(xc, yc)
    mx, my = w[1, :, 0], w[2, :, 0]
    s = h / 2 / math.sqrt(3.0)
    return (h * h * (X * my[0] + s * my[1] - Y * mx[0] - s * mx[2])).sum()


def test_dg2_conserves_angular_momentum_on_the_keplerian_disc():
    # Sec. 2.6: with test functions x and y in the space (k >= 1) DG
    # conserves angular momentum; the central force exerts no torque at any
    # node, and the background at rest with uniform pressure gives no net
    # boundary torque.  The minmod limiter breaks the conservation.  A warm
    # disc (background density 0.3, pressure 3) keeps the unlimited scheme
    # positive without the positivity limiter, which rescales slopes and so
    # would move L as well.
    wl = workloads.workload("kepler", n=(48, 48, 1), positivity=0, kepler_params=dict(rho0=0.3, p0=3.0))
    o = oracle.Oracle(wl)
    w0 = o.initial_state()
    L0 = _total_angular_momentum(o, w0)
    dt = o.max_dt(w0)
    w = w0
    for _ in range(6):
        w, _ = o.step(w, dt)
    drift = abs(_total_angular_momentum(o, w) - L0) / abs(L0)
    assert drift < 1e-13, drift
    lim = oracle.Oracle(dict(wl, limiter=1))
    w = w0
    for _ in range(6):
        w, _ = lim.step(w, dt)
    assert abs(_total_angular_momentum(o, w) - L0) / abs(L0) > 1e3 * max(drift, 1e-16)
