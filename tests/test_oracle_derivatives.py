"""Pins of the oracle's complex-step derivatives, which serve as the reference
for the discrete adjoint: they must agree with central finite differences of
the oracle's own real-valued right-hand side and trajectory (to O(h^2)),
and be linear in the direction."""
import numpy as np

import oracle
import workloads


def _setup(k=2, n=8):
    """A state whose neighbouring cells differ by O(0.1): no wave-speed
    bound of the Riemann solver sits at a tie (where min/max has a kink and
    only one-sided derivatives exist)."""
    o = oracle.Oracle(workloads.workload("vortex", k=k, n=(n, n, 1), noise=0.0))
    rng = np.random.default_rng(4)
    w = np.zeros(o.shape)
    shp = w.shape[2:]
    rho = 1.0 + 0.3 * rng.uniform(0, 1, size=shp)
    vx, vy = 0.5 * rng.uniform(-1, 1, size=shp), 0.5 * rng.uniform(-1, 1, size=shp)
    p = 1.0 + 0.3 * rng.uniform(0, 1, size=shp)
    w[0, 0], w[1, 0], w[2, 0] = rho, rho * vx, rho * vy
    w[3, 0] = p / 0.4 + 0.5 * rho * (vx ** 2 + vy ** 2)
    w[:, 1:] = 0.01 * rng.uniform(-1, 1, size=w[:, 1:].shape)
    v = rng.uniform(-1, 1, size=o.shape) * 0.1
    return o, w, v


def test_complex_step_rhs_matches_central_differences():
    o, w, v = _setup()
    L, dL = o.jvp_rhs(w, v)
    # the real part is the plain RHS up to the rounding of complex division
    np.testing.assert_allclose(L, o.rhs(w), atol=1e-13 * np.abs(L).max())
    for h in (1e-4, 1e-5):
        fd = (o.rhs(w + h * v) - o.rhs(w - h * v)) / (2 * h)
        err = np.abs(fd - dL).max() / np.abs(dL).max()
        assert err < 1e-7, (h, err)


def test_complex_step_rhs_is_linear_in_direction():
    o, w, v = _setup(k=1)
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, size=o.shape)
    _, d1 = o.jvp_rhs(w, v)
    _, d2 = o.jvp_rhs(w, u)
    _, d3 = o.jvp_rhs(w, 2.0 * v - 3.0 * u)
    np.testing.assert_allclose(d3, 2.0 * d1 - 3.0 * d2, atol=1e-12 * np.abs(d3).max())


def test_complex_step_trajectory_matches_central_differences():
    o, w, v = _setup(k=2, n=8)
    dt = o.max_dt(w)
    steps = 4
    wT, dwT = o.jvp_traj(w, v, steps, dt)
    wr, _ = o.run(w, steps, dt=dt)
    np.testing.assert_allclose(wT, wr, atol=1e-13 * np.abs(wr).max())
    h = 1e-5
    fd = (o.run(w + h * v, steps, dt=dt)[0] - o.run(w - h * v, steps, dt=dt)[0]) / (2 * h)
    assert np.abs(fd - dwT).max() / np.abs(dwT).max() < 1e-7
