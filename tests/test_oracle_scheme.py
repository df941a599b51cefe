"""Pins of the oracle's right-hand side, Riemann solver, time step and time
integrator (Sec. 2.4-2.5, App. D) against closed forms, an independent
special-case implementation and the paper's exact solutions."""
import math

import numpy as np
import pytest

import oracle
import workloads
from conftest import frac, read_golden


def _box(n, h=0.125):
    """Box lengths giving cubic cells of edge h on an n-cell grid."""
    return tuple(h * m for m in n)


def _uniform(dim, k, n, state, **kw):
    wl = workloads.workload("density_wave", dim=dim, k=k, n=n, length=_box(n), ic="uniform",
                            state=state, **kw)
    return wl


def _random_smooth_state(o, seed, amp=0.1):
    """A positive state: a smooth random mean field plus small higher modes."""
    rng = np.random.default_rng(seed)
    w = np.zeros(o.shape)
    cells = w.shape[2:]
    rho = 1.0 + amp * rng.uniform(-1, 1, size=cells)
    vel = [0.3 * rng.uniform(-1, 1, size=cells) for _ in range(o.dim)]
    p = 1.0 + amp * rng.uniform(-1, 1, size=cells)
    w[0, 0] = rho
    for a in range(o.dim):
        w[1 + a, 0] = rho * vel[a]
    w[o.dim + 1, 0] = p / (o.wl["gamma"] - 1) + 0.5 * rho * sum(v * v for v in vel)
    w[:, 1:] = 0.02 * amp * rng.uniform(-1, 1, size=w[:, 1:].shape) * np.abs(w[:, :1])
    return w


# --- free stream and conservation -------------------------------------------------

@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_free_stream_is_steady(dim, k):
    # A constant state: the volume term vanishes (the flux is constant and the
    # basis gradients have zero mean) and the face fluxes cancel by
    # consistency of the Riemann solver, so L = 0.
    n = (5, 4, 3)
    wl = _uniform(dim, k, n, (1.3, (0.4, -0.7, 0.2), 2.1))
    o = oracle.Oracle(wl)
    w = o.initial_state()
    L = o.rhs(w)
    assert np.abs(L).max() < 1e-13


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 1), (3, 2)])
def test_discrete_conservation(dim, k):
    # Periodic box: every face flux enters two cells with opposite signs, so
    # sum_K |K| dw_1/dt = 0 to round-off (Sec. 1, conservation of DG).
    o = oracle.Oracle(workloads.workload("density_wave", dim=dim, k=k, n=(6, 5, 4),
                                           length=_box((6, 5, 4))))
    w = _random_smooth_state(o, seed=11)
    L = o.rhs(w)
    tot = L[:, 0].reshape(o.nvar, -1).sum(axis=1)
    scale = np.abs(L[:, 0]).reshape(o.nvar, -1).sum(axis=1)
    assert np.all(np.abs(tot) <= 1e-14 * scale)


def test_conservation_over_steps():
    o = oracle.Oracle(workloads.workload("vortex", n=(16, 16, 1)))
    w0 = o.initial_state()
    w, _ = o.run(w0, 5)
    np.testing.assert_allclose(o.totals(w), o.totals(w0), rtol=1e-13)


def test_volume_term_has_no_mean_component():
    # dphi_1/dxi = 0, so V_1 = 0 exactly; the mean changes through faces only.
    o = oracle.Oracle(workloads.workload("density_wave", dim=3, k=2, n=(3, 3, 3)))
    w = _random_smooth_state(o, seed=5)
    V, S = o.terms_cell(w, 13)
    assert np.all(V[:, 0] == 0.0)
    assert np.abs(S[:, 0]).max() > 0


# --- independent special case: scalar upwind DG advection ---------------------------

def _scalar_upwind_dg_rhs(r, e, k, dim, dx, vel):
    """Textbook modal upwind DG for rho_t + c . grad rho = 0 on a periodic grid,
    written independently with numpy's Gauss rule and Legendre series.
    r: [N][nz][ny][nx]; e: exponent table of the modes."""
    g, gw = np.polynomial.legendre.leggauss(k + 1)
    N = len(e)

    def pt(n, x, deriv=False):
        c = np.zeros(n + 1); c[-1] = math.sqrt(2 * n + 1)
        if deriv:
            c = np.polynomial.legendre.legder(c) if n > 0 else np.zeros(1)
        return np.polynomial.legendre.legval(x, c)

    import itertools
    nodes = list(itertools.product(range(k + 1), repeat=dim))
    out = np.zeros_like(r)
    axes_cells = {0: -1, 1: -2, 2: -3}  # x is the last array axis
    # volume term
    for idx in nodes:
        xi = [g[i] for i in idx]
        wq = np.prod([gw[i] for i in idx])
        phi = np.array([np.prod([pt(e[l][a], xi[a]) for a in range(dim)]) for l in range(N)])
        val = np.tensordot(phi, r, axes=(0, 0))
        for a in range(dim):
            dphi = np.array([np.prod([pt(e[l][b], xi[b], deriv=(b == a)) for b in range(dim)])
                             for l in range(N)])
            out += vel[a] * wq * dphi[:, None, None, None] * val[None]
    # face terms, upwind flux c_a * rho_upwind
    fnodes = list(itertools.product(range(k + 1), repeat=dim - 1))
    for a in range(dim):
        tang = [b for b in range(dim) if b != a]
        for idx in fnodes:
            wr = np.prod([gw[i] for i in idx]) if idx else 1.0
            xp = [0.0] * dim; xm = [0.0] * dim
            xp[a], xm[a] = 1.0, -1.0
            for j, b in enumerate(tang):
                xp[b] = xm[b] = g[idx[j]]
            php = np.array([np.prod([pt(e[l][b], xp[b]) for b in range(dim)]) for l in range(N)])
            phm = np.array([np.prod([pt(e[l][b], xm[b]) for b in range(dim)]) for l in range(N)])
            tp = np.tensordot(php, r, axes=(0, 0))  # trace at +1 of each cell
            tm = np.tensordot(phm, r, axes=(0, 0))  # trace at -1
            ax = {0: 2, 1: 1, 2: 0}[a]
            tm_next = np.roll(tm, -1, axis=ax)      # high neighbour's -1 trace
            tp_prev = np.roll(tp, 1, axis=ax)       # low neighbour's +1 trace
            f_hi = vel[a] * (tp if vel[a] > 0 else tm_next)  # flux at the +a face
            f_lo = vel[a] * (tp_prev if vel[a] > 0 else tm)  # flux at the -a face
            out -= wr * php[:, None, None, None] * f_hi[None]
            out += wr * phm[:, None, None, None] * f_lo[None]
    return (2.0 / dx) / 2 ** dim * out


@pytest.mark.parametrize("dim,k,vel", [(2, 1, (1.0, -0.6, 0.0)), (2, 2, (-0.8, 0.5, 0.0)),
                                       (2, 3, (1.0, 1.0, 0.0)), (3, 1, (0.7, -0.4, 0.3)),
                                       (3, 2, (-0.5, 0.6, 0.9))])
def test_contact_reduces_to_scalar_upwind_dg(dim, k, vel):
    # With constant velocity and pressure the Euler system is advection of
    # rho; HLLC resolves the contact exactly (S* = u), so the DG RHS of rho
    # equals scalar upwind DG, and m = v rho, E = p/(g-1) + |v|^2 rho / 2 follow.
    n = (6, 5, 4)
    o = oracle.Oracle(workloads.workload("density_wave", dim=dim, k=k, n=n, length=_box(n)))
    rng = np.random.default_rng(7)
    r = np.zeros(o.shape[1:])
    r[0] = 1.0 + 0.3 * rng.uniform(-1, 1, size=r.shape[1:])
    r[1:] = 0.05 * rng.uniform(-1, 1, size=r[1:].shape)
    g = o.wl["gamma"]
    p = 1.0
    w = np.zeros(o.shape)
    w[0] = r
    for a in range(dim):
        w[1 + a] = vel[a] * r
    ke = 0.5 * sum(v * v for v in vel[:dim])
    w[dim + 1] = ke * r
    w[dim + 1, 0] += p / (g - 1)
    L = o.rhs(w)
    Lr = _scalar_upwind_dg_rhs(r, o.exponents().tolist(), k, dim, o.dx, vel)
    scale = np.abs(Lr).max()
    np.testing.assert_allclose(L[0], Lr, atol=1e-12 * scale)
    for a in range(dim):
        np.testing.assert_allclose(L[1 + a], vel[a] * Lr, atol=1e-12 * scale)
    np.testing.assert_allclose(L[dim + 1], ke * Lr, atol=1e-12 * scale)


def test_axis_swap_symmetry():
    # Transposing the grid and swapping m_x <-> m_y (and the x/y exponents
    # of the modes) transposes the RHS.
    o = oracle.Oracle(workloads.workload("density_wave", dim=2, k=2, n=(6, 6, 1)))
    w = _random_smooth_state(o, seed=3)
    e = o.exponents()
    perm = [int(np.where((e[:, 0] == e[l, 1]) & (e[:, 1] == e[l, 0]))[0][0]) for l in range(o.N)]
    def swap(a):
        b = a[[0, 2, 1, 3]][:, perm]
        return np.ascontiguousarray(np.swapaxes(b, -1, -2))
    L = o.rhs(w)
    Ls = o.rhs(swap(w))
    np.testing.assert_allclose(Ls, swap(L), atol=1e-13 * np.abs(L).max())


# --- exact solutions and convergence order (Sec. 5.1) -------------------------------------

def _order(errs, ns):
    return [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_density_wave_translates_with_order_k_plus_1(k):
    # rho = 1 + 0.2 sin(2 pi (x + y - 2t)) is the exact solution; the L1 error
    # (eq. L1_norm, integrated with (k+3)^2 points) must fall at order >= k+1
    # up to 0.2 (the paper observes the expected rate or better).
    ns = [8, 16, 32]
    errs = []
    t_end = 0.05
    for n in ns:
        o = oracle.Oracle(workloads.workload("density_wave", k=k, n=(n, n, 1)))
        w = o.initial_state()
        dt0 = o.max_dt(w)
        steps = int(math.ceil(t_end / dt0))
        w, t = o.run(w, steps, dt=t_end / steps)
        errs.append(o.l1_density_error(w, t))
    orders = _order(errs, ns)
    assert min(orders) >= k + 1 - 0.2, (errs, orders)


@pytest.mark.parametrize("k", [1, 2])
def test_boosted_vortex_translates_with_order_k_plus_1(k):
    # The isentropic vortex with boost (1,1) translates exactly (Sec. 5.1).
    ns = [16, 32, 64]
    errs = []
    t_end = 0.2
    for n in ns:
        o = oracle.Oracle(workloads.workload("vortex", k=k, n=(n, n, 1), noise=0.0))
        w = o.initial_state()
        steps = int(math.ceil(t_end / o.max_dt(w)))
        w, t = o.run(w, steps, dt=t_end / steps)
        errs.append(o.l1_density_error(w, t))
    orders = _order(errs, ns)
    assert min(orders) >= k + 1 - 0.2, (errs, orders)


def test_wrong_direction_would_be_caught():
    # Guard for the convergence tests: the error against the solution moving
    # the wrong way is O(1), far above the scheme's error.
    o = oracle.Oracle(workloads.workload("density_wave", k=2, n=(16, 16, 1)))
    w = o.initial_state()
    w, t = o.run(w, 40)
    good, bad = o.l1_density_error(w, t), o.l1_density_error(w, -t)
    assert bad > 20 * good, (good, bad)


# --- HLLC (Sec. 2.4 numerical flux) -----------------------------------------------------

def _cons(dim, g, rho, vel, p):
    U = [rho] + [rho * v for v in vel[:dim]] + [p / (g - 1) + 0.5 * rho * sum(v * v for v in vel[:dim])]
    return np.array(U)


@pytest.mark.parametrize("flux", [0, 1])
def test_hllc_consistency(flux):
    rng = np.random.default_rng(1)
    for dim in (2, 3):
        o = oracle.Oracle(workloads.workload("density_wave", dim=dim, k=1, n=(2, 2, 2), flux=flux))
        for _ in range(50):
            U = _cons(dim, 1.4, rng.uniform(0.1, 3), rng.uniform(-2, 2, 3), rng.uniform(0.1, 3))
            for a in range(dim):
                np.testing.assert_allclose(o.hllc(U, U, a), o.euler_flux(U, a), rtol=1e-13, atol=1e-13)


def test_euler_flux_closed_form():
    o = oracle.Oracle(workloads.workload("density_wave", dim=3, k=1, n=(2, 2, 2)))
    rho, v, p, g = 1.7, (0.3, -1.1, 0.6), 2.3, 1.4
    U = _cons(3, g, rho, v, p)
    E = U[4]
    for a in range(3):
        F = o.euler_flux(U, a)
        ref = [rho * v[a]] + [rho * v[a] * v[b] + (p if a == b else 0.0) for b in range(3)] + [(E + p) * v[a]]
        np.testing.assert_allclose(F, ref, rtol=1e-14)


def test_hllc_stationary_contact_and_shear():
    # A contact at rest (pressure and normal velocity equal) is exact: only
    # pressure flux in the normal momentum; a tangential-velocity jump too.
    o = oracle.Oracle(workloads.workload("density_wave", dim=3, k=1, n=(2, 2, 2)))
    UL = _cons(3, 1.4, 2.0, (0.0, 0.3, 0.0), 1.5)
    UR = _cons(3, 1.4, 0.5, (0.0, -0.2, 0.7), 1.5)
    F = o.hllc(UL, UR, 0)
    np.testing.assert_allclose(F, [0.0, 1.5, 0.0, 0.0, 0.0], atol=1e-14)


def test_hllc_reflection_symmetry():
    # Mirror x -> -x: F(UL, UR) = -M F(M UR, M UL), M flips the normal momentum.
    rng = np.random.default_rng(2)
    o = oracle.Oracle(workloads.workload("density_wave", dim=2, k=1, n=(2, 2, 1)))
    for _ in range(50):
        UL = _cons(2, 1.4, rng.uniform(0.1, 3), rng.uniform(-2, 2, 3), rng.uniform(0.1, 3))
        UR = _cons(2, 1.4, rng.uniform(0.1, 3), rng.uniform(-2, 2, 3), rng.uniform(0.1, 3))
        M = np.array([1.0, -1.0, 1.0, 1.0])
        F = o.hllc(UL, UR, 0)
        Fm = o.hllc(M * UR, M * UL, 0)
        np.testing.assert_allclose(F, -M * Fm, rtol=1e-12, atol=1e-12)


def test_hllc_supersonic_upwinding():
    o = oracle.Oracle(workloads.workload("density_wave", dim=2, k=1, n=(2, 2, 1)))
    UL = _cons(2, 1.4, 1.0, (5.0, 0.2, 0), 1.0)
    UR = _cons(2, 1.4, 0.8, (4.5, -0.1, 0), 0.9)
    assert np.array_equal(o.hllc(UL, UR, 0), o.euler_flux(UL, 0))
    UL = _cons(2, 1.4, 1.0, (0.1, -5.0, 0), 1.0)
    UR = _cons(2, 1.4, 0.8, (0.0, -4.5, 0), 0.9)
    assert np.array_equal(o.hllc(UL, UR, 1), o.euler_flux(UR, 1))


def test_hllc_positivity_of_wave_speeds_on_strong_rarefaction():
    # Two states moving apart fast: the flux stays finite and the mass flux
    # lies between the one-sided physical mass fluxes' bounds.
    o = oracle.Oracle(workloads.workload("density_wave", dim=2, k=1, n=(2, 2, 1)))
    UL = _cons(2, 1.4, 1.0, (-2.0, 0, 0), 0.4)
    UR = _cons(2, 1.4, 1.0, (2.0, 0, 0), 0.4)
    F = o.hllc(UL, UR, 0)
    assert np.all(np.isfinite(F))
    assert abs(F[0]) < 1e-14  # symmetric problem: no net mass flux


# --- time step (eq. time_step, eq. time_step_pos) --------------------------------------------------

@pytest.mark.parametrize("dim,k,pos", [(2, 1, 0), (2, 2, 0), (3, 3, 0), (2, 1, 1), (2, 2, 1), (3, 3, 1)])
def test_time_step_closed_form(dim, k, pos):
    rho, v, p, g, cfl = 1.3, (0.4, -0.7, 0.2), 2.1, 1.4, 0.2
    o = oracle.Oracle(_uniform(dim, k, (8, 8, 8), (rho, v, p), positivity=pos, cfl=cfl))
    w = o.initial_state()
    c = math.sqrt(g * p / rho)
    fk = 1.0 / (2 * k + 1)
    if pos:
        w1 = {1: 1.0, 2: 1.0 / 3.0, 3: 1.0 / 3.0}[k]  # first GLL weight (Sec. 3.4)
        fk = min(fk, w1 / 2)
    dt = cfl * fk / sum((abs(v[a]) + c) / o.dx for a in range(dim))
    assert o.max_dt(w) == pytest.approx(dt, rel=1e-14)


def test_time_step_is_global_minimum():
    o = oracle.Oracle(workloads.workload("density_wave", k=1, n=(32, 32, 1)))
    w = o.initial_state()
    rho = w[0, 0]; m = w[1:3, 0]; E = w[3, 0]
    p = 0.4 * (E - 0.5 * (m ** 2).sum(0) / rho)
    c = np.sqrt(1.4 * p / rho)
    rate = ((np.abs(m / rho) + c) / o.dx).sum(0)
    assert o.max_dt(w) == pytest.approx((0.3 / 3 / rate).min(), rel=1e-14)


# --- SSP-RK3 (App. D, table RK_3) -------------------------------------------------------------

def _butcher():
    rows = read_golden("ssp_rk3_tableau.txt")
    A = np.zeros((3, 3)); c = np.zeros(3)
    i = 0
    for r in rows:
        if r[0] == "c":
            c[i] = frac(r[1])
            for j, s in enumerate(r[2:]):
                A[i, j] = frac(s)
            i += 1
        else:
            b = np.array([frac(s) for s in r[1:]])
    return A, b, c


def _oracle_rk3(f, w0, dt):
    lib, _ = oracle._load()
    w = np.array([w0])
    stages = []
    out = np.zeros(1)
    wp = w.copy()
    for s in (1, 2, 3):
        L = np.array([f(wp[0])])
        out = np.zeros(1)
        lib.orc_rk3_combine(s, dt, w, wp, L, out, 1)
        wp = out.copy()
    return wp[0]


def test_rk3_matches_printed_butcher_tableau():
    A, b, c = _butcher()
    assert np.allclose(A.sum(axis=1), c)
    f = lambda w: -w * w + math.sin(w)   # dw/dt = f(w) (the paper writes -R)
    for w0, dt in [(0.7, 0.1), (-1.3, 0.05), (2.0, 0.2)]:
        k = []
        for i in range(3):
            k.append(f(w0 + dt * sum(A[i, j] * k[j] for j in range(i))))
        ref = w0 + dt * sum(b[i] * k[i] for i in range(3))
        assert _oracle_rk3(f, w0, dt) == pytest.approx(ref, rel=1e-14, abs=1e-15)


def test_rk3_linear_stability_polynomial():
    for z in [-0.1, -1.0, -2.5, 0.3]:
        got = _oracle_rk3(lambda w: z * w, 1.0, 1.0)
        assert got == pytest.approx(1 + z + z * z / 2 + z ** 3 / 6, rel=1e-14)


def test_rk3_third_order_on_scheme():
    # Halving dt on the full DG system shrinks the one-step difference to a
    # fine-dt reference by 2^4 (local error O(dt^4)).
    o = oracle.Oracle(workloads.workload("vortex", k=2, n=(8, 8, 1), noise=0.0))
    w0 = o.initial_state()
    dt = 0.05
    def run(h, n):
        w = w0
        for _ in range(n):
            w, _ = o.step(w, h)
        return w
    ref = run(dt / 32, 32)
    e1 = np.abs(run(dt, 1) - ref).max()
    e2 = np.abs(run(dt / 2, 2) - ref).max()
    assert e1 / e2 > 2 ** 3 * 0.8
