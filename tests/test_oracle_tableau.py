"""Pins of the oracle's general explicit Runge-Kutta integrator (App. D: the
Butcher tableau, the update for w^{n+1}, eq. rhs; tables RK_2, RK_3, RK_4)
against what the tableau itself fixes: the Butcher-form evaluation on a
scalar ODE, the linear stability function 1 + z b^T (I - zA)^{-1} 1, the
textbook Shu-Osher forms of Heun's method and SSP-RK3, the existing SSP-RK3
stages, and the observed orders on the DG scheme."""
import math

import numpy as np
import pytest

import oracle
import workloads
from conftest import frac, read_golden


def _golden_tableau(name):
    rows = read_golden(name)
    crow = [r for r in rows if r[0] == "c"]
    s = len(crow)
    A = np.zeros((s, s)); c = np.zeros(s)
    for i, r in enumerate(crow):
        c[i] = frac(r[1])
        for j, x in enumerate(r[2:]):
            A[i, j] = frac(x)
    b = np.array([frac(x) for x in [r for r in rows if r[0] == "b"][0][1:]])
    return A, b, c


TABLES = {"rk2": "ssp_rk2_tableau.txt", "rk3": "ssp_rk3_tableau.txt", "rk4": "ssp_rk4_tableau.txt"}


@pytest.mark.parametrize("name", sorted(TABLES))
def test_printed_tableaus(name):
    A, b, c = _golden_tableau(TABLES[name])
    np.testing.assert_allclose(A.sum(axis=1), c, atol=1e-13)  # nodes are the row sums
    assert np.all(np.triu(A) == 0.0)  # explicit
    oA, ob = oracle.TABLEAUS[name]
    np.testing.assert_array_equal(np.array(oA), A)
    np.testing.assert_array_equal(np.array(ob), b)
    # first-order consistency: exact for RK_2 and RK_3, to the printed digits for RK_4
    assert abs(b.sum() - 1.0) <= (1e-10 if name == "rk4" else 1e-15)


def test_shu_osher_forms_of_heun_and_ssp_rk3():
    A, b, _ = _golden_tableau(TABLES["rk2"])
    al, be = oracle.tableau_form(A, b)
    np.testing.assert_allclose(al[1, :1], [1.0], atol=1e-16)
    np.testing.assert_allclose(al[2, :2], [0.5, 0.5], atol=1e-16)
    np.testing.assert_allclose(be[1:], [1.0, 0.5], atol=1e-16)
    A, b, _ = _golden_tableau(TABLES["rk3"])
    al, be = oracle.tableau_form(A, b)
    np.testing.assert_allclose(al[2, :2], [0.75, 0.25], atol=1e-16)
    np.testing.assert_allclose(al[3, :3], [1 / 3, 0.0, 2 / 3], atol=1e-16)
    np.testing.assert_allclose(be[1:], [1.0, 0.25, 2 / 3], atol=1e-16)


def _oracle_ode_step(A, b, f, w0, dt):
    Y = [np.array([w0])]
    for m in range(1, len(b) + 1):
        Y.append(oracle.tableau_combine(A, b, m, dt, Y, f(Y[-1])))
    return float(Y[-1][0])


def _butcher_ode_step(A, b, f, w0, dt):
    k = []
    for i in range(len(b)):
        k.append(f(np.array([w0 + dt * sum(A[i, j] * k[j] for j in range(i))]))[0])
    return w0 + dt * sum(b[i] * k[i] for i in range(len(b)))


def _random_tableau(s, seed):
    rng = np.random.default_rng(seed)
    A = np.tril(rng.uniform(0.1, 0.6, size=(s, s)), -1)
    return A, rng.uniform(0.05, 0.4, size=s)


@pytest.mark.parametrize("which", ["rk2", "rk3", "rk4", "random4", "random6"])
def test_stage_values_reproduce_the_butcher_form(which):
    if which.startswith("random"):
        A, b = _random_tableau(int(which[-1]), seed=len(which))
    else:
        A, b, _ = _golden_tableau(TABLES[which])
    f = lambda w: -w * w + np.sin(w)  # noqa: E731  (dw/dt = f; the paper writes -R)
    for w0, dt in [(0.7, 0.1), (-1.3, 0.05), (2.0, 0.2)]:
        assert _oracle_ode_step(A, b, f, w0, dt) == pytest.approx(_butcher_ode_step(A, b, f, w0, dt), rel=2e-14)


@pytest.mark.parametrize("name", ["rk2", "rk4"])
def test_linear_stability_function(name):
    A, b, _ = _golden_tableau(TABLES[name])
    s = len(b)
    for z in [-0.1, -0.7, -1.9, -2.7, 0.4]:
        got = _oracle_ode_step(A, b, lambda w: z * w, 1.0, 1.0)
        R = 1.0 + z * b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))
        assert got == pytest.approx(R, rel=1e-13)
        taylor = sum(z ** q / math.factorial(q) for q in range(len(b) + 1 if name == "rk2" else 5))
        if name == "rk2":
            assert got == pytest.approx(taylor, rel=1e-14)
        else:  # fourth order up to the printed rounding (weights off by 8.8e-11)
            assert abs(got - taylor) <= abs(z) ** 5 / 60 + 2e-10 * abs(z)


def test_tableau_rejects_implicit_and_degenerate_tables():
    with pytest.raises(RuntimeError):
        oracle.tableau_form([[0.5, 0.0], [0.5, 0.0]], [0.5, 0.5])  # diagonal entry
    with pytest.raises(RuntimeError):
        oracle.tableau_form([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.5, 0.5, 0.0]], [0.2, 0.3, 0.5])  # a_21 = 0
    with pytest.raises(RuntimeError):
        oracle.tableau_form([[0.0, 0.0], [1.0, 0.0]], [1.0, 0.0])  # b_s = 0


@pytest.mark.parametrize("name,spec", [
    ("vortex", dict(name="vortex", k=2, n=(10, 8, 1), length=(10.0, 8.0, 1.0))),
    ("sod_limited", dict(name="sod", n=(24, 2, 1), length=(1.0, 2 / 24, 1.0), eps=1e-3)),
])
def test_rk3_tableau_step_equals_the_ssp_rk3_step(name, spec):
    spec = dict(spec)
    wl = workloads.workload(spec.pop("name"), **spec)
    o = oracle.Oracle(wl)
    w, st = o.limit(o.initial_state())
    assert st == 0
    A, b = oracle.TABLEAUS["rk3"]
    for _ in range(3):
        ref, dt = o.step(w)
        got, dt2 = o.step_tableau(w, A, b)
        assert dt == dt2
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14 * np.abs(ref).max())
        w = ref


def test_rk3_tableau_stage_on_the_refined_box():
    h = 1.0 / 8.0
    n = (8, 7, 6)
    wl = workloads.workload("blast_amr", dim=3, k=1, n=n, length=tuple(h * m for m in n), refine_lo=(2, 2, 1),
                            refine_hi=(6, 5, 4), ic="kh3d", noise=1e-2, seed=6140, limiter=0, positivity=0)
    o = oracle.AmrOracle(wl)
    w0 = o.initial_state()
    dt = o.max_dt(w0)
    A, b = oracle.TABLEAUS["rk3"]
    Y = [w0]
    for m in (1, 2, 3):
        Y.append(o.tableau_stage(A, b, m, dt, Y))
        ref = o.rk3_stage(m, dt, w0, Y[-2])
        np.testing.assert_allclose(Y[-1], ref, rtol=0, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("name,k,p", [("rk2", 1, 2), ("rk4", 3, 4)])
def test_local_error_order_on_the_scheme(name, k, p):
    # over a fixed interval (one step of dt, two of dt/2) the difference to a
    # fine-dt reference on the full DG system shrinks by 2^p
    o = oracle.Oracle(workloads.workload("vortex", k=k, n=(8, 8, 1), noise=0.0))
    A, b = oracle.TABLEAUS[name]
    w0 = o.initial_state()
    dt = 0.04

    def run(h, n):
        w = w0
        for _ in range(n):
            w, _ = o.step_tableau(w, A, b, h)
        return w

    ref = run(dt / 32, 32)
    e1 = np.abs(run(dt, 1) - ref).max()
    e2 = np.abs(run(dt / 2, 2) - ref).max()
    assert e1 / e2 > 2 ** p * 0.8, (e1, e2)


@pytest.mark.slow
def test_dg4_vortex_converges_at_fourth_order():
    # DG-4 (k = 3 with the five-stage RK_4) on the boosted vortex (Sec. 5.1):
    # L1 density error of order >= 4 - 0.2
    ns = [12, 24, 48]
    errs = []
    t_end = 0.2
    for n in ns:
        o = oracle.Oracle(workloads.workload("vortex", k=3, n=(n, n, 1), noise=0.0, rk="rk4"))
        w = o.initial_state()
        steps = int(math.ceil(t_end / o.max_dt(w)))
        w, t = o.run(w, steps, dt=t_end / steps)
        errs.append(o.l1_density_error(w, t))
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(len(ns) - 1)]
    assert min(orders) >= 4 - 0.2, (errs, orders)
