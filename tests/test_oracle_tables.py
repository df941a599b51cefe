"""Pins of the oracle's tables (App. A-C, Sec. 2.2) against closed forms and
the values the paper prints.  None of these checks calls the oracle to
produce its own expected value."""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads
from conftest import frac, read_golden


# --- Legendre polynomials (App. A) -----------------------------------------

def test_legendre_matches_printed_polynomials():
    rows = read_golden("legendre_polynomials.txt")
    xs = np.linspace(-1.0, 1.0, 17)
    for row in rows:
        n, den = int(row[0]), float(row[1])
        coef = [float(c) / den for c in row[2:]]
        assert len(coef) == n + 1
        dcoef = [j * coef[j] for j in range(1, n + 1)]
        for x in xs:
            P, dP = oracle.legendre(n, x)
            assert P == pytest.approx(sum(c * x ** j for j, c in enumerate(coef)), abs=1e-14)
            assert dP == pytest.approx(sum(c * x ** j for j, c in enumerate(dcoef)), abs=1e-13)


def test_scaled_legendre_end_values():
    # Ptilde_n(+-1) = (+-1)^n sqrt(2n+1): the basis at the faces.
    wl = workloads.workload("density_wave", k=4, dim=3, n=(2, 2, 2))
    o = oracle.Oracle(wl)
    e = o.exponents()
    for s in (-1.0, 1.0):
        B = o.basis_at([[s, 0.0, 0.0]])[0]
        for l in range(o.N):
            if e[l, 1] == 0 and e[l, 2] == 0:
                n = e[l, 0]
                assert B[l] == pytest.approx(s ** n * math.sqrt(2 * n + 1), rel=1e-14)


# --- Gauss-Legendre (App. B) and Gauss-Lobatto-Legendre (App. C) ---------------

GAUSS_CLOSED = {
    1: ([0.0], [2.0]),
    2: ([-1 / math.sqrt(3), 1 / math.sqrt(3)], [1.0, 1.0]),
    3: ([-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)], [5 / 9, 8 / 9, 5 / 9]),
    4: ([-math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5)), -math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)),
         math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)), math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))],
        [(18 - math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36,
         (18 + math.sqrt(30)) / 36, (18 - math.sqrt(30)) / 36]),
}

GLL_CLOSED = {
    2: ([-1.0, 1.0], [1.0, 1.0]),
    3: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    4: ([-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
}


@pytest.mark.parametrize("n", sorted(GAUSS_CLOSED))
def test_gauss_closed_forms(n):
    x, w = oracle.gauss(n)
    xr, wr = GAUSS_CLOSED[n]
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_exact_to_degree_2n_minus_1(n):
    x, w = oracle.gauss(n)
    assert w.sum() == pytest.approx(2.0, abs=1e-14)
    for p in range(2 * n):
        exact = 2.0 / (p + 1) if p % 2 == 0 else 0.0
        assert (w * x ** p).sum() == pytest.approx(exact, abs=1e-14)
    # ... and not beyond: degree 2n is integrated inexactly
    assert abs((w * x ** (2 * n)).sum() - 2.0 / (2 * n + 1)) > 1e-6


@pytest.mark.parametrize("m", sorted(GLL_CLOSED))
def test_gll_closed_forms(m):
    x, w = oracle.gll(m)
    xr, wr = GLL_CLOSED[m]
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-15)
    assert w.sum() == pytest.approx(2.0, abs=1e-14)
    for p in range(2 * m - 2):  # exact to degree 2m-3
        exact = 2.0 / (p + 1) if p % 2 == 0 else 0.0
        assert (w * x ** p).sum() == pytest.approx(exact, abs=1e-14)


def test_gll_first_weight_as_printed():
    for k, m, w1 in read_golden("gll_first_weight.txt"):
        k, m = int(k), int(m)
        assert m == math.ceil((k + 3) / 2)
        x, w = oracle.gll(m)
        assert w[0] == pytest.approx(frac(w1), abs=1e-15)


# --- basis (Sec. 2.2) ------------------------------------------------------------

@pytest.mark.parametrize("dim,k", [(2, 0), (2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_basis_count_and_order(dim, k):
    wl = workloads.workload("density_wave", dim=dim, k=k, n=(2, 2, 2))
    o = oracle.Oracle(wl)
    if dim == 3:
        assert o.N == (k + 1) * (k + 2) * (k + 3) // 6  # eq. nof_basis_functions
    else:
        assert o.N == (k + 1) * (k + 2) // 2
    e = o.exponents()
    assert sorted(map(tuple, e.tolist())) == sorted(
        t for t in itertools.product(range(k + 1), repeat=3)
        if sum(t) <= k and (dim == 3 or t[2] == 0))
    assert tuple(e[0]) == (0, 0, 0)  # phi_1 = 1, w_1 is the cell mean
    if k >= 1:
        for a in range(dim):
            unit = [0, 0, 0]; unit[a] = 1
            assert tuple(e[1 + a]) == tuple(unit)  # slopes w_2, w_3, w_4 (Sec. 3.1)
    deg = e.sum(axis=1)
    assert np.all(np.diff(deg) >= 0)


def test_2d_dof_per_cell_as_printed():
    for k, n in read_golden("dof_per_cell_2d.txt"):
        o = oracle.Oracle(workloads.workload("density_wave", dim=2, k=int(k), n=(2, 2, 1)))
        assert o.N == int(n)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_mass_matrix_is_identity(dim, k):
    # (1/|K|) int_K phi_i phi_j = delta_ij (eq. weights), with the oracle's own
    # (k+1)^d rule (exact: degree 2k <= 2k+1) and with an independent
    # numpy Gauss rule of higher order.
    o = oracle.Oracle(workloads.workload("density_wave", dim=dim, k=k, n=(2, 2, 2)))
    xi, wq = o.volume_rule()
    B = o.basis_at(xi)
    M = (B * wq[:, None]).T @ B / 2.0 ** dim
    np.testing.assert_allclose(M, np.eye(o.N), atol=2e-15)
    g, gw = np.polynomial.legendre.leggauss(k + 3)
    pts = np.array([p + (0.0,) * (3 - dim) for p in itertools.product(g, repeat=dim)])
    wts = np.array([np.prod(p) for p in itertools.product(gw, repeat=dim)])
    B2 = o.basis_at(pts)
    M2 = (B2 * wts[:, None]).T @ B2 / 2.0 ** dim
    np.testing.assert_allclose(M2, np.eye(o.N), atol=2e-14)


def test_basis_is_product_of_scaled_legendre():
    # phi = Ptilde_u(x) Ptilde_v(y) Ptilde_w(z) with Ptilde_n = sqrt(2n+1) P_n,
    # checked against numpy's Legendre series evaluation at random points.
    o = oracle.Oracle(workloads.workload("density_wave", dim=3, k=3, n=(2, 2, 2)))
    e = o.exponents()
    rng = np.random.default_rng(3)
    pts = rng.uniform(-1, 1, size=(20, 3))
    B = o.basis_at(pts)
    for l in range(o.N):
        ref = np.ones(len(pts))
        for a in range(3):
            c = np.zeros(e[l, a] + 1); c[-1] = 1.0
            ref *= math.sqrt(2 * e[l, a] + 1) * np.polynomial.legendre.legval(pts[:, a], c)
        np.testing.assert_allclose(B[:, l], ref, rtol=1e-13, atol=1e-13)


def test_union_points_rule_exact_for_degree_k():
    # The union set S of eq. union_quad_points: each S_a with the tensor
    # (GLL in a) x (Gauss elsewhere) weights integrates degree-k polynomials
    # exactly, so the cell mean is a convex combination of values on S.
    for dim, k in [(2, 1), (2, 2), (3, 2), (3, 3)]:
        o = oracle.Oracle(workloads.workload("density_wave", dim=dim, k=k, n=(2, 2, 2)))
        S = o.positivity_points()
        assert S.shape[0] == dim * o.m * (k + 1) ** (dim - 1)
        gx, gw = oracle.gauss(k + 1)
        lx, lw = oracle.gll(o.m)
        B = o.basis_at(S)
        per = o.m * (k + 1) ** (dim - 1)
        for a in range(dim):
            block = S[a * per:(a + 1) * per]
            wts = np.ones(per)
            for i, p in enumerate(block):
                for b in range(dim):
                    if b == a:
                        wts[i] *= lw[np.argmin(abs(lx - p[b]))]
                    else:
                        wts[i] *= gw[np.argmin(abs(gx - p[b]))]
            # mean of phi_l over the cell: 1 for l = 0, else 0
            means = (B[a * per:(a + 1) * per] * wts[:, None]).sum(axis=0) / 2.0 ** dim
            expect = np.zeros(o.N); expect[0] = 1.0
            np.testing.assert_allclose(means, expect, atol=1e-14)
