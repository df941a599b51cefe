"""Pins of the oracle on the static 2:1 refined box (Sec. 4: hanging-face
quadrature; Sec. 4.2 and App. F: refinement matrices; Sec. 4.4: limiting at
refinement boundaries)."""
import numpy as np
import pytest

import oracle
import workloads


def _amr(dim=3, k=2, n=(8, 8, 8), lo=(2, 3, 2), hi=(6, 6, 5), **kw):
    h = 1.0 / 8.0
    wl = workloads.workload("blast_amr", dim=dim, k=k, n=n, length=tuple(h * m for m in n),
                            refine_lo=lo, refine_hi=hi, limiter=0, positivity=0, **kw)
    return wl


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (3, 1), (3, 2), (3, 3)])
def test_refinement_matrices(dim, k):
    # (1/2^d) sum_c P_c^T P_c = I and P_c reproduces the coarse polynomial on
    # the child (eq. ref_pa_integral with the coarse basis at the mapped point)
    o = oracle.AmrOracle(_amr(dim=dim, k=k, n=(4, 4, 4), lo=(1, 1, 1), hi=(3, 3, 3)))
    nch = 2 ** dim
    Ps = [o.refine_matrix(c) for c in range(nch)]
    M = sum(P.T @ P for P in Ps) / nch
    np.testing.assert_allclose(M, np.eye(o.N), atol=1e-14)
    rng = np.random.default_rng(1)
    w = rng.uniform(-1, 1, o.N)
    pts = rng.uniform(-1, 1, size=(10, 3))
    if dim == 2:
        pts[:, 2] = 0.0
    for c in range(nch):
        sig = np.array([1.0 if (c >> a) & 1 else -1.0 for a in range(3)])
        mapped = 0.5 * (pts + sig)
        if dim == 2:
            mapped[:, 2] = 0.0
        coarse = o.basis_at(mapped) @ w
        child = o.basis_at(pts) @ (Ps[c] @ w)
        np.testing.assert_allclose(child, coarse, atol=1e-13)


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 1), (3, 2)])
def test_free_stream_on_refined_mesh(dim, k):
    wl = _amr(dim=dim, k=k, ic="uniform", state=(1.2, (0.3, -0.5, 0.2), 0.9))
    o = oracle.AmrOracle(wl)
    L = o.rhs(o.initial_state())
    assert np.abs(L).max() < 1e-12


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 2)])
def test_conservation_across_the_interface(dim, k):
    wl = _amr(dim=dim, k=k, ic="vortex", noise=0.0, x0=(-0.5, -0.5, -0.5))
    o = oracle.AmrOracle(wl)
    w = o.initial_state()
    rng = np.random.default_rng(3)
    w = w + 0.01 * rng.uniform(-1, 1, w.shape) * np.abs(w).max() * 0.01
    L = o.rhs(w)
    Lc, Lf = o.blocks(L)
    d = dim
    tot = Lc[:, 0, ~o.hole].sum(axis=1) * o.dx ** d + Lf[:, 0, :].sum(axis=1) * o.dxf ** d
    scale = np.abs(Lc[:, 0, ~o.hole]).sum(axis=1) * o.dx ** d + np.abs(Lf[:, 0, :]).sum(axis=1) * o.dxf ** d
    assert np.all(np.abs(tot) <= 1e-13 * scale), (tot, scale)


def _poly(k):
    terms = [(1.0, 0, 0, 0), (0.3, 1, 0, 0), (-0.2, 0, 1, 0), (0.25, 0, 0, 1)]
    if k >= 2:
        terms += [(0.15, 1, 1, 0), (-0.1, 0, 2, 0), (0.12, 1, 0, 1)]
    return terms


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_polynomial_contact_matches_uniform_grids(dim, k):
    # For a globally polynomial contact state of degree <= k the traces agree
    # across every face and the flux is polynomial, so every face quadrature
    # (coarse, fine, or the 2^(d-1) hanging fine faces) is exact: the refined
    # mesh must reproduce the uniform coarse-grid RHS on coarse cells and the
    # uniform fine-grid RHS on fine cells, away from the (non-periodic)
    # domain boundary.
    n = (8, 8, 8) if dim == 3 else (8, 8, 1)
    lo, hi = (2, 3, 2), (6, 6, 5)
    common = dict(ic="poly_contact", poly=_poly(k), velocity=(0.7, -0.4, 0.3), x0=(0.0, 0.0, 0.0))
    wl = _amr(dim=dim, k=k, n=n, lo=lo, hi=hi, **common)
    o = oracle.AmrOracle(wl)
    L = o.rhs(o.initial_state())
    Lc, Lf = o.blocks(L)
    h = 1.0 / 8.0
    uc = oracle.Oracle(workloads.workload("density_wave", dim=dim, k=k, n=n, length=tuple(h * m for m in n),
                                          **common))
    Luc = uc.rhs(uc.initial_state()).reshape(o.nvar, o.N, -1)
    n2 = tuple(2 * m if a < dim else 1 for a, m in enumerate(n))
    uf = oracle.Oracle(workloads.workload("density_wave", dim=dim, k=k, n=n2, length=tuple(h / 2 * m for m in n2),
                                          **common))
    Luf = uf.rhs(uf.initial_state()).reshape(o.nvar, o.N, -1)
    # coarse cells away from the box boundary of the domain
    cid = np.arange(o.ncoarse)
    ci = [cid % n[0], (cid // n[0]) % n[1], cid // (n[0] * n[1])]
    interior = ~o.hole
    for a in range(dim):
        interior &= (ci[a] >= 1) & (ci[a] <= n[a] - 2)
    scale = np.abs(Luc[:, :, interior]).max()
    np.testing.assert_allclose(Lc[:, :, interior], Luc[:, :, interior], atol=1e-11 * scale)
    # fine cells: map to the uniform fine grid
    fid = np.arange(o.nfine)
    nf = o.nf
    fi = [fid % nf[0], (fid // nf[0]) % nf[1], fid // (nf[0] * nf[1])]
    g = [2 * lo[a] + fi[a] if a < dim else 0 * fi[a] for a in range(3)]
    gidx = (g[2] * n2[1] + g[1]) * n2[0] + g[0]
    scale = np.abs(Luf[:, :, gidx]).max()
    np.testing.assert_allclose(Lf, Luf[:, :, gidx], atol=1e-11 * scale)
    # the hanging faces actually carry flux
    assert np.abs(Lf).max() > 1e-3


def test_limiter_on_refined_mesh_keeps_means_and_positivity():
    wl = _amr(dim=3, k=3, n=(8, 8, 8), lo=(2, 2, 2), hi=(6, 6, 6), ic="blast")
    wl = dict(wl, limiter=1, positivity=1)
    o = oracle.AmrOracle(wl)
    w = o.initial_state()
    out, st = o.limit(w)
    assert st == 0
    wc0, wf0 = o.blocks(w)
    wc1, wf1 = o.blocks(out)
    np.testing.assert_array_equal(wc1[:, 0], wc0[:, 0])
    np.testing.assert_array_equal(wf1[:, 0], wf0[:, 0])
    # a few steps stay positive and conservative
    tot0 = o.totals(out)
    w = out
    for _ in range(3):
        w, _ = o.step(w)
    np.testing.assert_allclose(o.totals(w), tot0, rtol=1e-12, atol=1e-14)
