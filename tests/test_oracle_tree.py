"""Pins of the oracle's 2D quadtree path (Sec. 4: leaves of any depth, level
jump at most one across a face) against results fixed independently of it:

* a tree whose leaves all sit on one level is a uniform grid: its RHS equals
  the uniform oracle's (base grid, or the grid of twice the resolution);
* a tree shaped like one 2:1 box equals the refined-box oracle, whose
  hanging-face quadrature is pinned on its own;
* on any periodic tree the face fluxes cancel in the area-weighted sum of the
  cell means (conservation), and a constant state has L = 0;
* the time step of a one-level tree equals the uniform oracle's, and halves
  when every leaf is split.
"""
import numpy as np
import pytest

import oracle
import workloads


def _wl(n=(6, 5), k=2, ic="vortex", **kw):
    base = dict(n=(n[0], n[1], 1), length=(10.0 * n[0] / max(n), 10.0 * n[1] / max(n), 1.0),
                x0=(-5.0, -5.0, 0.0), k=k, limiter=0, positivity=0)
    base.update(kw)
    return workloads.workload("vortex", **base) if ic == "vortex" else workloads.workload(ic, **base)


def _grid_leaves(n, level):
    nx, ny = n[0] << level, n[1] << level
    return np.array([(level, x, y) for y in range(ny) for x in range(nx)], dtype=np.int64)


def _close(a, b, tol):
    a = np.asarray(a).reshape(a.shape[0], -1) if a.ndim > 1 else a
    scale = np.abs(b).reshape(b.shape[0], -1).max(axis=1, keepdims=True)
    err = np.abs(np.asarray(a).reshape(b.shape[0], -1) - b.reshape(b.shape[0], -1)) / scale
    assert err.max() <= tol, err.max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_one_level_tree_is_the_uniform_grid(k):
    wl = _wl(k=k)
    u = oracle.Oracle(wl)
    w = u.initial_state()
    t = oracle.TreeOracle(wl, _grid_leaves((6, 5), 0))
    Lu = u.rhs(w).reshape(u.nvar, u.N, -1)
    Lt = t.rhs(w.reshape(u.nvar, u.N, -1))
    _close(Lt, Lu, 1e-14)
    assert t.max_dt(w.reshape(u.nvar, u.N, -1)) == pytest.approx(u.max_dt(w), rel=1e-15)


@pytest.mark.parametrize("k", [1, 3])
def test_split_tree_is_the_fine_grid(k):
    """Every base cell split once: the uniform grid of twice the resolution."""
    wl = _wl(k=k)
    fine = dict(wl, n=(12, 10, 1))
    u = oracle.Oracle(fine)
    w = u.initial_state()
    t = oracle.TreeOracle(wl, _grid_leaves((6, 5), 1))
    wt = w.reshape(u.nvar, u.N, -1)
    _close(t.rhs(wt), u.rhs(w).reshape(u.nvar, u.N, -1), 1e-14)
    assert t.max_dt(wt) == pytest.approx(u.max_dt(w), rel=1e-15)
    coarse = oracle.TreeOracle(wl, _grid_leaves((6, 5), 0))
    wc = oracle.Oracle(wl).initial_state().reshape(u.nvar, u.N, -1)
    assert coarse.max_dt(wc) > t.max_dt(wt)


@pytest.mark.parametrize("k,bc", [(1, (0, 0, 0)), (2, (0, 0, 0)), (3, (1, 0, 0)), (2, (1, 1, 0))])
def test_box_shaped_tree_is_the_refined_box(k, bc):
    n, lo, hi = (8, 6), (2, 1), (5, 4)
    wl = _wl(n=n, k=k, bc=bc, refine_lo=(lo[0], lo[1], 0), refine_hi=(hi[0], hi[1], 1))
    box = oracle.AmrOracle(wl)
    w = box.initial_state()
    wc, wf = box.blocks(w)
    leaves, cols = [], []
    for c in range(box.ncoarse):
        x, y = c % n[0], c // n[0]
        if not box.hole[c]:
            leaves.append((0, x, y)); cols.append(("c", c))
    nfx = box.nf[0]
    for f in range(box.nfine):
        fx, fy = f % nfx, f // nfx
        leaves.append((1, 2 * lo[0] + fx, 2 * lo[1] + fy)); cols.append(("f", f))
    wt = np.stack([wc[:, :, i] if b == "c" else wf[:, :, i] for b, i in cols], axis=2)
    t = oracle.TreeOracle(dict(wl, refine_lo=(0, 0, 0), refine_hi=(0, 0, 0)), np.array(leaves))
    Lc, Lf = box.blocks(box.rhs(w))
    Lb = np.stack([Lc[:, :, i] if b == "c" else Lf[:, :, i] for b, i in cols], axis=2)
    _close(t.rhs(wt), Lb, 1e-14)
    assert t.max_dt(wt) == pytest.approx(box.max_dt(w), rel=1e-15)


@pytest.mark.parametrize("seed,k", [(3, 1), (11, 2), (5, 3)])
def test_random_tree_conserves_and_keeps_free_stream(seed, k):
    n = (4, 4)
    wl = _wl(n=n, k=k)
    leaves = workloads.random_tree(n, 3, 0.45, seed)
    assert leaves[:, 0].max() == 3
    t = oracle.TreeOracle(wl, leaves)
    w = t.initial_state()
    L = t.rhs(w)
    area = (wl["length"][0] / n[0] / 2.0 ** leaves[:, 0]) ** 2
    total = (L[:, 0, :] * area).sum(axis=1)
    scale = (np.abs(L[:, 0, :]) * area).sum(axis=1)
    assert np.all(np.abs(total) <= 1e-13 * scale), total / scale
    # a constant state: every trace equals it, fluxes cancel, V is zero
    wc = np.zeros_like(w)
    wc[:, 0, :] = np.array([1.3, 0.4, -0.7, 3.1])[:, None]
    assert np.abs(t.rhs(wc)).max() <= 1e-12


def test_tree_rejects_gaps_and_overlaps():
    wl = _wl(n=(2, 2))
    good = _grid_leaves((2, 2), 0)
    with pytest.raises(RuntimeError):
        oracle.TreeOracle(wl, good[:3]).rhs(np.zeros((4, 6, 3)))
    bad = np.concatenate([good, [[1, 0, 0]]])
    with pytest.raises(RuntimeError):
        oracle.TreeOracle(wl, bad).rhs(np.zeros((4, 6, 5)))


def _balanced(leaves, n):
    """Brute force: every pair of leaves that touch (faces or corners, periodic)
    differs by at most one level."""
    lv = np.asarray(leaves)
    L = lv[:, 0].max()
    s = 1 << (L - lv[:, 0])
    x0, y0 = lv[:, 1] * s, lv[:, 2] * s
    NX, NY = n[0] << L, n[1] << L
    for i in range(len(lv)):
        for j in range(i + 1, len(lv)):
            if abs(lv[i, 0] - lv[j, 0]) <= 1:
                continue
            for ox in (-NX, 0, NX):
                for oy in (-NY, 0, NY):
                    if (x0[i] <= x0[j] + ox + s[j] and x0[j] + ox <= x0[i] + s[i]
                            and y0[i] <= y0[j] + oy + s[j] and y0[j] + oy <= y0[i] + s[i]):
                        return False
    return True


def test_adapt_refines_flagged_leaves_with_a_buffer_and_balances():
    n = (10, 10)
    wl = _wl(n=n, k=2, ic="kh2d", length=(1.0, 1.0, 1.0), x0=(0.0, 0.0, 0.0))
    t = oracle.TreeOracle(wl, _grid_leaves(n, 0))
    w = t.initial_state()
    new, w1 = oracle.tree_adapt(wl, t.leaves, w, max_level=2)
    assert _balanced(new, n)
    flagged = np.maximum(np.abs(w[0, 1]), np.abs(w[0, 2])) > 1.1 * 0.01
    assert flagged.any() and not flagged.all()
    have = {tuple(r) for r in new}
    for i in np.flatnonzero(flagged):
        l, x, y = t.leaves[i]
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                xx, yy = (x + dx) % n[0], (y + dy) % n[1]
                assert (0, xx, yy) not in have  # the flagged leaf and its buffer ring are split
    # a second pass may refine to level 2, still balanced
    t1 = oracle.TreeOracle(wl, new)
    new2, w2 = oracle.tree_adapt(wl, new, w1, max_level=2)
    assert new2[:, 0].max() == 2 and _balanced(new2, n)
    # the projections keep mass, momentum and energy: sum of area * mean
    for (lvs, ws), (lvb, wb) in (((t.leaves, w), (new, w1)), ((new, w1), (new2, w2))):
        a0 = (0.25 ** lvs[:, 0] * ws[:, 0, :]).sum(axis=1)
        a1 = (0.25 ** lvb[:, 0] * wb[:, 0, :]).sum(axis=1)
        assert np.all(np.abs(a0 - a1) <= 1e-14 * np.abs(a0).max())
    assert t1.nleaf == len(new)


def test_adapt_merges_smooth_groups_and_refine_merge_is_identity():
    """A state with no density slope merges every complete sibling group whose
    neighbours allow it; splitting a leaf and merging its children gives its
    polynomial back (degree k is exact on the children)."""
    n = (4, 4)
    wl = _wl(n=n, k=3, ic="kh2d", length=(1.0, 1.0, 1.0), x0=(0.0, 0.0, 0.0))
    leaves = workloads.random_tree(n, 2, 0.5, 9)
    t = oracle.TreeOracle(wl, leaves)
    w = t.initial_state()
    flat = w.copy()
    flat[:, 1:, :] = 0.0
    new, wn = oracle.tree_adapt(wl, leaves, flat, max_level=2)
    assert len(new) < len(leaves) and _balanced(new, n)
    # refine everything once from a coarse mesh, then merge back: w returns
    base = _grid_leaves(n, 0)
    tb = oracle.TreeOracle(wl, base)
    wb = tb.initial_state()
    P = oracle._tree_refine_mats(wl)
    kids = np.stack([(P[c] @ wb[:, :, i].T).T for i in range(len(base)) for c in range(4)], axis=2)
    kl = np.array([(1, 2 * x + (c & 1), 2 * y + (c >> 1)) for (_, x, y) in base for c in range(4)])
    back, wback = oracle.tree_adapt(wl, kl, np.where(np.arange(wb.shape[1])[None, :, None] == 0, kids, 0.0),
                                    wt=1e9, max_level=1)
    assert len(back) == len(base)
    # merging the projected children of the means alone returns the means
    order = {tuple(r): i for i, r in enumerate(base)}
    idx = [order[tuple(r)] for r in back]
    assert np.allclose(wback[:, 0, :], wb[:, 0, idx], rtol=1e-14, atol=1e-15)
    node = sum(P[c].T @ kids[:, :, 4 * 5 + c].T for c in range(4)).T / 4.0
    assert np.allclose(node, wb[:, :, 5], rtol=0, atol=1e-13)


@pytest.mark.parametrize("limiter", [1, 2])
def test_one_level_tree_limiter_is_the_uniform_limiter(limiter):
    n = (10, 10)
    wl = _wl(n=n, k=2, ic="kh2d", length=(1.0, 1.0, 1.0), x0=(0.0, 0.0, 0.0), limiter=limiter, positivity=1,
             eps=1e-8)
    u = oracle.Oracle(wl)
    w = u.initial_state()
    ref, st = u.limit(w)
    t = oracle.TreeOracle(wl, _grid_leaves(n, 0))
    got, st2 = t.limit(w.reshape(u.nvar, u.N, -1))
    assert st == st2 == 0
    assert np.abs(ref.reshape(got.shape) - w.reshape(got.shape)).max() > 1e-3  # the limiters act
    assert np.array_equal(got, ref.reshape(got.shape))


@pytest.mark.parametrize("k,limiter,bc", [(2, 1, (0, 0, 0)), (3, 2, (0, 0, 0)), (2, 2, (1, 1, 0))])
def test_box_shaped_tree_limiter_is_the_refined_box_limiter(k, limiter, bc):
    """Neighbour means across the refinement boundary (children's average on
    the coarse side, the coarse polynomial's mean over the adjacent child on
    the fine side) and the extra positivity points of the hanging faces."""
    # the box's x faces cross the lower shear layer; eps just below the outer
    # density makes the positivity limiter act near the jump
    n, lo, hi = (10, 10), (2, 1), (6, 4)
    wl = _wl(n=n, k=k, ic="kh2d", length=(1.0, 1.0, 1.0), x0=(0.0, 0.0, 0.0), bc=bc, limiter=limiter,
             positivity=1, eps=0.95, refine_lo=(lo[0], lo[1], 0), refine_hi=(hi[0], hi[1], 1))
    box = oracle.AmrOracle(wl)
    w = box.initial_state()
    wc, wf = box.blocks(w)
    leaves, cols = [], []
    for c in range(box.ncoarse):
        if not box.hole[c]:
            leaves.append((0, c % n[0], c // n[0])); cols.append(("c", c))
    for f in range(box.nfine):
        leaves.append((1, 2 * lo[0] + f % box.nf[0], 2 * lo[1] + f // box.nf[0])); cols.append(("f", f))
    pick = lambda x: np.stack([x[0][:, :, i] if b == "c" else x[1][:, :, i] for b, i in cols], axis=2)
    ref, st = box.limit(w)
    t = oracle.TreeOracle(dict(wl, refine_lo=(0, 0, 0), refine_hi=(0, 0, 0)), np.array(leaves))
    got, st2 = t.limit(pick((wc, wf)))
    r = pick(box.blocks(ref))
    assert st == st2 == 0
    assert np.abs(r - pick((wc, wf))).max() > 1e-3
    scale = np.abs(r).reshape(r.shape[0], -1).max(axis=1)[:, None, None]
    assert np.abs(got - r).max(axis=(1, 2)).max() <= 0 or np.all(np.abs(got - r) <= 1e-13 * scale)


def test_tree_positivity_checks_the_hanging_face_points():
    """A coarse leaf next to finer ones whose density dips lowest at a trace
    point of a half face (eta = (0.86 + 1)/2 = 0.93, k = 3), which is none of
    the union points S (Gauss 0.34, 0.86 and GLL 0, 1 in y): with eps between
    the dip and the lowest S value only the extra points of Sec. 4.4 make the
    limiter act; the box oracle, pinned on its own, agrees."""
    n, lo, hi = (6, 6), (2, 2), (4, 4)
    wl = _wl(n=n, k=3, ic="kh2d", length=(1.0, 1.0, 1.0), x0=(0.0, 0.0, 0.0), limiter=0, positivity=1,
             eps=0.52, refine_lo=(lo[0], lo[1], 0), refine_hi=(hi[0], hi[1], 1))
    box = oracle.AmrOracle(wl)
    xi, _ = oracle.Oracle(dict(wl, refine_lo=(0, 0, 0), refine_hi=(0, 0, 0))).volume_rule()
    g, _ = oracle.gauss(4)
    eta = 0.5 * (g.max() + 1.0)
    ncell = box.ncoarse + box.nfine
    prim = np.zeros((ncell, box.Q, 5))
    prim[..., 0] = 1.0
    prim[..., 4] = 2.5
    target = [c for c in range(box.ncoarse) if c % n[0] == lo[0] - 1 and lo[1] <= c // n[0] < hi[1]]
    for c in target:  # coarse leaves on the box's low x face
        prim[c, :, 0] = 1.0 + 10.0 * ((xi[:, 1] - eta) ** 2 - 0.05)
    w = np.zeros(box.size)
    lib, _ = oracle._load()
    assert lib.orc_amr_project(oracle.C.byref(box.c), np.ascontiguousarray(prim), w) == 0
    ref, st = box.limit(w)
    assert st == 0
    wc, wf = box.blocks(w)
    rc, _ = box.blocks(ref)
    assert np.abs(rc[:, :, target] - wc[:, :, target]).max() > 1e-3  # the box limiter acts there
    leaves, cols = [], []
    for c in range(box.ncoarse):
        if not box.hole[c]:
            leaves.append((0, c % n[0], c // n[0])); cols.append(("c", c))
    for f in range(box.nfine):
        leaves.append((1, 2 * lo[0] + f % box.nf[0], 2 * lo[1] + f // box.nf[0])); cols.append(("f", f))
    pick = lambda x: np.stack([x[0][:, :, i] if b == "c" else x[1][:, :, i] for b, i in cols], axis=2)
    t = oracle.TreeOracle(dict(wl, refine_lo=(0, 0, 0), refine_hi=(0, 0, 0)), np.array(leaves))
    got, st2 = t.limit(pick((wc, wf)))
    r = pick(box.blocks(ref))
    assert st2 == 0
    assert np.all(np.abs(got - r) <= 1e-13 * np.abs(r).max())
    # the same leaves on a one-level mesh (no finer neighbour): nothing to do
    flat = oracle.TreeOracle(dict(wl, refine_lo=(0, 0, 0), refine_hi=(0, 0, 0)), _grid_leaves(n, 0))
    wu = np.where(box.hole[None, None, :], wc[:, :, [0]], wc)  # hole cells: a plain cell's state
    gotu, _ = flat.limit(wu)
    assert np.array_equal(gotu[:, :, target], wc[:, :, target])


def test_per_leaf_entries_equal_whole_mesh_calls():
    n = (10, 10)
    wl = _wl(n=n, k=2, ic="kh2d", length=(1.0, 1.0, 1.0), x0=(0.0, -0.01, 0.0), limiter=2, positivity=1, eps=0.95)
    leaves = workloads.random_tree(n, 3, 0.4, 17)
    t = oracle.TreeOracle(wl, leaves)
    w = t.initial_state()
    cells = np.array([0, 5, 17, len(leaves) // 2, len(leaves) - 1])
    V, S, A = t.terms(w)
    Vc, Sc, Ac = t.terms_cells(w, cells)
    assert np.array_equal(Vc, V[:, :, cells]) and np.array_equal(Sc, S[:, :, cells]) and np.array_equal(Ac, A[:, :, cells])
    full, st = t.limit(w)
    part, st2 = t.limit_cells(w, cells)
    assert st == st2 == 0 and np.array_equal(part, full[:, :, cells])
