"""2D quadtree meshes on the GPU (Sec. 4: leaves of any depth, hanging faces,
refinement criterion, refine/derefine projections) against the oracle's
quadtree path, under the comparison rules of tests/parity.py."""
import numpy as np
import pytest
import torch

import oracle
import paper_1506_06140_amd as dg
import workloads
from parity import check_rhs_modes, check_state_modes, say

pytestmark = pytest.mark.gpu


def _vortex(n, k, **kw):
    base = dict(n=(n[0], n[1], 1), length=(10.0 * n[0] / max(n), 10.0 * n[1] / max(n), 1.0),
                x0=(-5.0, -5.0, 0.0), k=k, limiter=0, positivity=0)
    base.update(kw)
    return workloads.workload("vortex", **base)


def _kh(n, k, **kw):
    base = dict(n=(n[0], n[1], 1), k=k, limiter=0, positivity=0, rk="rk3")
    base.update(kw)
    return workloads.workload("kh2d", **base)


CASES = {
    "k1_random3": (lambda: _vortex((6, 5), 1), lambda: workloads.random_tree((6, 5), 3, 0.45, 3)),
    "k2_random3": (lambda: _vortex((6, 5), 2), lambda: workloads.random_tree((6, 5), 3, 0.45, 11)),
    "k3_random3": (lambda: _vortex((6, 5), 3), lambda: workloads.random_tree((6, 5), 3, 0.45, 5)),
    "k2_walls": (lambda: _vortex((6, 5), 2, bc=(1, 1, 0)), lambda: workloads.random_tree((6, 5), 3, 0.5, 21,
                                                                                          periodic=(False, False))),
    "k3_davis_kh": (lambda: _kh((10, 10), 3, flux=1), lambda: workloads.band_tree((10, 10), 3)),
    "k2_random4_large": (lambda: _vortex((16, 16), 2), lambda: workloads.random_tree((16, 16), 4, 0.35, 2)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_tree_rhs_matches_oracle(case):
    wl = CASES[case][0]()
    leaves = CASES[case][1]()
    say(case, "leaves", len(leaves), "per level", np.bincount(leaves[:, 0]))
    o = oracle.TreeOracle(wl, leaves)
    w = o.initial_state()
    V, S, A = o.terms(w)
    s = dg.TreeSolver(wl, leaves)
    assert np.array_equal(s.leaves, leaves)
    L = s.rhs(torch.from_numpy(w).cuda()).cpu().numpy()
    assert s.status() == 0
    check_rhs_modes(L, V, S, A, case)


@pytest.mark.parametrize("case", ["k1_random3", "k3_random3", "k2_walls", "k3_davis_kh"])
def test_tree_steps_match_oracle(case):
    wl = CASES[case][0]()
    leaves = CASES[case][1]()
    o = oracle.TreeOracle(wl, leaves)
    w = o.initial_state()
    s = dg.TreeSolver(wl, leaves)
    wg = torch.from_numpy(w).cuda()
    bufs = [s.empty() for _ in range(3)] + [s.scalar()]
    ref = w
    for it in range(3):
        ref, dt = o.step(ref)
        out = s.step(wg, bufs)
        dtg = float(bufs[3].item())
        assert dtg == pytest.approx(dt, rel=1e-14), (dtg, dt)
        check_state_modes(out.cpu().numpy(), ref, f"{case} step {it + 1}")
        wg = out.clone()
    assert s.status() == 0


def _refined_fraction(leaves):
    return float((0.25 ** leaves[:, 0] * (leaves[:, 0] > 0)).sum() / (0.25 ** leaves[:, 0]).sum())


@pytest.mark.parametrize("n,start,max_level,steps", [((10, 10), 1, 3, 4), ((16, 16), 2, 4, 2)])
def test_adaptive_kh_matches_oracle_step_for_step(n, start, max_level, steps):
    """The KH setup (Validation, KH instability) on a quadtree that adapts
    before every step (Sec. 4.1-4.3, wt = 0.01, alpha = 1.1): the GPU's leaf
    sets equal the oracle's exactly and the states agree under the parity
    rules, step after step."""
    # origin shifted by a fraction of the finest cell, so that the shear
    # layers cut cells on every level (on a face the density has no slope)
    wl = _kh(n, 3, x0=(0.0, -0.01, 0.0))
    leaves = workloads.band_tree(n, start)
    o = oracle.TreeOracle(wl, leaves)
    w = o.initial_state()
    s = dg.TreeSolver(wl, leaves)
    wg = torch.from_numpy(w).cuda()
    for it in range(steps):
        leaves_o, w = oracle.tree_adapt(wl, o.leaves, w, 0.01, 1.1, max_level)
        wg = s.adapt(wg, 0.01, 1.1, max_level)
        assert np.array_equal(s.leaves, leaves_o), f"mesh differs after adaptation {it + 1}"
        check_state_modes(wg.cpu().numpy(), w, f"regrid {it + 1}")
        o = oracle.TreeOracle(wl, leaves_o)
        w, dt = o.step(w)
        bufs = [s.empty() for _ in range(3)] + [s.scalar()]
        out = s.step(wg, bufs)
        assert float(bufs[3].item()) == pytest.approx(dt, rel=1e-14)
        check_state_modes(out.cpu().numpy(), w, f"step {it + 1}")
        wg = out.clone()
        say(f"step {it + 1}: {len(leaves_o)} leaves, per level {np.bincount(leaves_o[:, 0])}, "
            f"refined area fraction {_refined_fraction(leaves_o):.3f}")
    assert s.leaves[:, 0].max() == max_level
    assert s.status() == 0


def test_tree_set_rejects_invalid_meshes():
    wl = _vortex((4, 4), 2)
    good = np.array([(0, x, y) for y in range(4) for x in range(4)])
    s = dg.TreeSolver(wl, good)
    gap = good[1:]
    overlap = np.concatenate([good, [[1, 0, 0]]])
    jump = np.concatenate([good[good[:, 1] + 4 * good[:, 2] != 5],
                           [(2, 4 + (q & 3), 4 + (q >> 2)) for q in range(16)]])
    for bad in (gap, overlap, jump):
        with pytest.raises(dg.DGError):
            s.set_leaves(bad)
    s.set_leaves(good)
    assert s.nleaf == 16


LIMITED = {
    # KH with the shear layers cutting cells; eps just below the outer density
    # makes the positivity limiter act near the jumps
    "k2_minmod_random3": (lambda: _kh((10, 10), 2, limiter=1, positivity=1, eps=0.95, x0=(0.0, -0.01, 0.0)),
                          lambda: workloads.random_tree((10, 10), 3, 0.4, 17)),
    "k3_char_band3": (lambda: _kh((10, 10), 3, limiter=2, positivity=1, eps=0.95, x0=(0.0, -0.01, 0.0)),
                      lambda: workloads.band_tree((10, 10), 3)),
    "k1_minmod_walls": (lambda: _kh((10, 10), 1, limiter=1, positivity=1, eps=0.95, bc=(1, 1, 0),
                                    x0=(0.0, -0.01, 0.0)),
                        lambda: workloads.random_tree((10, 10), 2, 0.5, 4, periodic=(False, False))),
}


@pytest.mark.parametrize("case", list(LIMITED))
def test_tree_limiter_matches_oracle(case):
    wl = LIMITED[case][0]()
    leaves = LIMITED[case][1]()
    o = oracle.TreeOracle(wl, leaves)
    w = o.initial_state()
    ref, st = o.limit(w)
    assert st == 0
    assert np.abs(ref - w).max() > 1e-3
    s = dg.TreeSolver(wl, leaves)
    got = s.limit(torch.from_numpy(w).cuda()).cpu().numpy()
    assert s.status() == 0
    check_state_modes(got, ref, case)
    assert np.array_equal(got[:, 0], w[:, 0])  # means are never changed


@pytest.mark.parametrize("case", list(LIMITED))
def test_tree_limited_steps_match_oracle(case):
    wl = LIMITED[case][0]()
    leaves = LIMITED[case][1]()
    o = oracle.TreeOracle(wl, leaves)
    w = o.initial_state()
    s = dg.TreeSolver(wl, leaves)
    wg = torch.from_numpy(w).cuda()
    bufs = [s.empty() for _ in range(3)] + [s.scalar()]
    ref = w
    for it in range(2):
        ref, dt = o.step(ref)
        out = s.step(wg, bufs)
        assert float(bufs[3].item()) == pytest.approx(dt, rel=1e-14)
        check_state_modes(out.cpu().numpy(), ref, f"{case} limited step {it + 1}")
        wg = out.clone()
    assert s.status() == 0


def test_tree_positivity_at_hanging_face_points():
    """A coarse leaf next to finer ones whose density dips lowest at a trace
    point of a half face, not at a union point: only the extra points of the
    refinement boundary make the positivity limiter act (oracle pin
    test_tree_positivity_checks_the_hanging_face_points, same input)."""
    n = (6, 6)
    wl = _kh(n, 3, limiter=0, positivity=1, eps=0.52)
    leaves = [(0, x, y) for y in range(6) for x in range(6) if not (2 <= x < 4 and 2 <= y < 4)]
    leaves += [(1, x, y) for y in range(4, 8) for x in range(4, 8)]
    leaves = np.array(leaves)
    o = oracle.TreeOracle(wl, leaves)
    xi, _ = o.volume_rule()
    g, _ = oracle.gauss(4)
    eta = 0.5 * (g.max() + 1.0)
    prim = np.zeros((len(leaves), o.Q, 5))
    prim[..., 0] = 1.0
    prim[..., 4] = 2.5
    target = [i for i, (l, x, y) in enumerate(leaves) if l == 0 and x == 1 and 2 <= y < 4]
    for i in target:
        prim[i, :, 0] = 1.0 + 10.0 * ((xi[:, 1] - eta) ** 2 - 0.05)
    w = o.project_prim(prim)
    ref, st = o.limit(w)
    assert st == 0 and np.abs(ref[:, :, target] - w[:, :, target]).max() > 1e-3
    s = dg.TreeSolver(wl, leaves)
    got = s.limit(torch.from_numpy(w).cuda()).cpu().numpy()
    check_state_modes(got, ref, "hanging-face positivity")


def test_adaptive_limited_kh_matches_oracle():
    """The KH run as the paper sets it up (characteristic limiter and
    positivity after every stage, adaptation before every step), three steps
    to four levels."""
    n = (10, 10)
    wl = _kh(n, 3, limiter=2, positivity=1, eps=1e-8, x0=(0.0, -0.01, 0.0))
    leaves = workloads.band_tree(n, 1)
    o = oracle.TreeOracle(wl, leaves)
    w = o.initial_state()
    s = dg.TreeSolver(wl, leaves)
    wg = torch.from_numpy(w).cuda()
    for it in range(3):
        leaves_o, w = oracle.tree_adapt(wl, o.leaves, w, 0.01, 1.1, 3)
        wg = s.adapt(wg, 0.01, 1.1, 3)
        assert np.array_equal(s.leaves, leaves_o)
        o = oracle.TreeOracle(wl, leaves_o)
        w, dt = o.step(w)
        bufs = [s.empty() for _ in range(3)] + [s.scalar()]
        wg = s.step(wg, bufs).clone()
        check_state_modes(wg.cpu().numpy(), w, f"limited adaptive step {it + 1}")
        say(f"step {it + 1}: {len(leaves_o)} leaves, per level {np.bincount(leaves_o[:, 0])}")
    assert s.status() == 0


def test_tree_projection_matches_oracle():
    wl = _kh((10, 10), 3, x0=(0.0, -0.01, 0.0))
    leaves = workloads.random_tree((10, 10), 3, 0.4, 8)
    o = oracle.TreeOracle(wl, leaves)
    x = o.node_coords()  # [nleaf][Q][3]
    wlq = dict(wl, nq=o.Q)
    prim = np.stack(workloads.primitives(wlq, x[..., 0], x[..., 1], x[..., 2]), axis=-1)  # [nleaf][Q][5]
    ref = o.project_prim(prim)
    s = dg.TreeSolver(wl, leaves)
    got = s.project(torch.from_numpy(np.ascontiguousarray(prim.transpose(2, 1, 0))).cuda()).cpu().numpy()
    check_state_modes(got, ref, "tree projection")


@pytest.mark.slow
def test_full_size_kh_tree_matches_oracle():
    """The benchmark's quadtree KH mesh at full size (64^2 base adapted to the
    criterion with up to 5 levels below it, 42 112 leaves): every adaptation's
    leaf set equals the oracle's and every moved state matches it; then one
    limited stage, checked on a seeded sample of leaves plus leaves on the
    refinement boundaries against the oracle's per-leaf entries applied to the
    GPU's own input (RHS per element, time step, stage, limiters)."""
    n = 64
    wl = workloads.workload("kh2d", rk="rk3", x0=(0.0, -0.3 / n, 0.0))
    leaves = np.array([(0, x, y) for y in range(n) for x in range(n)])
    o = oracle.TreeOracle(wl, leaves)
    w0 = o.initial_state()
    w, st = o.limit(w0)
    assert st == 0
    s = dg.TreeSolver(wl, leaves)
    wg = s.limit(torch.from_numpy(w0).cuda())
    check_state_modes(wg.cpu().numpy(), w, "limited initial state")
    for it in range(6):
        leaves, w = oracle.tree_adapt(wl, leaves, w, wl["wt"], wl["alpha"], 5)
        wg = s.adapt(wg, wl["wt"], wl["alpha"], 5)
        assert np.array_equal(s.leaves, leaves), f"mesh differs after adaptation {it + 1}"
        check_state_modes(wg.cpu().numpy(), w, f"regrid {it + 1}")
    nl = len(leaves)
    say("leaves", nl, "per level", np.bincount(leaves[:, 0]))
    assert nl > 40000 and leaves[:, 0].max() >= 4
    o = oracle.TreeOracle(wl, leaves)
    # the sample: seeded leaves and leaves with a face neighbour on another level
    where = {tuple(t): i for i, t in enumerate(leaves)}
    edge = []
    for i, (l, x, y) in enumerate(leaves):
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            key = (l, (x + dx) % (n << l), (y + dy) % (n << l))
            if key not in where:
                edge.append(i)
                break
    rng = workloads.splitmix64(2015, np.arange(1500)) % np.uint64(nl)
    cells = np.unique(np.concatenate([rng.astype(np.int64), np.array(edge[::max(1, len(edge) // 1500)])]))
    say("sampled leaves", cells.size, "on refinement boundaries", len(edge))
    wnp = wg.cpu().numpy()
    V, S, A = o.terms_cells(wnp, cells)
    L = s.rhs(wg).cpu().numpy()
    check_rhs_modes(L[:, :, cells], V, S, A, "full-size tree RHS")
    dt = s.max_dt(wg)
    dto = o.max_dt(wnp)
    assert float(dt.item()) == pytest.approx(dto, rel=1e-14)
    u1 = s.rk_stage(1, dt, None, wg)
    ref = wnp[:, :, cells] + dto * (V - S)
    from parity import stage_scale
    check_state_modes(u1.cpu().numpy()[:, :, cells], ref, "full-size tree stage",
                      scale=stage_scale(0.0, 1.0, dto, wnp[:, :, cells], wnp[:, :, cells], A))
    u1np = u1.cpu().numpy()
    lim = s.limit(u1).cpu().numpy()
    refl, st = o.limit_cells(u1np, cells)
    assert st == 0
    check_state_modes(lim[:, :, cells], refl, "full-size tree limiters")
    assert s.status() == 0


def test_tree_step_graph_replays_match_eager():
    """The limited tree step (time step, three stages, limiters with their
    positivity list) captured in a HIP graph: several replays, with eager
    work and synchronisations between them, each equal to the eager step
    bit for bit."""
    wl, leaves = LIMITED["k3_char_band3"][0](), LIMITED["k3_char_band3"][1]()
    o = oracle.TreeOracle(wl, leaves)
    w0 = torch.from_numpy(o.initial_state()).cuda()
    s = dg.TreeSolver(wl, leaves)
    bufs = [s.empty() for _ in range(3)] + [s.scalar()]
    eager = s.step(w0, bufs).clone()
    src = w0.clone()
    stream = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        s.step(src, bufs)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.step(src, bufs)
    for rep in range(4):
        s.rhs(w0)  # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bufs[2], eager), f"replay {rep + 1} differs from the eager step"
    assert s.status() == 0


def test_grid_calls_refuse_a_tree_context():
    import ctypes as C
    wl = _vortex((4, 4), 2)
    s = dg.TreeSolver(wl, workloads.random_tree((4, 4), 2, 0.5, 3))
    w = s.empty()
    with pytest.raises(dg.DGError):
        dg.Solver.rhs(s, w)
    n = C.c_int64()
    assert s.lib.dg_state_size(s.ctx, C.byref(n)) == 0 and n.value == w.numel()
