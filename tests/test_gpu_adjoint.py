"""GPU checks of the discrete adjoint (dg_adjoint_rhs, dg_adjoint_rk_stage and
the checkpointed trajectory gradient) against the oracle's complex-step
derivatives (exact to rounding, computed through the oracle's own code) and
against central finite differences.

Tolerances: the dot-product identity <mu, v> = <lam, J v> to 1e-12 of
sum |lam_i (J v)_i|; element-wise VJP to 1e-11 relative L1; trajectory
gradient directional derivatives to 1e-10 relative; finite differences to
1e-6 relative (the FD truncation and rounding errors are about 1e-8 here)."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _state(o, seed):
    """Positive state whose neighbouring cells differ by O(0.1), so that no
    wave-speed bound of the Riemann solver sits at a tie (a kink)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(o.shape)
    d = o.dim
    shp = w.shape[2:]
    rho = 1.0 + 0.3 * rng.uniform(0, 1, size=shp)
    vel = [0.5 * rng.uniform(-1, 1, size=shp) for _ in range(d)]
    p = 1.0 + 0.3 * rng.uniform(0, 1, size=shp)
    w[0, 0] = rho
    for a in range(d):
        w[1 + a, 0] = rho * vel[a]
    w[d + 1, 0] = p / (o.wl["gamma"] - 1) + 0.5 * rho * sum(v * v for v in vel)
    w[:, 1:] = 0.02 * rng.uniform(-1, 1, size=w[:, 1:].shape)
    return w


ADJ_CASES = [
    ("2d_k1", dict(dim=2, k=1, n=(9, 7, 1))),
    ("2d_k2", dict(dim=2, k=2, n=(9, 7, 1))),
    ("2d_k3", dict(dim=2, k=3, n=(9, 7, 1))),
    ("2d_k2_davis", dict(dim=2, k=2, n=(9, 7, 1), flux=1)),
    ("2d_k2_transmissive", dict(dim=2, k=2, n=(9, 7, 1), bc=(1, 0, 0))),
    ("2d_k3_transmissive_xy_davis", dict(dim=2, k=3, n=(9, 7, 1), bc=(1, 1, 0), flux=1)),
    ("3d_k1", dict(dim=3, k=1, n=(5, 4, 3))),
    ("3d_k2", dict(dim=3, k=2, n=(5, 4, 3))),
]


def _wl(over):
    n = over["n"]
    return workloads.workload("vortex", noise=0.0, x0=(0.0, 0.0, 0.0),
                              length=tuple(0.1 * m for m in n), **over)


@pytest.mark.parametrize("case,over", ADJ_CASES, ids=[c[0] for c in ADJ_CASES])
def test_adjoint_rhs_dot_product(case, over):
    import paper_1506_06140_amd as dg
    wl = _wl(over)
    o = oracle.Oracle(wl)
    s = dg.Solver(wl)
    w = _state(o, seed=3)
    rng = np.random.default_rng(7)
    for trial in range(3):
        lam = rng.uniform(-1, 1, size=o.shape)
        v = rng.uniform(-1, 1, size=o.shape)
        _, Jv = o.jvp_rhs(w, v)
        mu = _host(s.adjoint_rhs(_dev(w), _dev(lam)))
        lhs, rhs = (mu * v).sum(), (lam * Jv).sum()
        scale = np.abs(lam * Jv).sum()
        _say(case, trial, "<mu,v>", lhs, "<lam,Jv>", rhs, "rel", abs(lhs - rhs) / scale)
        assert abs(lhs - rhs) <= 1e-12 * scale
    assert s.status() == 0


@pytest.mark.parametrize("dim,k,bc", [(2, 1, 0), (2, 2, 0), (2, 2, 1), (3, 1, 0)])
def test_adjoint_rhs_elementwise(dim, k, bc):
    # mu_i = lam . (J e_i) with every Jacobian column from the oracle.
    import paper_1506_06140_amd as dg
    n = (5, 4, 3) if dim == 3 else (5, 4, 1)
    wl = _wl(dict(dim=dim, k=k, n=n, bc=(bc, 0, 0)))
    o = oracle.Oracle(wl)
    s = dg.Solver(wl)
    w = _state(o, seed=11)
    lam = np.random.default_rng(12).uniform(-1, 1, size=o.shape)
    ref = np.zeros(o.shape).ravel()
    e = np.zeros(o.shape)
    ef = e.ravel()
    for i in range(ref.size):
        ef[i] = 1.0
        _, Je = o.jvp_rhs(w, e)
        ref[i] = (lam * Je).sum()
        ef[i] = 0.0
    mu = _host(s.adjoint_rhs(_dev(w), _dev(lam))).ravel()
    err = np.abs(mu - ref).sum() / np.abs(ref).sum()
    _say("elementwise VJP", dim, k, bc, "rel-L1", err)
    assert err <= 1e-11


def test_adjoint_rk_stage_combinations():
    # The transposed Shu-Osher stages against their definition, built from
    # dg_adjoint_rhs outputs.
    import torch
    import paper_1506_06140_amd as dg
    wl = _wl(dict(dim=2, k=2, n=(9, 7, 1)))
    o = oracle.Oracle(wl)
    s = dg.Solver(wl)
    u = _dev(_state(o, seed=5))
    rng = np.random.default_rng(9)
    lam = _dev(rng.uniform(-1, 1, size=o.shape))
    acc = _dev(rng.uniform(-1, 1, size=o.shape))
    dt = _dev(np.array([1e-3]))
    mu = s.adjoint_rhs(u, lam)
    out, acc_out = s.empty(), s.empty()
    s.adjoint_rk_stage(3, dt, u, lam, None, out, acc_out)
    torch.testing.assert_close(out, 2 / 3 * (lam + 1e-3 * mu), rtol=1e-14, atol=1e-15)
    torch.testing.assert_close(acc_out, lam / 3, rtol=1e-15, atol=0)
    s.adjoint_rk_stage(2, dt, u, lam, acc, out, acc_out)
    torch.testing.assert_close(out, 0.25 * (lam + 1e-3 * mu), rtol=1e-14, atol=1e-15)
    torch.testing.assert_close(acc_out, acc + 0.75 * lam, rtol=1e-15, atol=1e-16)
    s.adjoint_rk_stage(1, dt, u, lam, acc, out, None)
    torch.testing.assert_close(out, acc + lam + 1e-3 * mu, rtol=1e-14, atol=1e-15)


def _grad(s, w0, steps, dt, ckpt):
    import torch
    from paper_1506_06140_amd import adjoint
    x = w0.clone().requires_grad_(True)
    wT = adjoint.trajectory(s, x, steps, dt, ckpt)
    J = adjoint.density_square_integral(s, wT)
    J.backward()
    return float(J.detach()), x.grad.detach()


def test_trajectory_gradient_matches_oracle_directional_derivatives():
    # Boosted vortex, k=3, 64^2 (a reduced adjoint workload), 40 steps at a
    # fixed dt, checkpoint every 10 steps; J = int rho(T)^2.
    import paper_1506_06140_amd as dg
    wl = workloads.workload("vortex_adjoint", n=(64, 64, 1))
    o = oracle.Oracle(wl)
    s = dg.Solver(wl)
    w0 = o.initial_state()
    dt = o.max_dt(w0)
    steps = 40
    J, g = _grad(s, _dev(w0), steps, _dev(np.array([dt])), 10)
    g = _host(g)
    vol = o.dx ** 2
    rng = np.random.default_rng(21)
    for j in range(3):
        d = rng.uniform(-1, 1, size=o.shape)
        wT, dwT = o.jvp_traj(w0, d, steps, dt)
        dJ_ref = 2.0 * vol * (wT[0] * dwT[0]).sum()
        J_ref = vol * (wT[0] ** 2).sum()
        dJ = (g * d).sum()
        _say("direction", j, "dJ gpu", dJ, "oracle", dJ_ref, "rel", abs(dJ - dJ_ref) / abs(dJ_ref))
        assert J == pytest.approx(J_ref, rel=1e-12)
        assert abs(dJ - dJ_ref) <= 1e-10 * abs(dJ_ref)


def _J(s, w0, steps, dt):
    import torch
    from paper_1506_06140_amd import adjoint
    with torch.no_grad():
        wT = adjoint.trajectory(s, w0, steps, dt, steps)
        return float(adjoint.density_square_integral(s, wT))


def test_trajectory_gradient_central_differences():
    # Central differences of J on 64 seeded +-1 directions (SplitMix64 seeds
    # 1..64) scaled to |d|_2 = |w0|_2, steps h in {1e-5, 1e-6, 1e-7}; the best
    # h per direction agrees with <grad J, d> to 1e-6 relative.
    import paper_1506_06140_amd as dg
    wl = workloads.workload("vortex_adjoint", n=(64, 64, 1))
    o = oracle.Oracle(wl)
    s = dg.Solver(wl)
    w0 = o.initial_state()
    dt = _dev(np.array([o.max_dt(w0)]))
    steps = 40
    J, g = _grad(s, _dev(w0), steps, dt, 10)
    g = _host(g)
    scale = np.linalg.norm(w0) / np.sqrt(w0.size)
    for seed in range(1, 65):
        d = workloads.sign_direction(seed, w0.size).reshape(w0.shape) * scale
        dJ = float((g * d).sum())
        errs = []
        for h in (1e-5, 1e-6, 1e-7):
            jp = _J(s, _dev(w0 + h * d), steps, dt)
            jm = _J(s, _dev(w0 - h * d), steps, dt)
            errs.append(abs((jp - jm) / (2 * h) - dJ) / abs(dJ))
        _say("direction seed", seed, "dJ", dJ, "FD rel err per h", errs)
        assert min(errs) <= 1e-6, errs
