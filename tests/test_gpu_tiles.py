"""GPU: both tile sizes of the 2D stage kernel (the 8 x 8 tiles, and the
16-wide tiles that k = 4 runs on large grids), each forced in turn, against
the FP64 oracle on ragged grids: the RHS to 1e-12 of fac(|V| + |S|), three
one-call steps to relative L1 1e-12 and dt to 1e-14, for k = 1..4, with the
limiters and with transmissive walls."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from parity import check_rhs_modes, check_state

pytestmark = pytest.mark.gpu
# dg_config.tile2d values (DG_TILE2D_LARGE, DG_TILE2D_8X8)
TILES = {"large": 2, "8x8": 1}


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


CASES = [
    ("vortex_k1_33x17", dict(name="vortex", k=1, n=(33, 17, 1), length=(11.0, 17 / 3, 1.0))),
    ("vortex_k2_40x24", dict(name="vortex", n=(40, 24, 1), length=(10.0, 6.0, 1.0))),
    ("vortex_k3_20x18", dict(name="vortex", k=3, n=(20, 18, 1), length=(10.0, 9.0, 1.0))),
    ("vortex_k4_37x21", dict(name="vortex", k=4, n=(37, 21, 1), length=(37 / 3.6, 21 / 3.6, 1.0))),
    ("sod_char_davis", dict(name="sod", n=(40, 4, 1), length=(1.0, 0.1, 1.0), flux=1, eps=1e-3, limiter=2)),
]


@pytest.mark.parametrize("tiles", ["large", "8x8"])
@pytest.mark.parametrize("case,spec", CASES, ids=[c[0] for c in CASES])
def test_tile_sizes_match_oracle(case, spec, tiles):
    import paper_1506_06140_amd as dg
    print("tiles", case, tiles, flush=True)
    spec = dict(spec)
    wl = workloads.workload(spec.pop("name"), **spec)
    wl["tile2d"] = TILES[tiles]
    o = oracle.Oracle(wl)
    w0 = o.initial_state()
    if wl["limiter"] or wl["positivity"]:
        w0, st = o.limit(w0)
        assert st == 0
    s = dg.Solver(wl)
    V, S, A = o.terms_cells(w0, with_abs=True)
    L = _host(s.rhs(_dev(w0))).reshape(V.shape)
    check_rhs_modes(L, V, S, A, f"{case} tiles {tiles} rhs")
    fb = [s.empty() for _ in range(s.stages)]
    dt, rate = s.scalar(), s.rate_state()
    w = _dev(w0)
    s.max_rate(w, rate)
    ref = w0
    for i in range(3):
        ref, dt_ref = o.step(ref)
        w = s.rk_step(w, fb, dt, rate).clone()
        assert float(_host(dt)[0]) == pytest.approx(dt_ref, rel=1e-14)
        check_state(o, _host(w), ref, f"{case} tiles {tiles} step {i}")
    assert s.status() == 0


GRAV_CASES = [
    ("kepler_k1_33x17", dict(name="kepler", n=(33, 17, 1), length=(6.0, 6.0 * 17 / 33, 1.0))),
    ("kepler_k2_40x24", dict(name="kepler", k=2, n=(40, 24, 1), length=(6.0, 3.6, 1.0), rk="rk3")),
    ("kepler_k4_37x21", dict(name="kepler", k=4, n=(37, 21, 1), length=(6.0, 6.0 * 21 / 37, 1.0))),
]


@pytest.mark.parametrize("tiles", ["large", "8x8"])
@pytest.mark.parametrize("case,spec", GRAV_CASES, ids=[c[0] for c in GRAV_CASES])
def test_tile_sizes_with_gravity_match_oracle(case, spec, tiles):
    # the gravity source of both tile shapes (Sec. 2.4): RHS and three steps
    import paper_1506_06140_amd as dg
    print("tiles gravity", case, tiles, flush=True)
    spec = dict(spec)
    wl = workloads.workload(spec.pop("name"), **spec)
    wl["tile2d"] = TILES[tiles]
    o = oracle.Oracle(wl)
    w0, st = o.limit(o.initial_state())
    assert st == 0
    s = dg.Solver(wl)
    assert s.gravity is not None
    check_state(o, _host(s.rhs(_dev(w0))), o.rhs(w0), f"{case} tiles {tiles} rhs")
    fb = [s.empty() for _ in range(s.stages)]
    dt, rate = s.scalar(), s.rate_state()
    w = _dev(w0)
    s.max_rate(w, rate)
    ref = w0
    for i in range(3):
        ref, dt_ref = o.step(ref)
        w = s.rk_step(w, fb, dt, rate).clone()
        assert float(_host(dt)[0]) == pytest.approx(dt_ref, rel=1e-14)
        check_state(o, _host(w), ref, f"{case} tiles {tiles} step {i}")
    assert s.status() == 0
