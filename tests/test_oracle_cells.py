"""CPU: the oracle's per-cell entries (used by the sampled full-size GPU
checks) give exactly what its whole-mesh calls give on those cells, and the
summand-magnitude output bounds the volume and face terms."""
import numpy as np

import oracle
import workloads


def _rough(o, w, seed, amp):
    rng = np.random.default_rng(seed)
    w = np.array(w, copy=True)
    if isinstance(o, oracle.AmrOracle):
        for b in o.blocks(w):
            b[:, 1:] += amp * rng.uniform(-1, 1, size=b[:, 1:].shape)
    else:
        w[:, 1:] += amp * rng.uniform(-1, 1, size=w[:, 1:].shape)
    return w


def test_uniform_cells_equal_whole_mesh():
    wl = workloads.workload("kh3d", n=(8, 7, 6), length=(0.8, 0.7, 0.6))
    o = oracle.Oracle(wl)
    w = _rough(o, o.initial_state(), 3, 0.05)
    cells = np.array([0, 5, 17, 100, 201, o.ncell - 1])
    ref, st = o.limit(w)
    got, st2 = o.limit_cells(w, cells)
    assert st == st2 == 0
    assert np.array_equal(got, ref.reshape(o.nvar, o.N, -1)[:, :, cells])
    # at least one listed cell is changed by the limiter
    assert not np.array_equal(got, w.reshape(o.nvar, o.N, -1)[:, :, cells])
    L = o.rhs(w).reshape(o.nvar, o.N, -1)
    assert np.array_equal(o.rhs_cells(w, cells), L[:, :, cells])
    V, S, A = o.terms_cells(w, cells, with_abs=True)
    assert np.all(A >= (np.abs(V) + np.abs(S)) * (1 - 1e-14))


def test_refined_box_cells_equal_whole_mesh():
    wl = workloads.workload("blast_amr", dim=3, k=2, n=(8, 7, 6), length=(1.0, 7 / 8, 6 / 8), refine_lo=(2, 2, 1),
                            refine_hi=(6, 5, 4), eps=1e-3)
    o = oracle.AmrOracle(wl)
    w0, st = o.limit(o.initial_state())
    assert st == 0
    w = _rough(o, w0, 4, 0.02)
    allc = np.arange(o.ncoarse + o.nfine)[~np.concatenate([o.hole, np.zeros(o.nfine, bool)])]
    cells = allc[::7]
    ref, st = o.limit(w)
    got, st2 = o.limit_cells(w, cells)
    assert st == st2 == 0
    assert np.array_equal(got, o.cells_of(ref, cells))
    # the right-hand side of the limited state (the rough one has negative
    # node pressures)
    assert np.array_equal(o.rhs_cells(ref, cells), o.cells_of(o.rhs(ref), cells))
    V, S, A = o.terms_cells(ref, with_abs=True)
    V2, S2, A2 = o.terms_cells(ref, cells, with_abs=True)
    assert np.array_equal(V2, o.cells_of(V, cells)) and np.array_equal(A2, o.cells_of(A, cells))
    assert np.all(A2 >= (np.abs(V2) + np.abs(S2)) * (1 - 1e-14))
