"""Python wrapper of the plain C FP64 oracle (``dg_oracle.c``).

TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It imports nothing from the GPU
library; the only code it shares with it is the seeded workload generator in
``workloads`` (problem definitions and random numbers, no DG arithmetic).

State arrays use the layout ``[nvar][N][nz][ny][nx]`` (x fastest, nz = 1 in
2D), modes ordered by total degree, then x-exponent descending, then
y-exponent descending; variables (rho, m_x, m_y[, m_z], E).
"""
from __future__ import annotations

import ctypes as C
import itertools
import os
import subprocess

import numpy as np

import workloads

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_CS = os.path.join(_HERE, "liboracle_cs.so")

ORC_OK, ORC_EINVAL, ORC_ENEGATIVE = 0, -1, -2


def build(force: bool = True) -> None:
    """Compile the oracle (real and complex-step variants) with gcc."""
    common = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared", "-Wall"]
    for out, extra in ((_LIB, []), (_LIB_CS, ["-DORC_CS", "-fcx-limited-range"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            tmp = out + ".tmp"
            subprocess.run(common + extra + ["-o", tmp, _SRC, "-lm"], check=True)
            os.replace(tmp, out)


class Config(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("k", C.c_int), ("n", C.c_int * 3),
        ("x0", C.c_double * 3), ("len", C.c_double * 3),
        ("gamma", C.c_double), ("cfl", C.c_double),
        ("bc", C.c_int * 3), ("flux", C.c_int), ("limiter", C.c_int),
        ("beta", C.c_double), ("mtilde", C.c_double),
        ("positivity", C.c_int), ("eps", C.c_double),
        ("refine_lo", C.c_int * 3), ("refine_hi", C.c_int * 3),
        ("accel", C.POINTER(C.c_double)),
    ]


_lib = None
_lib_cs = None


def _load():
    global _lib, _lib_cs
    if _lib is None:
        if not (os.path.exists(_LIB) and os.path.exists(_LIB_CS)):
            build(force=False)
        _lib = C.CDLL(_LIB)
        _lib_cs = C.CDLL(_LIB_CS)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        cp = C.POINTER(Config)
        sig = {
            "orc_sizes": [cp, lp],
            "orc_gauss": [C.c_int, dp, dp],
            "orc_gll": [C.c_int, dp, dp],
            "orc_exponents": [cp, ip],
            "orc_basis_at": [cp, C.c_long, dp, dp],
            "orc_volume_rule": [cp, dp, dp],
            "orc_node_coords": [cp, dp],
            "orc_project": [cp, dp, dp],
            "orc_eval_points": [cp, dp, C.c_long, dp, dp],
            "orc_hllc": [cp, dp, dp, C.c_int, dp],
            "orc_euler_flux": [cp, dp, C.c_int, dp],
            "orc_rhs": [cp, dp, dp],
            "orc_rhs_cells": [cp, dp, C.c_long, lp, dp],
            "orc_terms_cell": [cp, dp, C.c_long, dp, dp],
            "orc_terms_cells": [cp, dp, C.c_long, lp, dp, dp, dp],
            "orc_max_dt": [cp, dp, dp],
            "orc_rk3_stage": [cp, C.c_int, C.c_double, dp, dp, dp],
            "orc_limit": [cp, dp],
            "orc_eigvecs": [cp, dp, C.c_int, dp, dp],
            "orc_positivity_points": [cp, dp],
            "orc_amr_sizes": [cp, lp],
            "orc_amr_node_coords": [cp, dp],
            "orc_amr_project": [cp, dp, dp],
            "orc_amr_rhs": [cp, dp, dp],
            "orc_amr_rk3_stage": [cp, C.c_int, C.c_double, dp, dp, dp],
            "orc_amr_max_dt": [cp, dp, dp],
            "orc_amr_limit": [cp, dp],
            "orc_refine_matrix": [cp, C.c_int, dp],
            "orc_amr_terms": [cp, dp, dp, dp, dp],
            "orc_limit_cells": [cp, dp, C.c_long, lp],
            "orc_amr_limit_cells": [cp, dp, C.c_long, lp],
            "orc_amr_rhs_cells": [cp, dp, C.c_long, lp, dp],
            "orc_amr_terms_cells": [cp, dp, C.c_long, lp, dp, dp, dp],
        }
        for name, args in sig.items():
            f = getattr(_lib, name)
            f.argtypes = args
            f.restype = C.c_int
        _lib.orc_legendre.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        _lib.orc_legendre.restype = None
        _lib.orc_rk3_combine.argtypes = [C.c_int, C.c_double, dp, dp, dp, dp, C.c_long]
        _lib.orc_rk3_combine.restype = None
        for name, args in {
            "orc_tableau_form": [C.c_int, dp, dp, dp, dp],
            "orc_tableau_combine": [C.c_int, dp, dp, C.c_int, C.c_double, dp, dp, dp, C.c_long],
            "orc_tableau_stage": [cp, C.c_int, dp, dp, C.c_int, C.c_double, dp, dp],
            "orc_amr_tableau_stage": [cp, C.c_int, dp, dp, C.c_int, C.c_double, dp, dp],
            "orc_amr_flags": [cp, dp, C.c_double, C.c_double, ip],
            "orc_amr_regrid": [cp, dp, cp, dp],
            "orc_tree_rhs": [cp, C.c_long, ip, lp, lp, dp, dp],
            "orc_tree_terms": [cp, C.c_long, ip, lp, lp, dp, dp, dp, dp],
            "orc_tree_limit": [cp, C.c_long, ip, lp, lp, dp],
            "orc_tree_terms_cells": [cp, C.c_long, ip, lp, lp, dp, C.c_long, lp, dp, dp, dp],
            "orc_tree_limit_cells": [cp, C.c_long, ip, lp, lp, dp, C.c_long, lp],
            "orc_tree_max_dt": [cp, C.c_long, ip, lp, lp, dp, dp],
            "orc_tree_node_coords": [cp, C.c_long, ip, lp, lp, dp],
            "orc_tree_project": [cp, C.c_long, ip, lp, lp, dp, dp],
        }.items():
            getattr(_lib, name).argtypes = args
            getattr(_lib, name).restype = C.c_int
        _lib_cs.orc_cs_rhs.argtypes = [cp, dp, dp, C.c_double, dp, dp]
        _lib_cs.orc_cs_rhs.restype = C.c_int
        _lib_cs.orc_cs_traj.argtypes = [cp, dp, dp, C.c_double, C.c_int, C.c_double, dp, dp]
        _lib_cs.orc_cs_traj.restype = C.c_int
    return _lib, _lib_cs


def _check(st: int, what: str) -> None:
    if st != ORC_OK:
        raise RuntimeError(f"oracle {what} failed with status {st}")


# ---------------------------------------------------------------------------
# 1D rules and Legendre polynomials
# ---------------------------------------------------------------------------

# Butcher tableaus (A, b) of App. D as printed: table RK_2 (Heun), table RK_3,
# table RK_4 (five stages, 14 printed digits; its weights sum to 1 - 8.8e-11).
TABLEAUS = {
    "rk2": ([[0.0, 0.0], [1.0, 0.0]], [0.5, 0.5]),
    "rk3": ([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.25, 0.25, 0.0]], [1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0]),
    "rk4": ([[0.0, 0.0, 0.0, 0.0, 0.0],
             [0.39175222700392, 0.0, 0.0, 0.0, 0.0],
             [0.21766909633821, 0.36841059262959, 0.0, 0.0, 0.0],
             [0.08269208670950, 0.13995850206999, 0.25189177424738, 0.0, 0.0],
             [0.06796628370320, 0.11503469844438, 0.20703489864929, 0.54497475021237, 0.0]],
            [0.14681187618661, 0.24848290924556, 0.10425883036650, 0.27443890091960, 0.22600748319395]),
}


def _tab(A, b):
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    s = b.size
    if A.shape != (s, s):
        raise ValueError("A must be s x s")
    return s, A, b


def tableau_form(A, b):
    """(alpha, beta) of the tableau's Shu-Osher form (see shu_osher in the C source)."""
    lib, _ = _load()
    s, A, b = _tab(A, b)
    alpha = np.zeros((s + 1, s + 1)); beta = np.zeros(s + 1)
    _check(lib.orc_tableau_form(s, A, b, alpha, beta), "tableau_form")
    return alpha, beta


def rk3_combine(stage: int, dt: float, wn, wp, L) -> np.ndarray:
    """The SSP-RK3 stage combination (App. D, table RK_3, Shu-Osher form) of
    arrays of any shape: wp + dt L (stage 1), a wn + b (wp + dt L) (2, 3)."""
    lib, _ = _load()
    wp = np.ascontiguousarray(wp, dtype=np.float64)
    wn = np.ascontiguousarray(wn if wn is not None else wp, dtype=np.float64)
    L = np.ascontiguousarray(L, dtype=np.float64)
    assert wn.shape == wp.shape == L.shape
    out = np.zeros_like(wp)
    lib.orc_rk3_combine(stage, dt, wn, wp, L, out, out.size)
    return out


def tableau_combine(A, b, m: int, dt: float, Y, L):
    """Stage value Y_m from Y_0..Y_{m-1} (a list of equal-size arrays) and L(Y_{m-1})."""
    lib, _ = _load()
    s, A, b = _tab(A, b)
    Ys = np.ascontiguousarray(np.stack([np.asarray(y, dtype=np.float64).ravel() for y in Y]))
    L = np.ascontiguousarray(np.asarray(L, dtype=np.float64).ravel())
    out = np.zeros(L.size)
    _check(lib.orc_tableau_combine(s, A, b, m, dt, Ys, L, out, L.size), "tableau_combine")
    return out


def make(wl: dict):
    """Oracle for a workload: with a refined box (refine_lo != refine_hi) or without."""
    boxed = any(a != b for a, b in zip(wl.get("refine_lo", (0, 0, 0)), wl.get("refine_hi", (0, 0, 0))))
    return AmrOracle(wl) if boxed else Oracle(wl)


def amr_flags(wl: dict, w, wt: float = 0.01, alpha: float = 1.1) -> np.ndarray:
    """Refinement flags (0/1) of the base cells (Sec. 4.1, eqs. cell_ref, node_ref)."""
    lib, _ = _load()
    o = make(wl)
    flags = np.zeros(o.ncoarse if isinstance(o, AmrOracle) else o.ncell, dtype=np.int32)
    _check(lib.orc_amr_flags(C.byref(o.c), o._s(w), wt, alpha, flags), "amr_flags")
    return flags


def box_from_flags(wl: dict, flags, layer: int = 1):
    """(refine_lo, refine_hi) of the box around the flagged base cells grown by
    `layer` cells (the buffer layer of Sec. 4), kept inside [1, n-1] per axis;
    None when no cell is flagged."""
    d = wl["dim"]
    n = list(wl["n"][:d])
    f = np.asarray(flags).reshape([wl["n"][2] if d == 3 else 1, wl["n"][1], wl["n"][0]])
    idx = np.argwhere(f)
    if idx.size == 0:
        return None
    lo, hi = [0, 0, 0], [0, 0, 0]
    for a in range(d):
        col = idx[:, 2 - a]
        lo[a] = max(1, int(col.min()) - layer)
        hi[a] = min(n[a] - 1, int(col.max()) + 1 + layer)
        if hi[a] <= lo[a]:
            return None
    return tuple(lo), tuple(hi)


def regrid(wl_old: dict, w_old, wl_new: dict) -> np.ndarray:
    """State on wl_new's grid from a state on wl_old's (Sec. 4.2, 4.3)."""
    lib, _ = _load()
    a, b = make(wl_old), make(wl_new)
    out = np.zeros(b.shape)
    _check(lib.orc_amr_regrid(C.byref(a.c), a._s(w_old), C.byref(b.c), out), "amr_regrid")
    return out


def gauss(n: int):
    lib, _ = _load()
    x = np.zeros(n); w = np.zeros(n)
    _check(lib.orc_gauss(n, x, w), "gauss")
    return x, w


def gll(m: int):
    lib, _ = _load()
    x = np.zeros(m); w = np.zeros(m)
    _check(lib.orc_gll(m, x, w), "gll")
    return x, w


def legendre(n: int, x: float):
    lib, _ = _load()
    P = C.c_double(); dP = C.c_double()
    lib.orc_legendre(n, float(x), C.byref(P), C.byref(dP))
    return P.value, dP.value


class Oracle:
    """One configured DG run (uniform Cartesian grid)."""

    def __init__(self, wl: dict):
        self.wl = dict(wl)
        c = Config()
        c.dim = wl["dim"]; c.k = wl["k"]
        c.n[:] = list(wl["n"])
        c.x0[:] = list(wl["x0"]); c.len[:] = list(wl["length"])
        c.gamma = wl["gamma"]; c.cfl = wl["cfl"]
        c.bc[:] = list(wl.get("bc", (0, 0, 0)))
        c.flux = wl.get("flux", 0)
        c.limiter = wl.get("limiter", 0)
        c.beta = wl.get("beta", 1.0); c.mtilde = wl.get("mtilde", 0.5)
        c.positivity = wl.get("positivity", 0); c.eps = wl.get("eps", 1e-10)
        c.refine_lo[:] = list(wl.get("refine_lo", (0, 0, 0)))
        c.refine_hi[:] = list(wl.get("refine_hi", (0, 0, 0)))
        self.c = c
        lib, _ = _load()
        sizes = np.zeros(7, dtype=np.int64)
        _check(lib.orc_sizes(C.byref(c), sizes), "sizes")
        self.N, self.Q, self.Qf, self.nvar, self.ncell, self.m, self.nS = (int(s) for s in sizes)
        self.dim = c.dim
        nz = wl["n"][2] if c.dim == 3 else 1
        self.shape = (self.nvar, self.N, nz, wl["n"][1], wl["n"][0])
        self.dx = wl["length"][0] / wl["n"][0]
        self._accel = None
        if wl.get("gravity") is not None:
            # the external acceleration sampled at the oracle's own volume nodes
            x = self.node_coords()  # [ncell][Q][3]
            acc = workloads.acceleration(wl, x[..., 0].T, x[..., 1].T, x[..., 2].T)  # d x [Q][ncell]
            self._accel = np.ascontiguousarray(np.stack(acc), dtype=np.float64)
            c.accel = self._accel.ctypes.data_as(C.POINTER(C.c_double))

    # -- tables -------------------------------------------------------------
    def exponents(self) -> np.ndarray:
        lib, _ = _load()
        e = np.zeros(self.N * 3, dtype=np.int32)
        _check(lib.orc_exponents(C.byref(self.c), e), "exponents")
        return e.reshape(self.N, 3)

    def basis_at(self, xi) -> np.ndarray:
        lib, _ = _load()
        xi = np.ascontiguousarray(np.asarray(xi, dtype=np.float64).reshape(-1, 3))
        out = np.zeros((xi.shape[0], self.N))
        _check(lib.orc_basis_at(C.byref(self.c), xi.shape[0], xi, out), "basis_at")
        return out

    def volume_rule(self):
        lib, _ = _load()
        xi = np.zeros((self.Q, 3)); w = np.zeros(self.Q)
        _check(lib.orc_volume_rule(C.byref(self.c), xi, w), "volume_rule")
        return xi, w

    def positivity_points(self) -> np.ndarray:
        lib, _ = _load()
        xi = np.zeros((self.nS, 3))
        _check(lib.orc_positivity_points(C.byref(self.c), xi), "positivity_points")
        return xi

    # -- initial state ------------------------------------------------------
    def node_coords(self) -> np.ndarray:
        lib, _ = _load()
        x = np.zeros((self.ncell, self.Q, 3))
        _check(lib.orc_node_coords(C.byref(self.c), x), "node_coords")
        return x

    def project_prim(self, prim: np.ndarray) -> np.ndarray:
        """L2 projection of primitives prim[ncell][Q][5] given at the nodes."""
        lib, _ = _load()
        prim = np.ascontiguousarray(prim, dtype=np.float64)
        assert prim.shape == (self.ncell, self.Q, 5)
        w = np.zeros(self.shape)
        _check(lib.orc_project(C.byref(self.c), prim, w), "project")
        return w

    def initial_state(self, t: float = 0.0) -> np.ndarray:
        """Project the workload's initial (or, with t > 0, exact) solution."""
        x = self.node_coords()
        cell = np.repeat(np.arange(self.ncell), self.Q).reshape(self.ncell, self.Q)
        node = np.tile(np.arange(self.Q), self.ncell).reshape(self.ncell, self.Q)
        wl = dict(self.wl); wl["nq"] = self.Q
        prim = np.stack(workloads.primitives(wl, x[..., 0], x[..., 1], x[..., 2],
                                             cell=cell, node=node, t=t), axis=-1)
        return self.project_prim(prim)

    # -- evaluation ---------------------------------------------------------
    def eval_points(self, w: np.ndarray, xi) -> np.ndarray:
        lib, _ = _load()
        xi = np.ascontiguousarray(np.asarray(xi, dtype=np.float64).reshape(-1, 3))
        out = np.zeros((self.ncell, xi.shape[0], self.nvar))
        _check(lib.orc_eval_points(C.byref(self.c), self._s(w), xi.shape[0], xi, out), "eval")
        return out

    def hllc(self, UL, UR, axis: int) -> np.ndarray:
        lib, _ = _load()
        F = np.zeros(self.nvar)
        _check(lib.orc_hllc(C.byref(self.c), np.ascontiguousarray(UL, dtype=np.float64),
                            np.ascontiguousarray(UR, dtype=np.float64), axis, F), "hllc")
        return F

    def euler_flux(self, U, axis: int) -> np.ndarray:
        lib, _ = _load()
        F = np.zeros(self.nvar)
        _check(lib.orc_euler_flux(C.byref(self.c), np.ascontiguousarray(U, dtype=np.float64), axis, F), "flux")
        return F

    # -- the scheme ---------------------------------------------------------
    def _s(self, w):
        w = np.ascontiguousarray(w, dtype=np.float64)
        assert w.size == int(np.prod(self.shape)), (w.shape, self.shape)
        return w

    def rhs(self, w: np.ndarray) -> np.ndarray:
        lib, _ = _load()
        L = np.zeros(self.shape)
        _check(lib.orc_rhs(C.byref(self.c), self._s(w), L), "rhs")
        return L

    def rhs_cells(self, w: np.ndarray, cells) -> np.ndarray:
        """RHS of selected (flat-indexed) cells: out[nvar][N][len(cells)]."""
        lib, _ = _load()
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros((self.nvar, self.N, cells.size))
        _check(lib.orc_rhs_cells(C.byref(self.c), self._s(w), cells.size, cells, out), "rhs_cells")
        return out

    def terms_cell(self, w: np.ndarray, cell: int):
        lib, _ = _load()
        V = np.zeros((self.nvar, self.N)); S = np.zeros((self.nvar, self.N))
        _check(lib.orc_terms_cell(C.byref(self.c), self._s(w), cell, V, S), "terms")
        return V, S

    def terms_cells(self, w: np.ndarray, cells=None, with_abs: bool = False):
        """(fac V, fac S) of selected cells (all if None): [nvar][N][ncells] each;
        with_abs adds fac times the summed magnitudes of all summands of V and S
        (the per-element rounding scale of L = fac (V - S))."""
        lib, _ = _load()
        cells = np.arange(self.ncell) if cells is None else cells
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        V = np.zeros((self.nvar, self.N, cells.size)); S = np.zeros_like(V); A = np.zeros_like(V)
        _check(lib.orc_terms_cells(C.byref(self.c), self._s(w), cells.size, cells, V, S, A), "terms_cells")
        return (V, S, A) if with_abs else (V, S)

    def max_dt(self, w: np.ndarray) -> float:
        lib, _ = _load()
        dt = np.zeros(1)
        _check(lib.orc_max_dt(C.byref(self.c), self._s(w), dt), "max_dt")
        return float(dt[0])

    def rk3_stage(self, stage: int, dt: float, wn: np.ndarray, wp: np.ndarray) -> np.ndarray:
        lib, _ = _load()
        out = np.zeros(self.shape)
        _check(lib.orc_rk3_stage(C.byref(self.c), stage, dt, self._s(wn), self._s(wp), out), "rk3_stage")
        return out

    def limit(self, w: np.ndarray) -> tuple[np.ndarray, int]:
        """Slope then positivity limiter; returns (limited copy, status)."""
        lib, _ = _load()
        out = np.array(self._s(w), copy=True)
        st = lib.orc_limit(C.byref(self.c), out)
        return out, st

    def limit_cells(self, w: np.ndarray, cells) -> tuple[np.ndarray, int]:
        """The limiters applied to the listed (flat-indexed) cells of w, with
        the neighbour means of w: ([nvar][N][len(cells)], status)."""
        lib, _ = _load()
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.array(self._s(w), copy=True)
        st = lib.orc_limit_cells(C.byref(self.c), out, cells.size, cells)
        return out.reshape(self.nvar, self.N, -1)[:, :, cells], st

    def eigvecs(self, U, axis: int):
        """(R, L): right and left eigenvectors of the flux Jacobian in `axis`
        at the conserved state U (App. E)."""
        lib, _ = _load()
        R = np.zeros((self.nvar, self.nvar)); L = np.zeros((self.nvar, self.nvar))
        _check(lib.orc_eigvecs(C.byref(self.c), np.ascontiguousarray(U, dtype=np.float64), axis, R, L), "eigvecs")
        return R, L

    _tableau_stage_fn = "orc_tableau_stage"

    def tableau_stage(self, A, b, m: int, dt: float, Y) -> np.ndarray:
        """Stage value Y_m of the tableau (A, b) from Y_0..Y_{m-1}, unlimited."""
        lib, _ = _load()
        s, A, b = _tab(A, b)
        Ys = np.ascontiguousarray(np.stack([np.asarray(self._s(y)).ravel() for y in Y]))
        out = np.zeros(self.shape)
        _check(getattr(lib, self._tableau_stage_fn)(C.byref(self.c), s, A, b, m, dt, Ys, out), "tableau_stage")
        return out

    def step_tableau(self, w, A, b, dt: float | None = None):
        """One step of the tableau (A, b), the limiters after every stage."""
        if dt is None:
            dt = self.max_dt(w)
        Y = [w]
        for m in range(1, len(b) + 1):
            out = self.tableau_stage(A, b, m, dt, Y)
            if self.c.limiter or self.c.positivity:
                out, st = self.limit(out)
                _check(st, "limit")
            Y.append(out)
        return Y[-1], dt

    def stage(self, stage: int, dt: float, wn: np.ndarray, wp: np.ndarray) -> np.ndarray:
        """RK stage followed by the limiters, if the run has any (main loop)."""
        out = self.rk3_stage(stage, dt, wn, wp)
        if self.c.limiter or self.c.positivity:
            out, st = self.limit(out)
            _check(st, "limit")
        return out

    def step(self, w: np.ndarray, dt: float | None = None) -> tuple[np.ndarray, float]:
        """One step of the workload's integrator ("rk" key; SSP-RK3 by default)."""
        rk = self.wl.get("rk", "rk3")
        if rk != "rk3":
            return self.step_tableau(w, *TABLEAUS[rk], dt=dt)
        if dt is None:
            dt = self.max_dt(w)
        w1 = self.stage(1, dt, w, w)
        w2 = self.stage(2, dt, w, w1)
        w3 = self.stage(3, dt, w, w2)
        return w3, dt

    def run(self, w: np.ndarray, steps: int, dt: float | None = None):
        t = 0.0
        for _ in range(steps):
            w, h = self.step(w, dt)
            t += h
        return w, t

    # -- derivatives (complex step) ------------------------------------------
    def jvp_rhs(self, w: np.ndarray, v: np.ndarray, h: float = 1e-30):
        """(L(w), dL/dw . v) by the complex step."""
        _, cs = _load()
        L = np.zeros(self.shape); dL = np.zeros(self.shape)
        _check(cs.orc_cs_rhs(C.byref(self.c), self._s(w), self._s(v), h, L, dL), "cs_rhs")
        return L, dL

    def jvp_traj(self, w0: np.ndarray, v: np.ndarray, steps: int, dt: float, h: float = 1e-30):
        """(w_T, dw_T/dw_0 . v) of `steps` unlimited SSP-RK3 steps at fixed dt."""
        _, cs = _load()
        wT = np.zeros(self.shape); dwT = np.zeros(self.shape)
        _check(cs.orc_cs_traj(C.byref(self.c), self._s(w0), self._s(v), h, steps, dt, wT, dwT), "cs_traj")
        return wT, dwT

    # -- diagnostics -------------------------------------------------------
    def totals(self, w: np.ndarray) -> np.ndarray:
        """Domain integrals of the conserved variables: sum_K |K| w_1."""
        w = np.asarray(w).reshape(self.nvar, self.N, -1)
        return w[:, 0, :].sum(axis=1) * self.dx ** self.dim

    def l1_density_error(self, w: np.ndarray, t: float) -> float:
        """(1/V) int |rho_h - rho_exact(t)| dV with (k+3)^d Gauss points per cell."""
        k, d = self.wl["k"], self.dim
        g, gw = gauss(k + 3)
        pts, wq = [], []
        for idx in itertools.product(range(g.size), repeat=d):
            idx = idx[::-1]  # x index fastest
            p = [0.0, 0.0, 0.0]
            ww = 1.0
            for a in range(d):
                p[a] = g[idx[a]]
                ww *= gw[idx[a]]
            pts.append(p)
            wq.append(ww)
        xi = np.array(pts)
        wq = np.array(wq)
        u = self.eval_points(w, xi)  # [ncell][npts][nvar]
        nx, ny = self.wl["n"][0], self.wl["n"][1]
        nz = self.wl["n"][2] if d == 3 else 1
        cid = np.arange(self.ncell)
        ix, iy, iz = cid % nx, (cid // nx) % ny, cid // (nx * ny)
        x0 = self.wl["x0"]
        X = x0[0] + (ix[:, None] + 0.5 + 0.5 * xi[None, :, 0]) * self.dx
        Y = x0[1] + (iy[:, None] + 0.5 + 0.5 * xi[None, :, 1]) * self.dx
        Z = (x0[2] + (iz[:, None] + 0.5 + 0.5 * xi[None, :, 2]) * self.dx) if d == 3 else np.zeros_like(X)
        wl = dict(self.wl); wl["noise"] = 0.0
        rho_ex = workloads.primitives(wl, X, Y, Z, t=t)[0]
        err = np.abs(u[:, :, 0] - rho_ex)
        return float((err * wq[None, :]).sum() / (2.0 ** d) / self.ncell)


class AmrOracle(Oracle):
    _tableau_stage_fn = "orc_amr_tableau_stage"

    """The oracle on a base grid with a static 2:1 refined box (Sec. 4).

    State: coarse block [nvar][N][ncoarse] (base grid, hole cells ignored)
    followed by the fine block [nvar][N][nfine], as one flat array."""

    def __init__(self, wl: dict):
        super().__init__(dict(wl, refine_lo=(0, 0, 0), refine_hi=(0, 0, 0)))
        self.wl = dict(wl)
        self.c.refine_lo[:] = list(wl["refine_lo"])
        self.c.refine_hi[:] = list(wl["refine_hi"])
        lib, _ = _load()
        sz = np.zeros(5, dtype=np.int64)
        _check(lib.orc_amr_sizes(C.byref(self.c), sz), "amr_sizes")
        self.ncoarse, self.nfine = int(sz[0]), int(sz[1])
        self.nf = tuple(int(x) for x in sz[2:5])
        self.size = self.nvar * self.N * (self.ncoarse + self.nfine)
        self.shape = (self.size,)
        self.dxf = 0.5 * self.dx
        d = self.dim
        lo, hi = wl["refine_lo"], wl["refine_hi"]
        n = wl["n"]
        self.hole = np.zeros(self.ncoarse, dtype=bool)
        cid = np.arange(self.ncoarse)
        idx = [cid % n[0], (cid // n[0]) % n[1], cid // (n[0] * n[1])]
        inside = np.ones(self.ncoarse, dtype=bool)
        for a in range(d):
            inside &= (idx[a] >= lo[a]) & (idx[a] < hi[a])
        self.hole = inside

    def blocks(self, w):
        """(coarse [nvar][N][ncoarse], fine [nvar][N][nfine]) views of a state."""
        w = np.asarray(w).reshape(-1)
        nc = self.nvar * self.N * self.ncoarse
        return (w[:nc].reshape(self.nvar, self.N, self.ncoarse),
                w[nc:].reshape(self.nvar, self.N, self.nfine))

    def node_coords(self):
        lib, _ = _load()
        x = np.zeros((self.ncoarse + self.nfine, self.Q, 3))
        _check(lib.orc_amr_node_coords(C.byref(self.c), x), "amr_node_coords")
        return x

    def initial_state(self, t: float = 0.0):
        lib, _ = _load()
        x = self.node_coords()
        nct = self.ncoarse + self.nfine
        cell = np.repeat(np.arange(nct), self.Q).reshape(nct, self.Q)
        node = np.tile(np.arange(self.Q), nct).reshape(nct, self.Q)
        wl = dict(self.wl); wl["nq"] = self.Q
        prim = np.ascontiguousarray(np.stack(workloads.primitives(wl, x[..., 0], x[..., 1], x[..., 2],
                                                                  cell=cell, node=node, t=t), axis=-1))
        w = np.zeros(self.size)
        _check(lib.orc_amr_project(C.byref(self.c), prim, w), "amr_project")
        return w

    def rhs(self, w):
        lib, _ = _load()
        L = np.zeros(self.size)
        _check(lib.orc_amr_rhs(C.byref(self.c), self._s(w), L), "amr_rhs")
        return L

    def max_dt(self, w):
        lib, _ = _load()
        dt = np.zeros(1)
        _check(lib.orc_amr_max_dt(C.byref(self.c), self._s(w), dt), "amr_max_dt")
        return float(dt[0])

    def rk3_stage(self, stage, dt, wn, wp):
        lib, _ = _load()
        out = np.zeros(self.size)
        _check(lib.orc_amr_rk3_stage(C.byref(self.c), stage, dt, self._s(wn), self._s(wp), out), "amr_rk3")
        return out

    def limit(self, w):
        lib, _ = _load()
        out = np.array(self._s(w), copy=True)
        st = lib.orc_amr_limit(C.byref(self.c), out)
        return out, st

    def cells_of(self, x, cells):
        """[nvar][N][len(cells)] of a flat state at cells of the combined
        numbering (coarse cells, then fine cells)."""
        c, f = self.blocks(x)
        full = np.concatenate([c, f], axis=2)
        return full[:, :, np.asarray(cells, dtype=np.int64)]

    def limit_cells(self, w, cells):
        """The limiters on the listed cells (combined numbering) of w:
        ([nvar][N][len(cells)], status)."""
        lib, _ = _load()
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.array(self._s(w), copy=True)
        st = lib.orc_amr_limit_cells(C.byref(self.c), out, cells.size, cells)
        return self.cells_of(out, cells), st

    def rhs_cells(self, w, cells):
        """dw/dt of the listed cells (combined numbering): [nvar][N][len(cells)]."""
        lib, _ = _load()
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros((self.nvar, self.N, cells.size))
        _check(lib.orc_amr_rhs_cells(C.byref(self.c), self._s(w), cells.size, cells, out), "amr_rhs_cells")
        return out

    def totals(self, w):
        """Domain integrals of the conserved variables (hole cells excluded)."""
        wc, wf = self.blocks(w)
        d = self.dim
        tc = wc[:, 0, ~self.hole].sum(axis=1) * self.dx ** d
        tf = wf[:, 0, :].sum(axis=1) * self.dxf ** d
        return tc + tf

    def _s(self, w):
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
        assert w.size == self.size
        return w

    def terms_cells(self, w, cells=None, with_abs: bool = False):
        """(fac V, fac S) of every cell of both blocks, flat like the state
        (with_abs: and the summed magnitudes of their summands, as for the
        uniform grid); with `cells` (combined numbering) only those cells,
        [nvar][N][len(cells)] each."""
        lib, _ = _load()
        if cells is not None:
            cells = np.ascontiguousarray(cells, dtype=np.int64)
            V = np.zeros((self.nvar, self.N, cells.size)); S = np.zeros_like(V); A = np.zeros_like(V)
            _check(lib.orc_amr_terms_cells(C.byref(self.c), self._s(w), cells.size, cells, V, S, A),
                   "amr_terms_cells")
            return (V, S, A) if with_abs else (V, S)
        V = np.zeros(self.size); S = np.zeros(self.size); A = np.zeros(self.size)
        _check(lib.orc_amr_terms(C.byref(self.c), self._s(w), V, S, A), "amr_terms")
        return (V, S, A) if with_abs else (V, S)

    def refine_matrix(self, child: int):
        lib, _ = _load()
        P = np.zeros((self.N, self.N))
        _check(lib.orc_refine_matrix(C.byref(self.c), child, P), "refine_matrix")
        return P


class TreeOracle(Oracle):
    """A 2D run on a quadtree of leaves (Sec. 4): `leaves` is an integer array
    [nleaf][3] of (level, ix, iy), level 0 the workload's base grid.  The state
    is [nvar][N][nleaf] in leaf order."""

    def __init__(self, wl: dict, leaves):
        if wl["dim"] != 2:
            raise ValueError("the quadtree oracle is 2D")
        super().__init__(dict(wl, refine_lo=(0, 0, 0), refine_hi=(0, 0, 0)))
        lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int64).reshape(-1, 3))
        self.leaves = lv
        self.nleaf = lv.shape[0]
        self._lev = np.ascontiguousarray(lv[:, 0], dtype=np.int32)
        self._ix = np.ascontiguousarray(lv[:, 1], dtype=np.int64)
        self._iy = np.ascontiguousarray(lv[:, 2], dtype=np.int64)
        self.shape = (self.nvar, self.N, self.nleaf)
        self.ncell = self.nleaf

    def _a(self):
        return (C.byref(self.c), self.nleaf, self._lev, self._ix, self._iy)

    def node_coords(self) -> np.ndarray:
        """[nleaf][Q][3] physical coordinates of the leaves' volume nodes."""
        lib, _ = _load()
        x = np.zeros((2, self.Q, self.nleaf))
        _check(lib.orc_tree_node_coords(*self._a(), x), "tree_node_coords")
        out = np.zeros((self.nleaf, self.Q, 3))
        out[..., 0] = x[0].T
        out[..., 1] = x[1].T
        return out

    def project_prim(self, prim: np.ndarray) -> np.ndarray:
        lib, _ = _load()
        prim = np.ascontiguousarray(prim, dtype=np.float64)
        assert prim.shape == (self.nleaf, self.Q, 5)
        w = np.zeros(self.shape)
        _check(lib.orc_tree_project(*self._a(), prim, w), "tree_project")
        return w

    def rhs(self, w: np.ndarray) -> np.ndarray:
        lib, _ = _load()
        L = np.zeros(self.shape)
        _check(lib.orc_tree_rhs(*self._a(), self._s(w), L), "tree_rhs")
        return L

    def terms(self, w: np.ndarray):
        """(fac V, fac S, fac A) of every leaf, each [nvar][N][nleaf] (L = V - S;
        A the summed magnitudes of the summands)."""
        lib, _ = _load()
        V, S, A = np.zeros(self.shape), np.zeros(self.shape), np.zeros(self.shape)
        _check(lib.orc_tree_terms(*self._a(), self._s(w), V, S, A), "tree_terms")
        return V, S, A

    def max_dt(self, w: np.ndarray) -> float:
        lib, _ = _load()
        dt = np.zeros(1)
        _check(lib.orc_tree_max_dt(*self._a(), self._s(w), dt), "tree_max_dt")
        return float(dt[0])

    def rk3_stage(self, stage: int, dt: float, wn, wp) -> np.ndarray:
        return rk3_combine(stage, dt, wn, wp, self.rhs(wp))

    def terms_cells(self, w: np.ndarray, cells):
        """(fac V, fac S, fac A) of the listed leaves, each [nvar][N][len(cells)]."""
        lib, _ = _load()
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        sh = (self.nvar, self.N, cells.size)
        V, S, A = np.zeros(sh), np.zeros(sh), np.zeros(sh)
        _check(lib.orc_tree_terms_cells(*self._a(), self._s(w), cells.size, cells, V, S, A), "tree_terms_cells")
        return V, S, A

    def limit_cells(self, w: np.ndarray, cells):
        """The limiters on the listed leaves of w (neighbour values from w):
        ([nvar][N][len(cells)], status)."""
        lib, _ = _load()
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.array(self._s(w), copy=True)
        st = lib.orc_tree_limit_cells(*self._a(), out, cells.size, cells)
        return out[:, :, cells], st

    def limit(self, w: np.ndarray):
        """Slope then positivity limiter with the AMR rules of Sec. 4.4:
        (limited copy, status)."""
        lib, _ = _load()
        out = np.array(self._s(w), copy=True)
        st = lib.orc_tree_limit(*self._a(), out)
        return out, st

    def step(self, w0: np.ndarray, dt: float | None = None):
        """One SSP-RK3 step (App. D, table RK_3), the limiters after every
        stage when the workload asks for them; returns (w1, dt)."""
        if dt is None:
            dt = self.max_dt(w0)
        lim = self.wl.get("limiter", 0) or self.wl.get("positivity", 0)

        def L(x):
            return self.limit(x)[0] if lim else x
        w1 = L(self.rk3_stage(1, dt, w0, w0))
        w2 = L(self.rk3_stage(2, dt, w0, w1))
        return L(self.rk3_stage(3, dt, w0, w2)), dt


def _tree_refine_mats(wl: dict):
    """P_c (eq. ref_pa_integral) of the 4 children, each [N][N] with
    (P_c)[j][l] the weight of coarse mode l in child mode j."""
    lib, _ = _load()
    o = Oracle(dict(wl, refine_lo=(0, 0, 0), refine_hi=(0, 0, 0)))
    P = []
    for ch in range(4):
        m = np.zeros(o.N * o.N)
        _check(lib.orc_refine_matrix(C.byref(o.c), ch, m), "refine_matrix")
        P.append(m.reshape(o.N, o.N))
    return P


def tree_adapt(wl: dict, leaves, w, wt: float = 0.01, alpha: float = 1.1, max_level: int = 3):
    """One adaptation of a 2D quadtree (Sec. 4, 4.1-4.3): returns (new leaves
    [n][3] in Morton order of their lower-left corners, new state
    [nvar][N][n]).  Steps, in this order:
      1. a leaf is flagged if max_a |w_rho,1+a| > alpha wt (eq. cell_ref); a
         flagged leaf below max_level is split, and so is every leaf of the
         same or a coarser level (below max_level) that covers one of the
         eight cells around it on its level (one buffer layer);
      2. a split leaf forces the split of any coarser leaf covering one of the
         eight cells around it on its level (level jump at most one to face and
         corner neighbours), repeated until nothing changes;
      3. four sibling leaves (all leaves, none split) whose node weights
         2^-d sum_c P_c^T w^c (eq. deref_weights) have max_a |w_rho,1+a| <=
         wt / alpha (eq. node_ref fails) are merged when no cell around any of
         them on their level is finer than them after step 2; all such merges
         at once.
    Split leaves' children get P_c w (eq. ref_weights), merged groups the
    node weights, other leaves keep their weights."""
    lv = [tuple(int(v) for v in t) for t in np.asarray(leaves).reshape(-1, 3)]
    w = np.asarray(w, dtype=np.float64)
    nvar, N, nl = w.shape
    n = wl["n"]
    bc = wl.get("bc", (0, 0, 0))
    where = {t: i for i, t in enumerate(lv)}
    P = _tree_refine_mats(wl)

    def wrap(l, x, y):
        nx, ny = n[0] << l, n[1] << l
        if not 0 <= x < nx:
            if bc[0] != 0:
                return None
            x %= nx
        if not 0 <= y < ny:
            if bc[1] != 0:
                return None
            y %= ny
        return x, y

    def covering(l, x, y):
        for q in range(l, -1, -1):
            j = where.get((q, x >> (l - q), y >> (l - q)))
            if j is not None:
                return j
        return None

    def around(i):
        l, x, y = lv[i]
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                if dx or dy:
                    p = wrap(l, x + dx, y + dy)
                    if p is not None:
                        yield l, p[0], p[1]

    flag = [max(abs(w[0, 1, i]), abs(w[0, 2, i])) > alpha * wt for i in range(nl)]
    split = [False] * nl
    for i in range(nl):
        if flag[i] and lv[i][0] < max_level:
            split[i] = True
            for c in around(i):
                j = covering(*c)
                if j is not None and lv[j][0] < max_level:
                    split[j] = True
    changed = True
    while changed:
        changed = False
        for i in range(nl):
            if not split[i]:
                continue
            for c in around(i):
                j = covering(*c)
                if j is not None and lv[j][0] < lv[i][0] and not split[j]:
                    split[j] = True
                    changed = True

    def level_after(l, x, y):
        j = covering(l, x, y)
        return l + 1 if j is None else lv[j][0] + int(split[j])

    groups = {}
    for i, (l, x, y) in enumerate(lv):
        if l < 1:
            continue
        sib = [where.get((l, 2 * (x >> 1) + (c & 1), 2 * (y >> 1) + (c >> 1))) for c in range(4)]
        if all(s is not None for s in sib) and sib[0] == i:
            groups[i] = sib
    merged = {}
    for i0, sib in groups.items():
        node = sum(P[c].T @ w[:, :, sib[c]].T for c in range(4)).T / 4.0  # [nvar][N]
        if max(abs(node[0, 1]), abs(node[0, 2])) > wt / alpha:
            continue
        if any(split[m] for m in sib):
            continue
        l = lv[i0][0]
        if any(level_after(*c) > l for m in sib for c in around(m)):
            continue
        merged[i0] = (sib, node)
    members = {m for sib, _ in merged.values() for m in sib}
    new = []  # (leaf, state [nvar][N])
    for i, (l, x, y) in enumerate(lv):
        if split[i]:
            for c in range(4):
                new.append(((l + 1, 2 * x + (c & 1), 2 * y + (c >> 1)), (P[c] @ w[:, :, i].T).T))
        elif i in merged:
            new.append(((l - 1, x >> 1, y >> 1), merged[i][1]))
        elif i not in members:
            new.append(((l, x, y), w[:, :, i]))
    L = max(t[0][0] for t in new)

    def morton(t):
        l, x, y = t[0]
        x <<= L - l
        y <<= L - l
        k = 0
        for b in range(60):
            k |= ((x >> b) & 1) << (2 * b) | ((y >> b) & 1) << (2 * b + 1)
        return k
    new.sort(key=morton)
    out_l = np.array([t[0] for t in new], dtype=np.int64)
    out_w = np.ascontiguousarray(np.stack([t[1] for t in new], axis=2))
    return out_l, out_w
