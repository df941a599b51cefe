"""MI355X modal discontinuous Galerkin hot path: Python binding of libdg.so.

The binding only marshals arguments: every step of the right-hand side, the
SSP-RK3 stage, the time step, the limiters and the adjoint runs in the HIP
kernels of ``libdg.so`` (see ``include/dg.h``).  PyTorch provides device
memory and streams.  There is no CPU fallback: if the library is missing or
no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DG_LIBRARY may point at another build of the same sources (tuning runs)
LIB_PATH = os.environ.get("DG_LIBRARY", os.path.join(_HERE, "libdg.so"))

DG_OK, DG_EINVAL, DG_EUNSUPPORTED, DG_ENOMEM, DG_EHIP, DG_ENEGATIVE, DG_ENAN, DG_ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
DG_STATIC_SCRATCH_FLOATS = 8 * 1024 * 1024
DG_FP64, DG_FP32, DG_BF16_VOL = 0, 1, 2
DG_LIM_NONE, DG_LIM_MINMOD, DG_LIM_CHAR = 0, 1, 2
DG_TILE2D_AUTO, DG_TILE2D_8X8, DG_TILE2D_LARGE = 0, 1, 2
DG_PATH3D_AUTO, DG_PATH3D_VALU = 0, 1
# doubles in the carried rate state (8 slots, 16 apart; the rate is the largest slot)
DG_RATE_STATE, RATE_SLOTS, RATE_STRIDE = 128, 8, 16
PRECISIONS = {"fp64": DG_FP64, "fp32": DG_FP32, "bf16": DG_BF16_VOL}
DG_MAX_STAGES = 5
# Butcher tableaus (a, b) of App. D for dg_set_tableau: table RK_2 (Heun),
# table RK_3 and the five-stage table RK_4 as printed (14 digits).
TABLEAUS = {
    "rk2": ((0.0, 0.0,
             1.0, 0.0), (0.5, 0.5)),
    "rk3": ((0.0, 0.0, 0.0,
             1.0, 0.0, 0.0,
             0.25, 0.25, 0.0), (1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0)),
    "rk4": ((0.0, 0.0, 0.0, 0.0, 0.0,
             0.39175222700392, 0.0, 0.0, 0.0, 0.0,
             0.21766909633821, 0.36841059262959, 0.0, 0.0, 0.0,
             0.08269208670950, 0.13995850206999, 0.25189177424738, 0.0, 0.0,
             0.06796628370320, 0.11503469844438, 0.20703489864929, 0.54497475021237, 0.0),
            (0.14681187618661, 0.24848290924556, 0.10425883036650, 0.27443890091960, 0.22600748319395)),
}


class DGError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class dg_config(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("k", C.c_int), ("n", C.c_int * 3),
        ("x0", C.c_double * 3), ("len", C.c_double * 3),
        ("gamma", C.c_double), ("cfl", C.c_double),
        ("bc", C.c_int * 3), ("flux", C.c_int), ("precision", C.c_int),
        ("slope_limiter", C.c_int), ("beta", C.c_double), ("m_tilde", C.c_double),
        ("positivity", C.c_int), ("eps", C.c_double),
        ("refine_lo", C.c_int * 3), ("refine_hi", C.c_int * 3),
        ("tile2d", C.c_int), ("path3d", C.c_int),
    ]


EXPORTS = (
    "dg_init", "dg_state_size", "dg_sizes", "dg_amr_sizes", "dg_quadrature", "dg_project", "dg_rhs", "dg_rhs_noalloc",
    "dg_max_dt", "dg_rk_stage", "dg_max_rate", "dg_rk_step", "dg_set_tableau", "dg_tableau_stage", "dg_tableau_step",
    "dg_set_gravity", "dg_amr_flags", "dg_amr_regrid", "dg_limit", "dg_adjoint_rhs", "dg_adjoint_rk_stage", "dg_status", "dg_destroy", "dg_strerror",
    "dg_tree_set", "dg_tree_size", "dg_tree_leaves", "dg_tree_rhs", "dg_tree_rk_stage", "dg_tree_max_dt",
    "dg_tree_adapt", "dg_tree_regrid", "dg_tree_limit",
)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdg.so and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1506_06140_amd.build`")
    lib = C.CDLL(path)
    vp, dp = C.c_void_p, C.c_void_p
    ctxp = C.c_void_p
    lib.dg_init.argtypes = [C.POINTER(dg_config), C.POINTER(ctxp)]
    lib.dg_state_size.argtypes = [ctxp, C.POINTER(C.c_int64)]
    lib.dg_sizes.argtypes = [ctxp, C.POINTER(C.c_int64)]
    lib.dg_amr_sizes.argtypes = [ctxp, C.POINTER(C.c_int64)]
    lib.dg_quadrature.argtypes = [ctxp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.dg_project.argtypes = [ctxp, dp, dp, vp]
    lib.dg_rhs.argtypes = [ctxp, dp, dp, vp]
    lib.dg_rhs_noalloc.argtypes = [ctxp, dp, dp, vp]
    lib.dg_max_dt.argtypes = [ctxp, dp, dp, vp]
    lib.dg_rk_stage.argtypes = [ctxp, C.c_int, dp, dp, dp, dp, vp]
    lib.dg_max_rate.argtypes = [ctxp, dp, dp, vp]
    lib.dg_rk_step.argtypes = [ctxp, dp, dp, dp, dp, dp, dp, vp]
    lib.dg_set_tableau.argtypes = [ctxp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.dg_tableau_stage.argtypes = [ctxp, C.c_int, dp, C.POINTER(C.c_void_p), dp, vp]
    lib.dg_tableau_step.argtypes = [ctxp, dp, C.POINTER(C.c_void_p), dp, dp, dp, vp]
    lib.dg_limit.argtypes = [ctxp, dp, vp]
    lib.dg_set_gravity.argtypes = [ctxp, dp, vp]
    lib.dg_amr_flags.argtypes = [ctxp, dp, C.c_double, C.c_double, dp, dp, vp]
    lib.dg_amr_regrid.argtypes = [ctxp, dp, ctxp, dp, vp]
    lib.dg_adjoint_rhs.argtypes = [ctxp, dp, dp, dp, vp]
    lib.dg_adjoint_rk_stage.argtypes = [ctxp, C.c_int, dp, dp, dp, dp, dp, dp, vp]
    lib.dg_status.argtypes = [ctxp, vp]
    ip32 = C.POINTER(C.c_int32)
    lib.dg_tree_set.argtypes = [ctxp, C.c_int64, ip32]
    lib.dg_tree_size.argtypes = [ctxp, C.POINTER(C.c_int64)]
    lib.dg_tree_leaves.argtypes = [ctxp, ip32]
    lib.dg_tree_rhs.argtypes = [ctxp, dp, dp, vp]
    lib.dg_tree_rk_stage.argtypes = [ctxp, C.c_int, dp, dp, dp, dp, vp]
    lib.dg_tree_max_dt.argtypes = [ctxp, dp, dp, vp]
    lib.dg_tree_adapt.argtypes = [ctxp, dp, C.c_double, C.c_double, C.c_int, C.POINTER(C.c_int64), vp]
    lib.dg_tree_regrid.argtypes = [ctxp, dp, dp, vp]
    lib.dg_tree_limit.argtypes = [ctxp, dp, vp]
    lib.dg_destroy.argtypes = [ctxp]
    lib.dg_destroy.restype = None
    lib.dg_strerror.argtypes = [C.c_int]
    lib.dg_strerror.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("dg_destroy", "dg_strerror"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load_library().dg_strerror(code).decode()


def _check(code: int, what: str) -> None:
    if code != DG_OK:
        raise DGError(code, what)


def make_config(wl: dict, precision: str = "fp64") -> dg_config:
    c = dg_config()
    c.dim = wl["dim"]; c.k = wl["k"]
    c.n[:] = list(wl["n"])
    c.x0[:] = list(wl["x0"]); c.len[:] = list(wl["length"])
    c.gamma = wl["gamma"]; c.cfl = wl["cfl"]
    c.bc[:] = list(wl.get("bc", (0, 0, 0)))
    c.flux = wl.get("flux", 0)
    c.precision = PRECISIONS[precision]
    c.slope_limiter = wl.get("limiter", 0)
    c.beta = wl.get("beta", 1.0); c.m_tilde = wl.get("mtilde", 0.5)
    c.positivity = wl.get("positivity", 0); c.eps = wl.get("eps", 1e-10)
    c.refine_lo[:] = list(wl.get("refine_lo", (0, 0, 0)))
    c.refine_hi[:] = list(wl.get("refine_hi", (0, 0, 0)))
    c.tile2d = wl.get("tile2d", DG_TILE2D_AUTO)
    c.path3d = wl.get("path3d", DG_PATH3D_AUTO)
    return c


def _ptr(t, numel: int | None = None) -> int:
    """Device pointer of a contiguous float64 CUDA tensor of the expected size."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"tensor has {t.numel()} elements, expected {numel}")
    return t.data_ptr()


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Solver:
    """A configured DG discretisation on the current GPU (one libdg context)."""

    def __init__(self, wl: dict, precision: str = "fp64"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libdg needs a GPU: no HIP device is visible")
        self.lib = load_library()
        self.wl = dict(wl)
        self.precision = precision
        self.cfg = make_config(wl, precision)
        ctx = C.c_void_p()
        torch.cuda.init()
        _check(self.lib.dg_init(C.byref(self.cfg), C.byref(ctx)), "dg_init")
        self.ctx = ctx
        sz = (C.c_int64 * 6)()
        _check(self.lib.dg_sizes(self.ctx, sz), "dg_sizes")
        self.nvar, self.N, self.Q, self.Qf, self.ncell, self.nS = (int(x) for x in sz)
        nz = wl["n"][2] if wl["dim"] == 3 else 1
        self.shape = (self.nvar, self.N, nz, wl["n"][1], wl["n"][0])
        self.dx = wl["length"][0] / wl["n"][0]
        self.size = self.nvar * self.N * self.ncell
        az = (C.c_int64 * 5)()
        _check(self.lib.dg_amr_sizes(self.ctx, az), "dg_amr_sizes")
        self.ncoarse, self.nfine = int(az[0]), int(az[1])
        self.nf = tuple(int(x) for x in az[2:5])
        self.amr = self.nfine > 0
        self.nhole = 0
        if self.amr:
            self.shape = (self.size,)
            self.nhole = 1
            for a in range(wl["dim"]):
                self.nhole *= wl["refine_hi"][a] - wl["refine_lo"][a]
        self.rk = wl.get("rk", "rk3")
        self.stages = 3
        if self.rk != "rk3":
            self.set_tableau(*TABLEAUS[self.rk])
        self.gravity = None
        if wl.get("gravity") is not None:
            # the workload's external acceleration at the library's volume nodes
            import torch
            import workloads
            x = self.node_coords()
            acc = np.stack(workloads.acceleration(self.wl, x[0], x[1], x[2]))
            self.set_gravity(torch.from_numpy(np.ascontiguousarray(acc)).cuda())

    def _s(self, t) -> int:
        return _ptr(t, self.size)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self.lib.dg_destroy(ctx)
            self.ctx = None

    # -- buffers -----------------------------------------------------------
    def empty(self):
        import torch
        return torch.empty(self.shape, dtype=torch.float64, device="cuda")

    def scalar(self):
        import torch
        return torch.zeros(1, dtype=torch.float64, device="cuda")

    # -- set-up ------------------------------------------------------------
    def quadrature(self):
        xi = np.zeros((self.Q, 3)); w = np.zeros(self.Q)
        _check(self.lib.dg_quadrature(self.ctx, xi.ctypes.data_as(C.POINTER(C.c_double)),
                                      w.ctypes.data_as(C.POINTER(C.c_double))), "dg_quadrature")
        return xi, w

    def node_coords(self) -> np.ndarray:
        """Physical coordinates [3][Q][cells] of the Gauss nodes (host); with a
        refined box the coarse block's cells come first, then the fine block's."""
        xi, _ = self.quadrature()
        blocks = [(self.wl["n"], self.wl["x0"], self.dx)]
        if self.amr:
            lo = self.wl["refine_lo"]
            x0f = [self.wl["x0"][a] + lo[a] * self.dx for a in range(3)]
            blocks.append((self.nf, x0f, 0.5 * self.dx))
        parts = []
        for n, x0, h in blocks:
            nc = n[0] * n[1] * (n[2] if self.wl["dim"] == 3 else 1)
            cid = np.arange(nc)
            idx = [cid % n[0], (cid // n[0]) % n[1], cid // (n[0] * n[1])]
            out = np.zeros((3, self.Q, nc))
            for a in range(self.wl["dim"]):
                out[a] = x0[a] + (idx[a][None, :] + 0.5 + 0.5 * xi[:, a][:, None]) * h
            parts.append(out)
        return np.concatenate(parts, axis=2)

    def project(self, prim, out=None, stream=None):
        """L2 projection of primitives prim[5][Q][cells] (device) onto the basis."""
        out = self.empty() if out is None else out
        _check(self.lib.dg_project(self.ctx, _ptr(prim, 5 * self.Q * self.ncell), self._s(out), _stream(stream)),
               "dg_project")
        return out

    # -- the hot path ----------------------------------------------------------
    def rhs(self, w, out=None, stream=None):
        out = self.empty() if out is None else out
        _check(self.lib.dg_rhs(self.ctx, self._s(w), self._s(out), _stream(stream)), "dg_rhs")
        return out

    def max_dt(self, w, dt=None, stream=None):
        dt = self.scalar() if dt is None else dt
        _check(self.lib.dg_max_dt(self.ctx, self._s(w), _ptr(dt, 1), _stream(stream)), "dg_max_dt")
        return dt

    def rk_stage(self, stage, dt, wn, wp, out=None, stream=None):
        out = self.empty() if out is None else out
        wn_p = self._s(wn) if wn is not None else None
        _check(self.lib.dg_rk_stage(self.ctx, stage, _ptr(dt, 1), wn_p, self._s(wp), self._s(out), _stream(stream)),
               "dg_rk_stage")
        return out

    def rate_state(self):
        """A zeroed device rate state (DG_RATE_STATE doubles) for max_rate / rk_step."""
        import torch
        return torch.zeros(DG_RATE_STATE, dtype=torch.float64, device="cuda")

    @staticmethod
    def rate_value(rate) -> float:
        """The maximum signal rate a rate state holds (its largest slot)."""
        return float(rate[::RATE_STRIDE][:RATE_SLOTS].max())

    def max_rate(self, w, rate=None, stream=None):
        """Rate state (maximum signal rate of w's cell means) into a device tensor."""
        rate = self.rate_state() if rate is None else rate
        _check(self.lib.dg_max_rate(self.ctx, self._s(w), _ptr(rate, DG_RATE_STATE), _stream(stream)),
               "dg_max_rate")
        return rate

    def set_tableau(self, a, b):
        """Time integrator of tableau_stage / tableau_step (and of rk_step and
        step when it is not SSP-RK3): Butcher matrix a (s x s, row-major or
        nested) and weights b."""
        b = [float(x) for x in b]
        a = [float(x) for x in np.asarray(a, dtype=np.float64).ravel()]
        s = len(b)
        if len(a) != s * s:
            raise ValueError("a must have stages x stages entries")
        _check(self.lib.dg_set_tableau(self.ctx, s, (C.c_double * (s * s))(*a), (C.c_double * s)(*b)),
               "dg_set_tableau")
        self.stages = s
        self.rk = next((k for k, (ta, tb) in TABLEAUS.items() if list(ta) == a and list(tb) == b), "custom")

    def set_gravity(self, accel, stream=None):
        """External acceleration [dim][Q][ncell] at the volume nodes (device
        tensor), or None to switch gravity off."""
        ptr = _ptr(accel, self.wl["dim"] * self.Q * self.ncell) if accel is not None else None
        _check(self.lib.dg_set_gravity(self.ctx, ptr, _stream(stream)), "dg_set_gravity")
        self.gravity = accel

    # -- adaptive refinement of the one-box mesh ------------------------------
    def amr_flags(self, w, wt=0.01, alpha=1.1, stream=None):
        """(flags, box): device int32 flags per base cell (Sec. 4.1) and, on
        the host, the library's refined box of the next mesh ((refine_lo,
        refine_hi): the flagged range plus the buffer layer, clipped), or
        None when there is none."""
        import torch
        nb = self.ncoarse if self.amr else self.ncell
        flags = torch.empty(nb, dtype=torch.int32, device="cuda")
        box = torch.empty(6, dtype=torch.int32, device="cuda")
        _check(self.lib.dg_amr_flags(self.ctx, self._s(w), wt, alpha, flags.data_ptr(), box.data_ptr(),
                                     _stream(stream)), "dg_amr_flags")
        b = box.cpu().tolist()
        if not any(b):
            return flags, None
        return flags, (tuple(b[:3]), tuple(b[3:]))

    def regrid(self, w, box, precision=None, stream=None):
        """(solver, state) on the same base grid with the refined box `box`
        ((lo, hi), or None for none), the state moved by L2 projection."""
        if self.rk == "custom":
            raise ValueError("regrid keeps the named integrators only")
        wl = dict(self.wl)
        wl["refine_lo"], wl["refine_hi"] = box if box is not None else ((0, 0, 0), (0, 0, 0))
        s = Solver(wl, precision or self.precision)
        out = s.empty()
        _check(self.lib.dg_amr_regrid(self.ctx, self._s(w), s.ctx, s._s(out), _stream(stream)), "dg_amr_regrid")
        return s, out

    def tableau_stage(self, m, dt, ys, out=None, stream=None):
        """Stage value Y_m of the configured tableau from ys = [Y_0, .., Y_{m-1}] (unlimited)."""
        if len(ys) != m:
            raise ValueError("tableau_stage needs the m stage values Y_0..Y_{m-1}")
        out = self.empty() if out is None else out
        ptrs = (C.c_void_p * m)(*[self._s(y) for y in ys])
        _check(self.lib.dg_tableau_stage(self.ctx, m, _ptr(dt, 1), ptrs, self._s(out), _stream(stream)),
               "dg_tableau_stage")
        return out

    def rk_step(self, w, bufs, dt, rate, stream=None):
        """One time step with limiters from w into bufs[s-1] (bufs[0..s-2] are
        the stage buffers; s = 3 for SSP-RK3) in one library call: dg_rk_step
        for SSP-RK3, dg_tableau_step otherwise.  rate (a rate_state()) holds
        the rate state of w on entry (max_rate, or the previous rk_step) and of
        the result on return; dt receives the step.  Returns bufs[s-1]."""
        if self.rk != "rk3":
            s = self.stages
            if len(bufs) < s:
                raise ValueError(f"rk_step needs {s} buffers")
            ptrs = (C.c_void_p * max(s - 1, 1))(*[self._s(b) for b in bufs[:s - 1]])
            _check(self.lib.dg_tableau_step(self.ctx, self._s(w), ptrs, self._s(bufs[s - 1]), _ptr(dt, 1),
                                            _ptr(rate, DG_RATE_STATE), _stream(stream)), "dg_tableau_step")
            return bufs[s - 1]
        u1, u2, out = bufs[0], bufs[1], bufs[2]
        _check(self.lib.dg_rk_step(self.ctx, self._s(w), self._s(u1), self._s(u2), self._s(out), _ptr(dt, 1),
                                   _ptr(rate, DG_RATE_STATE), _stream(stream)), "dg_rk_step")
        return out

    def limit(self, w, stream=None):
        _check(self.lib.dg_limit(self.ctx, self._s(w), _stream(stream)), "dg_limit")
        return w

    def adjoint_rhs(self, w, lam, out=None, stream=None):
        out = self.empty() if out is None else out
        _check(self.lib.dg_adjoint_rhs(self.ctx, self._s(w), self._s(lam), self._s(out), _stream(stream)),
               "dg_adjoint_rhs")
        return out

    def adjoint_rk_stage(self, stage, dt, u, lam, acc, lam_out, acc_out, stream=None):
        _check(self.lib.dg_adjoint_rk_stage(self.ctx, stage, _ptr(dt, 1), self._s(u), self._s(lam),
                                            self._s(acc) if acc is not None else None, self._s(lam_out),
                                            self._s(acc_out) if acc_out is not None else None, _stream(stream)),
               "dg_adjoint_rk_stage")
        return lam_out

    def status(self, stream=None) -> int:
        return self.lib.dg_status(self.ctx, _stream(stream))

    @property
    def limited(self) -> bool:
        return bool(self.cfg.slope_limiter or self.cfg.positivity)

    def step(self, w, bufs, dt=None, stream=None):
        """One step from w into bufs[s-1] using bufs[0..s-2] as stage buffers
        (the main loop of Sec. 4.5 without refinement; s = 3 for SSP-RK3),
        one call per stage and limiter.  If dt (a one-element device tensor)
        is None the CFL step is computed first into bufs[s].  Returns the new
        state tensor (bufs[s-1])."""
        if self.rk != "rk3":
            s = self.stages
            if dt is None:
                dt = self.max_dt(w, bufs[s], stream)
            ys = [w]
            for m in range(1, s + 1):
                out = self.tableau_stage(m, dt, ys, bufs[m - 1], stream)
                if self.limited:
                    self.limit(out, stream)
                ys.append(out)
            return ys[-1]
        u1, u2, u3 = bufs[0], bufs[1], bufs[2]
        if dt is None:
            dt = self.max_dt(w, bufs[3], stream)
        self.rk_stage(1, dt, None, w, u1, stream)
        if self.limited:
            self.limit(u1, stream)
        self.rk_stage(2, dt, w, u1, u2, stream)
        if self.limited:
            self.limit(u2, stream)
        self.rk_stage(3, dt, w, u2, u3, stream)
        if self.limited:
            self.limit(u3, stream)
        return u3


class TreeSolver(Solver):
    """A 2D run on a quadtree of leaves (Sec. 4) over the workload's base
    grid: `leaves` is an integer array [nleaf][3] of (level, ix, iy).  States
    are device tensors [nvar][N][nleaf] in the mesh's leaf order (after an
    adaptation, the Morton order the library chose: see `leaves`)."""

    def __init__(self, wl: dict, leaves):
        if wl["dim"] != 2:
            raise ValueError("quadtree meshes are 2D")
        super().__init__(dict(wl, refine_lo=(0, 0, 0), refine_hi=(0, 0, 0)))
        self.set_leaves(leaves)

    def set_leaves(self, leaves):
        lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 3))
        _check(self.lib.dg_tree_set(self.ctx, lv.shape[0], lv.ctypes.data_as(C.POINTER(C.c_int32))), "dg_tree_set")
        self._sync_leaves()

    def _sync_leaves(self):
        n = C.c_int64()
        _check(self.lib.dg_tree_size(self.ctx, C.byref(n)), "dg_tree_size")
        lv = np.zeros((n.value, 3), dtype=np.int32)
        _check(self.lib.dg_tree_leaves(self.ctx, lv.ctypes.data_as(C.POINTER(C.c_int32))), "dg_tree_leaves")
        self.leaves = lv.astype(np.int64)
        self.nleaf = n.value
        self.ncell = self.nleaf
        self.shape = (self.nvar, self.N, self.nleaf)
        self.size = self.nvar * self.N * self.nleaf

    def rhs(self, w, out=None, stream=None):
        out = self.empty() if out is None else out
        _check(self.lib.dg_tree_rhs(self.ctx, self._s(w), self._s(out), _stream(stream)), "dg_tree_rhs")
        return out

    def max_dt(self, w, dt=None, stream=None):
        dt = self.scalar() if dt is None else dt
        _check(self.lib.dg_tree_max_dt(self.ctx, self._s(w), _ptr(dt, 1), _stream(stream)), "dg_tree_max_dt")
        return dt

    def rk_stage(self, stage, dt, wn, wp, out=None, stream=None):
        out = self.empty() if out is None else out
        wn_p = self._s(wn) if wn is not None else None
        _check(self.lib.dg_tree_rk_stage(self.ctx, stage, _ptr(dt, 1), wn_p, self._s(wp), self._s(out),
                                         _stream(stream)), "dg_tree_rk_stage")
        return out

    def limit(self, w, stream=None):
        _check(self.lib.dg_tree_limit(self.ctx, self._s(w), _stream(stream)), "dg_tree_limit")
        return w

    def step(self, w, bufs, dt=None, stream=None):
        """One SSP-RK3 step from w into bufs[2] (bufs[0..1] stage buffers,
        bufs[3] the time step when dt is None), the limiters after every stage
        when configured."""
        if dt is None:
            dt = self.max_dt(w, bufs[3], stream)
        self.rk_stage(1, dt, None, w, bufs[0], stream)
        if self.limited:
            self.limit(bufs[0], stream)
        self.rk_stage(2, dt, w, bufs[0], bufs[1], stream)
        if self.limited:
            self.limit(bufs[1], stream)
        self.rk_stage(3, dt, w, bufs[1], bufs[2], stream)
        if self.limited:
            self.limit(bufs[2], stream)
        return bufs[2]

    def adapt(self, w, wt=0.01, alpha=1.1, max_level=3, stream=None):
        """Plans the next mesh from w and moves w onto it (Sec. 4.1-4.3);
        returns the new state tensor (the mesh in `leaves` is updated)."""
        import torch
        n = C.c_int64()
        _check(self.lib.dg_tree_adapt(self.ctx, self._s(w), wt, alpha, max_level, C.byref(n), _stream(stream)),
               "dg_tree_adapt")
        out = torch.empty((self.nvar, self.N, n.value), dtype=torch.float64, device="cuda")
        _check(self.lib.dg_tree_regrid(self.ctx, self._s(w), _ptr(out, self.nvar * self.N * n.value),
                                       _stream(stream)), "dg_tree_regrid")
        self._sync_leaves()
        return out
