"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module holds the *problem definitions* only: mesh sizes, run lengths, the
initial primitive fields (density, velocity, pressure) of the paper's test
problems, and a counter-based random generator for the seeded noise.  It holds
none of the discontinuous Galerkin arithmetic (no basis, quadrature, projection,
flux or update): each consumer evaluates these fields at quadrature points it
computes itself and projects them with its own code.

Random numbers come from SplitMix64 (Steele, Lea & Flood 2014) used as a
counter-based generator: draw i of stream `seed` is mix(seed + (i+1)*GOLDEN),
so any subset of draws can be generated in any order.  U(-1,1) variates are
2*(z >> 11)*2^-53 - 1.

Problem sources (the paper's validation section):
  * isentropic vortex: primitive fields of the stationary vortex with
    strength beta = 5 plus a uniform boost (Validation, isentropic vortex);
  * shock tube: Sod states (1, 0, 1) | (0.125, 0, 0.1) (Validation, shock tube);
  * shear layer: the KH layer profile rho in {1, 2}, v_x = -/+0.5, p = 2.5
    (Validation, KH instability), here in 3D with cell-constant seeded
    velocity noise in place of the single-mode perturbation;
  * blast: a Sod-type spherical over-pressure region;
  * density wave: rho = 1 + 0.2 sin(2 pi (x + y)) advected at constant velocity
    and pressure;
  * KH instability (2D): the sharp two-layer setup with a single-mode v_y
    seed (Validation, KH instability);
  * cold Keplerian disc: a pressure-less ring on Keplerian orbits in a static
    softened central potential (Validation, Keplerian disc), with its
    external acceleration field (`acceleration`).
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter) -> np.ndarray:
    """Draw number `counter` (array of non-negative ints) of SplitMix64 stream `seed`."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, counter) -> np.ndarray:
    """U(-1, 1) variates from draw `counter` of stream `seed` (53-bit mantissa)."""
    z = splitmix64(seed, counter)
    return 2.0 * (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) - 1.0


def sign_direction(seed: int, size: int) -> np.ndarray:
    """A seeded direction of +-1 entries (sign of U(-1, 1) draws 0..size-1 of
    stream `seed`), used for finite-difference checks of gradients."""
    return np.where(uniform_pm1(seed, np.arange(size)) >= 0.0, 1.0, -1.0)


# ---------------------------------------------------------------------------
# Workload table.  Sizes follow the five benchmark configurations plus small
# variants used by tests.  `n` is the base grid, `x0`/`length` the box.
# ---------------------------------------------------------------------------

WORKLOADS: dict[str, dict] = {
    # 2D KH instability on [0,1]^2 (sharp layers at y = 0.25, 0.75, single-mode
    # v_y seed), DG-4 with RK_4, characteristic limiter + positivity, base grid
    # 64^2 refined where the density slope is steep (w_t = 0.01, alpha = 1.1).
    "kh2d": dict(dim=2, k=3, n=(64, 64, 1), x0=(0.0, 0.0, 0.0), length=(1.0, 1.0, 1.0), gamma=1.4, cfl=0.2,
                 limiter=2, positivity=1, eps=1e-8, ic="kh2d", rk="rk4", t_end=0.8, wt=0.01, alpha=1.1),
    # 2D cold Keplerian disc on [0,6]^2, gamma 5/3, to t = 120 (about 20 orbits
    # at r = 1), DG-2 with the positivity limiter only and the central
    # potential's acceleration as the gravity source.
    "kepler": dict(dim=2, k=1, n=(128, 128, 1), x0=(0.0, 0.0, 0.0), length=(6.0, 6.0, 1.0),
                   gamma=5.0 / 3.0, cfl=0.2, limiter=0, positivity=1, eps=1e-8, ic="kepler",
                   gravity="kepler", rk="rk2", t_end=120.0),
    # 2D, k=1, 32^2, smooth density wave, CFL 0.3, 20 steps, no limiter.
    "density_wave": dict(dim=2, k=1, n=(32, 32, 1), x0=(0.0, 0.0, 0.0),
                         length=(1.0, 1.0, 1.0), gamma=1.4, cfl=0.3, steps=20,
                         limiter=0, positivity=0, ic="density_wave",
                         velocity=(1.0, 1.0, 0.0)),
    # 2D, k=2, 256^2, boosted isentropic vortex on [-5,5]^2 with seeded
    # +-1e-3 density noise at every projection node; CFL 0.2, 200 steps.
    "vortex": dict(dim=2, k=2, n=(256, 256, 1), x0=(-5.0, -5.0, 0.0),
                   length=(10.0, 10.0, 1.0), gamma=1.4, cfl=0.2, steps=200,
                   limiter=0, positivity=0, ic="vortex", noise=1e-3, seed=1506),
    # 3D, k=2, 128^3 shear layer, minmod (TVB) + positivity, 10 steps.
    "kh3d": dict(dim=3, k=2, n=(128, 128, 128), x0=(0.0, 0.0, 0.0),
                 length=(1.0, 1.0, 1.0), gamma=1.4, cfl=0.2, steps=10,
                 limiter=1, positivity=1, ic="kh3d", noise=1e-2, seed=6140),
    # 2D, k=3, 512^2 boosted vortex (no noise), fixed dt, 400 steps, adjoint.
    "vortex_adjoint": dict(dim=2, k=3, n=(512, 512, 1), x0=(-5.0, -5.0, 0.0),
                           length=(10.0, 10.0, 1.0), gamma=1.4, cfl=0.2,
                           steps=400, limiter=0, positivity=0, ic="vortex",
                           checkpoint=20),
    # 3D, k=3 Sod-type blast on a 64^3 base grid whose central base cells
    # [16,48)^3 are refined 2:1; minmod + positivity, 10 steps.
    "blast_amr": dict(dim=3, k=3, n=(64, 64, 64), x0=(0.0, 0.0, 0.0),
                      length=(1.0, 1.0, 1.0), gamma=1.4, cfl=0.2, steps=10,
                      limiter=1, positivity=1, ic="blast",
                      refine_lo=(16, 16, 16), refine_hi=(48, 48, 48)),
    # 2D Sod shock tube on [0,1]^2 (transmissive in x, periodic in y).
    "sod": dict(dim=2, k=2, n=(64, 4, 1), x0=(0.0, 0.0, 0.0),
                length=(1.0, 1.0 / 16.0, 1.0), gamma=1.4, cfl=0.2,
                limiter=1, positivity=1, ic="sod", bc=(1, 0, 0), t_end=0.228),
}

VORTEX_BETA = 5.0
VORTEX_BOOST = (1.0, 1.0)
VORTEX_CENTRE = (0.0, 0.0)


def workload(name: str, **overrides) -> dict:
    """A copy of a named workload with fields overridden (e.g. n=(16,16,1))."""
    w = dict(WORKLOADS[name])
    w.update(overrides)
    w.setdefault("bc", (0, 0, 0))
    w.setdefault("beta", 1.0)
    w.setdefault("mtilde", 0.5)
    w.setdefault("eps", 1e-10)
    w.setdefault("refine_lo", (0, 0, 0))
    w.setdefault("refine_hi", (0, 0, 0))
    w.setdefault("flux", 0)
    w.setdefault("rk", "rk3")  # time integrator: "rk2", "rk3" or "rk4" (App. D tables)
    w.setdefault("gravity", None)  # external acceleration field (see acceleration), or None
    w["name"] = name
    return w


# Keplerian disc: background rho0 = p0 = 1e-5, disc density 1 between radii
# 0.5 and 2 with linear ramps of width 0.1, centre (3, 3), potential softened
# with eps = 0.25 inside r = 0.5 - 0.05.
KEPLER = dict(centre=(3.0, 3.0), rho0=1e-5, p0=1e-5, rho_disc=1.0, r_in=0.5, r_out=2.0, dr=0.1, soft=0.25)


def _kepler_primitives(x, y, over=None):
    k = dict(KEPLER, **(over or {}))
    dx, dy = x - k["centre"][0], y - k["centre"][1]
    r = np.sqrt(dx * dx + dy * dy)
    r_in, r_out, dr, r0, rd = k["r_in"], k["r_out"], k["dr"], k["rho0"], k["rho_disc"]
    rho = np.full_like(r, r0)
    ramp_in = (r >= r_in - dr / 2) & (r < r_in + dr / 2)
    rho = np.where(ramp_in, (rd - r0) / dr * (r - (r_in - dr / 2)) + r0, rho)
    rho = np.where((r >= r_in + dr / 2) & (r < r_out - dr / 2), rd, rho)
    ramp_out = (r >= r_out - dr / 2) & (r < r_out + dr / 2)
    rho = np.where(ramp_out, (r0 - rd) / dr * (r - (r_out - dr / 2)) + rd, rho)
    moving = (r > r_in - 2 * dr) & (r < r_out + 2 * dr)
    rs = np.where(r > 0.0, r, 1.0)
    vx = np.where(moving, -dy / rs ** 1.5, 0.0)
    vy = np.where(moving, dx / rs ** 1.5, 0.0)
    return rho, vx, vy, np.full_like(r, k["p0"])


def acceleration(wl: dict, x, y, z):
    """External acceleration a = -grad Phi of workload `wl` at points (x, y, z),
    as a tuple of `dim` arrays: the softened central field of the Keplerian
    disc, or a uniform vector (`gravity` = ("uniform", (gx, gy, gz)))."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    d = wl["dim"]
    gtype = wl["gravity"]
    if isinstance(gtype, (tuple, list)) and gtype[0] == "uniform":
        return tuple(np.full_like(x, gtype[1][a]) for a in range(d))
    if gtype == "kepler":
        k = KEPLER
        dx, dy = x - k["centre"][0], y - k["centre"][1]
        r = np.sqrt(dx * dx + dy * dy)
        outer = r > k["r_in"] - 0.5 * k["dr"]
        rs = np.where(r > 0.0, r, 1.0)
        inv = np.where(outer, 1.0 / rs ** 3, 1.0 / (rs * (rs * rs + k["soft"] ** 2)))
        inv = np.where(r > 0.0, inv, 0.0)
        return (-dx * inv, -dy * inv)
    raise ValueError(f"unknown gravity field {gtype!r}")


def _wrap(d: np.ndarray, length: float) -> np.ndarray:
    """Minimum-image offset in a periodic box of the given length."""
    return d - length * np.round(d / length)


def primitives(wl: dict, x, y, z, cell=None, node=None, t: float = 0.0):
    """Primitive fields (rho, vx, vy, vz, p) of workload `wl` at points (x, y, z).

    `cell` and `node` (integer arrays broadcastable with x) index the seeded
    noise counters; `nq` in the workload (nodes per cell) must be set by the
    caller for node-level noise.  `t` > 0 gives the exact solution of the
    translating problems (density wave, boosted vortex) at time t.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    g = wl["gamma"]
    ic = wl["ic"]
    zeros = np.zeros_like(x)
    if ic == "density_wave":
        u, v, w = wl.get("velocity", (1.0, 1.0, 0.0))
        rho = 1.0 + 0.2 * np.sin(2.0 * math.pi * (x + y - (u + v) * t))
        return rho, zeros + u, zeros + v, zeros + w, zeros + 1.0
    if ic == "vortex":
        bx, by = VORTEX_BOOST
        dx = _wrap(x - VORTEX_CENTRE[0] - bx * t, wl["length"][0])
        dy = _wrap(y - VORTEX_CENTRE[1] - by * t, wl["length"][1])
        r2 = dx * dx + dy * dy
        b = VORTEX_BETA
        rho = (1.0 - (g - 1.0) * b * b / (8.0 * g * math.pi ** 2)
               * np.exp(1.0 - r2)) ** (1.0 / (g - 1.0))
        p = rho ** g
        e = b / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
        vx = bx - dy * e
        vy = by + dx * e
        if wl.get("noise") and t == 0.0:
            if cell is None or node is None:
                raise ValueError("vortex noise needs cell and node indices")
            ctr = np.asarray(cell, dtype=np.int64) * int(wl["nq"]) + np.asarray(node, dtype=np.int64)
            rho = rho + wl["noise"] * uniform_pm1(wl["seed"], ctr)
        return rho, vx, vy, zeros, p
    if ic == "kh3d":
        inner = (y > 0.25) & (y < 0.75)
        rho = np.where(inner, 2.0, 1.0)
        vx = np.where(inner, 0.5, -0.5)
        vy = zeros.copy()
        vz = zeros.copy()
        if wl.get("noise"):
            if cell is None:
                raise ValueError("kh3d noise needs cell indices")
            c3 = np.asarray(cell, dtype=np.int64) * 3
            vx = vx + wl["noise"] * uniform_pm1(wl["seed"], c3 + 0)
            vy = vy + wl["noise"] * uniform_pm1(wl["seed"], c3 + 1)
            vz = vz + wl["noise"] * uniform_pm1(wl["seed"], c3 + 2)
        return rho, vx, vy, vz, zeros + 2.5
    if ic == "blast":
        r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
        inside = r2 < 0.2 ** 2
        return (np.where(inside, 1.0, 0.125), zeros, zeros, zeros,
                np.where(inside, 1.0, 0.1))
    if ic == "sod":
        left = x < 0.5
        return (np.where(left, 1.0, 0.125), zeros, zeros, zeros,
                np.where(left, 1.0, 0.1))
    if ic == "poly_contact":
        # a polynomial density sum_t c x^ex y^ey z^ez advected at constant
        # velocity and pressure (a contact): exact for degree <= k
        rho = zeros + 0.0
        for c, ex, ey, ez in wl["poly"]:
            rho = rho + c * x ** ex * y ** ey * z ** ez
        vel = wl.get("velocity", (0.7, -0.4, 0.3))
        return rho, zeros + vel[0], zeros + vel[1], zeros + vel[2], zeros + wl.get("pressure", 1.0)
    if ic == "kh2d":
        inner = (y > 0.25) & (y < 0.75)
        sig = 0.05 / math.sqrt(2.0)
        vy = 0.1 * np.sin(4.0 * math.pi * x) * (np.exp(-(y - 0.25) ** 2 / (2 * sig * sig))
                                                + np.exp(-(y - 0.75) ** 2 / (2 * sig * sig)))
        return np.where(inner, 2.0, 1.0), np.where(inner, 0.5, -0.5), vy, zeros, zeros + 2.5
    if ic == "kepler":
        # `kepler_params` may override the background values (rho0, p0)
        rho, vx, vy, p = _kepler_primitives(x, y, wl.get("kepler_params"))
        return rho, vx, vy, zeros, p
    if ic == "uniform":
        rho0, vel, p0 = wl["state"]
        return (zeros + rho0, zeros + vel[0], zeros + vel[1], zeros + vel[2],
                zeros + p0)
    raise ValueError(f"unknown initial condition {ic!r}")


# ---------------------------------------------------------------------------
# Quadtree leaf sets (2D): seeded synthetic meshes with several refinement
# levels for the tree path.  A leaf is (level, ix, iy), level 0 the base grid
# n, a level-l leaf one of the 4^l cells of a base cell.  These are inputs
# (which cells exist), not the method's refinement logic: the generator refines
# where a predicate or a seeded coin says so and then splits any leaf whose
# eight neighbours (faces and corners) are more than one level finer.
# ---------------------------------------------------------------------------

def _balance(leaves: set, n, periodic=(True, True)) -> set:
    """Split leaves until every leaf's face and corner neighbours differ from
    it by at most one level."""
    leaves = set(leaves)

    def covering(l, x, y):
        # the leaf containing cell (x, y) of level l, if it is that cell or coarser
        for m in range(l, -1, -1):
            key = (m, x >> (l - m), y >> (l - m))
            if key in leaves:
                return key
        return None

    changed = True
    while changed:
        changed = False
        for (l, x, y) in sorted(leaves, key=lambda t: -t[0]):
            if l < 2 or (l, x, y) not in leaves:
                continue
            nx, ny = n[0] << l, n[1] << l
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    if dx == 0 and dy == 0:
                        continue
                    xx, yy = x + dx, y + dy
                    if not (0 <= xx < nx):
                        if not periodic[0]:
                            continue
                        xx %= nx
                    if not (0 <= yy < ny):
                        if not periodic[1]:
                            continue
                        yy %= ny
                    c = covering(l, xx, yy)
                    if c is not None and c[0] < l - 1:
                        leaves.discard(c)
                        cl, cx, cy = c
                        for q in range(4):
                            leaves.add((cl + 1, 2 * cx + (q & 1), 2 * cy + (q >> 1)))
                        changed = True
    return leaves


def _morton(leaves, lmax):
    def key(t):
        l, x, y = t
        x <<= lmax - l
        y <<= lmax - l
        k = 0
        for b in range(40):
            k |= ((x >> b) & 1) << (2 * b) | ((y >> b) & 1) << (2 * b + 1)
        return k
    return sorted(leaves, key=key)


def tree_leaves(n, levels: int, refine, periodic=(True, True)) -> np.ndarray:
    """Leaf array [nleaf][3] of (level, ix, iy) in Morton order: starting from
    the base grid n (2D), `levels` passes each split the leaves of the current
    finest level for which refine(level, ix, iy) is true, followed by the
    one-level balance of faces and corners."""
    leaves = {(0, x, y) for x in range(n[0]) for y in range(n[1])}
    for l in range(levels):
        new = set()
        for t in leaves:
            if t[0] == l and refine(*t):
                new.update((l + 1, 2 * t[1] + (q & 1), 2 * t[2] + (q >> 1)) for q in range(4))
            else:
                new.add(t)
        leaves = _balance(new, n, periodic)
    lmax = max(t[0] for t in leaves)
    return np.array(_morton(leaves, lmax), dtype=np.int64).reshape(-1, 3)


def random_tree(n, levels: int, frac: float, seed: int, periodic=(True, True)) -> np.ndarray:
    """Seeded random quadtree: each pass splits a leaf of the finest level with
    probability `frac` (draw = the leaf's own index on its level)."""
    def refine(l, x, y):
        idx = (y * (n[0] << l) + x) + sum((n[0] * n[1]) << (2 * m) for m in range(l))
        return float(uniform_pm1(seed, idx)) < 2.0 * frac - 1.0
    return tree_leaves(n, levels, refine, periodic)


def band_tree(n, levels: int, y_bands=(0.25, 0.75), width: float = 0.0, length=(1.0, 1.0)) -> np.ndarray:
    """Quadtree refined around horizontal lines y = y_b (the two shear layers
    of the KH setup): a leaf is split if its y range comes within `width` of a
    line."""
    def refine(l, x, y):
        h = length[1] / (n[1] << l)
        y0, y1 = y * h, (y + 1) * h
        return any(y0 - width <= yb <= y1 + width for yb in y_bands)
    return tree_leaves(n, levels, refine)
