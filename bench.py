#!/usr/bin/env python3
"""Benchmark of the DG right-hand side + SSP-RK3 hot path on one MI355X.

Headline workload: 3D Kelvin-Helmholtz shear layer on the periodic unit cube,
128^3 cells, degree k = 2 (N = 10 modes, 5 variables), FP64, layers rho = 2,
v_x = +0.5 for 1/4 < y < 3/4 and rho = 1, v_x = -0.5 outside, p = 2.5, gamma
1.4, seeded cell-constant velocity noise of 1e-2 (seed 6140), CFL 0.2, the
component-wise TVB minmod limiter and the positivity limiter after every
stage.  This is the largest of the five workloads that fits one GPU as a
uniform grid.  One *step* is the whole hot path for one SSP-RK3 step: the
time step from the carried signal rate, three fused RHS + stage kernels and
the limiter pass after each stage, issued by one dg_rk_step call and
replayed from a HIP graph.  The metric is DOF-updates per second per RK
stage: cells * N * 3 / step time.

The initial state is built by the library itself (seeded primitives from
``workloads`` sampled at the library's Gauss nodes, L2-projected by
``dg_project``, then limited); it is resident in HBM before the timed region
starts.

The `roofline` object is for the dominant kernel, the fused 3D RHS + stage
kernel, against its binding roof, the FP64 vector peak (algorithmic flops
per launch over the launch's mean duration, timed with HIP events on the
stream it runs on), with its HBM fraction beside it; `traffic` is the HBM
bytes per launch from the committed rocprofv3 counter summary while that
summary's kernel-source fingerprint matches the source.  The 2D vortex
(256^2, k = 2) line, the FP32 / BF16 paths, the refined-box blast, the
adaptive 2D KH run and the adjoint are reported under `variants`.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on a
single GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
METRIC = "DOF-updates/s per RK stage"
KERNEL_SRC = os.path.join(ROOT, "paper_1506_06140_amd", "csrc", "dg_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")

# source regions whose text fingerprints a kernel (a counter summary taken on
# another version of the kernel is not reported)
_HELPERS = [
    # reciprocal helpers, the time-step rate, the Euler flux, the Riemann solver
    ("// Reciprocal and reciprocal square root from the hardware estimates plus",
     "// HLLC numerical flux in +a between traces UL (low side) and UR (high side),"),
    ("// HLLC numerical flux in +a between traces UL (low side) and UR (high side),",
     "// ---------------------------------------------------------------------------\n// Right-hand side and fused stage."),
]
KERNELS = {
    "stage3d": dict(name="k_rhs_mfma3d<2>", traffic="k_rhs_mfma3d_kh3d128_k2_traffic.txt",
                    regions=_HELPERS + [("// 3D right-hand side + stage with the contractions on MFMA (FP64; FP32 and",
                                         "// Discrete adjoint of the right-hand side and of the SSP-RK3 stages.")]),
    "stage3d_amr": dict(name="k_rhs_mfma3d<3,AMR>", traffic="k_rhs_mfma3d_blast64box_k3_traffic.txt",
                        regions=_HELPERS + [("// 3D right-hand side + stage with the contractions on MFMA (FP64; FP32 and",
                                             "// Discrete adjoint of the right-hand side and of the SSP-RK3 stages.")]),
    "stage3d_valu": dict(name="k_rhs_stage<3,2,double>", traffic="k_rhs_stage_kh3d128_k2_traffic.txt",
                         regions=_HELPERS + [("// Right-hand side and fused stage.",
                                              "// 2D right-hand side + SSP-RK3 stage on LDS tiles, four lanes per cell.")]),
    "tile2d": dict(name="k_rhs_tile2d<2,double> (8x8 tiles)", traffic="k_rhs_tile2d_vortex256_k2_traffic.txt",
                   regions=_HELPERS + [("// 2D right-hand side + SSP-RK3 stage on LDS tiles, four lanes per cell.",
                                        "// 3D right-hand side + stage with the contractions on MFMA (FP64; FP32 and")]),
}


def alg_work(d: int, k: int):
    """Algorithmic bytes and flops per cell per RK stage (fused RHS + stage,
    each face evaluated once): 8/3 state passes; modal->nodal, projection onto
    the basis gradients, both traces of the d owned faces and the lifting as
    dense multiply-adds (2 flops each), about 12 flops per volume node and
    direction for the Euler flux and 110 per face node for HLLC."""
    nvar = d + 2
    n1 = k + 1
    N = (k + 1) * (k + 2) // 2 if d == 2 else (k + 1) * (k + 2) * (k + 3) // 6
    Q = n1 ** d
    QF = Q // n1
    bytes_ = 8.0 / 3.0 * nvar * N * 8
    flops = (2 * nvar * N * Q + 2 * d * nvar * Q * (N - 1) + 2 * (2 * 2 * d * nvar * N * QF)
             + 12 * Q * d + 110 * d * QF)
    return bytes_, float(flops)


def kernel_hash(kernel: str) -> str:
    """Fingerprint of the source of a benchmarked kernel (its own region plus
    the Riemann solver and the reciprocal helpers)."""
    src = open(KERNEL_SRC).read()
    parts = []
    for a, b in KERNELS[kernel]["regions"]:
        i = src.find(a)
        j = src.find(b, i + 1) if i >= 0 else -1
        if i < 0 or j < 0:
            raise RuntimeError(f"kernel fingerprint marker not found in {KERNEL_SRC}: {a if i < 0 else b!r}")
        parts.append(src[i:j])
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, or None if absent or taken on a different kernel source."""
    path = os.path.join(PROFILES, KERNELS[kernel]["traffic"])
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*(\w+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_hash(kernel):
        return None
    return float(b.group(1))


def build_state(s, wl):
    import torch
    x = s.node_coords()  # [3][Q][cells]
    cell = np.broadcast_to(np.arange(s.ncell)[None, :], (s.Q, s.ncell))
    node = np.broadcast_to(np.arange(s.Q)[:, None], (s.Q, s.ncell))
    wlq = dict(wl)
    wlq["nq"] = s.Q
    prim = np.stack(workloads.primitives(wlq, x[0], x[1], x[2], cell=cell, node=node), axis=0)
    prim_d = torch.from_numpy(np.ascontiguousarray(prim)).cuda()
    w = s.project(prim_d)
    torch.cuda.synchronize()
    return w


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, slab: int = 64):
    """The FP64 oracle (single-threaded C, built -O2 -ffp-contract=off),
    pinned to one host core, on a bounded sample of the headline workload:
    one limited SSP-RK3 stage (right-hand side, stage update, slope and
    positivity limiters) of the cells in `slab` z-planes of the full 128^3
    state (the oracle's per-cell entries; the work per cell is that of the
    whole mesh)."""
    import oracle
    o = oracle.Oracle(wl)
    w0 = o.initial_state()
    w0, _ = o.limit(w0)
    dt = o.max_dt(w0)
    nxy = wl["n"][0] * wl["n"][1]
    cells = np.arange(slab * nxy, dtype=np.int64)
    aff = os.sched_getaffinity(0)
    core = min(aff)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        L = o.rhs_cells(w0, cells)
        wc = w0.reshape(o.nvar, o.N, -1)[:, :, cells]
        u = oracle.rk3_combine(1, dt, wc, wc, L)
        t1 = time.perf_counter()
        full = w0.copy()
        full.reshape(o.nvar, o.N, -1)[:, :, cells] = u
        t2 = time.perf_counter()
        o.limit_cells(full, cells)
        t3 = time.perf_counter()
    finally:
        os.sched_setaffinity(0, aff)
    el = (t1 - t0) + (t3 - t2)
    dof = cells.size * o.N
    return {"value": dof / el, "unit": METRIC, "cores": 1, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus": len(aff), "pinned_core": core,
            "sample": f"one limited SSP-RK3 stage (RHS + update {t1 - t0:.2f} s, limiters {t3 - t2:.2f} s) of "
                      f"{cells.size} cells ({slab} z-planes) of the 128^3 k=2 shear-layer state, single-threaded "
                      f"C oracle pinned to core {core} (sched_setaffinity, as taskset) of {len(aff)}"}


def cpu_other_workloads():
    """The oracle, pinned to one host core, on bounded samples of the two
    other 3D/adjoint workloads (context beside the headline's CPU leg):
    the refined blast (64^3 + the 64^3-cell fine box, k=3): one SSP-RK3
    stage (RHS, update, limiters) of two coarse z-planes through the box
    and two fine z-planes, on the full-size initial projection (the
    whole-mesh limiting that precedes the run, about 45 s on one core, is
    left out); one whole-mesh stage of the 2D vortex at 512^2, k=3 (the
    adjoint workload's forward pass); and one limited stage of 2 000 leaves
    of the quadtree KH mesh."""
    import oracle
    aff = os.sched_getaffinity(0)
    core = min(aff)
    out = {}
    wl = workloads.workload("blast_amr")
    o = oracle.AmrOracle(wl)
    w0 = o.initial_state()
    dt = o.max_dt(w0)
    n, (nfx, nfy, nfz) = wl["n"], o.nf
    zc = (wl["refine_lo"][2] + wl["refine_hi"][2]) // 2
    cc = np.arange((zc - 1) * n[0] * n[1], (zc + 1) * n[0] * n[1], dtype=np.int64)
    cc = cc[~o.hole[cc]]
    cf = o.ncoarse + np.arange((nfz // 2 - 1) * nfx * nfy, (nfz // 2 + 1) * nfx * nfy, dtype=np.int64)
    cells = np.concatenate([cc, cf])
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        L = o.rhs_cells(w0, cells)
        wc = o.cells_of(w0, cells)
        oracle.rk3_combine(1, dt, wc, wc, L)
        t1 = time.perf_counter()
        o.limit_cells(w0, cells)
        t2 = time.perf_counter()
    finally:
        os.sched_setaffinity(0, aff)
    out["blast_amr_64box_k3"] = {
        "value": cells.size * o.N / (t2 - t0), "unit": METRIC, "cores": 1, "kind": "oracle",
        "sample": f"one limited SSP-RK3 stage (RHS + update {t1 - t0:.2f} s, limiters {t2 - t1:.2f} s) of "
                  f"{cc.size} coarse cells (2 z-planes through the box) and {cf.size} fine cells (2 z-planes) of the "
                  f"full-size k=3 blast, single-threaded C oracle pinned to core {core}"}
    wl = workloads.workload("vortex_adjoint")
    o = oracle.Oracle(wl)
    w0 = o.initial_state()
    dt = o.max_dt(w0)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        o.rk3_stage(1, dt, w0, w0)
        el = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, aff)
    out["vortex512_k3"] = {
        "value": o.ncell * o.N / el, "unit": METRIC, "cores": 1, "kind": "oracle",
        "sample": f"one SSP-RK3 stage of the full {wl['n'][0]}^2 k={wl['k']} vortex state ({el:.2f} s; the "
                  f"adjoint workload's forward pass), single-threaded C oracle pinned to core {core}"}
    # the quadtree KH mesh of the tree variant, built by the oracle's own
    # adaptation; one limited stage on 2 000 seeded leaves
    n = 64
    wl = workloads.workload("kh2d", rk="rk3", x0=(0.0, -0.3 / n, 0.0))
    leaves = np.array([(0, x, y) for y in range(n) for x in range(n)])
    o = oracle.TreeOracle(wl, leaves)
    w, _ = o.limit(o.initial_state())
    for _ in range(6):
        leaves, w = oracle.tree_adapt(wl, leaves, w, wl["wt"], wl["alpha"], 5)
    o = oracle.TreeOracle(wl, leaves)
    cells = np.unique((workloads.splitmix64(2015, np.arange(2000)) % np.uint64(len(leaves))).astype(np.int64))
    dt = o.max_dt(w)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        V, S, _ = o.terms_cells(w, cells)
        oracle.rk3_combine(1, dt, w[:, :, cells], w[:, :, cells], V - S)
        t1 = time.perf_counter()
        o.limit_cells(w, cells)
        t2 = time.perf_counter()
    finally:
        os.sched_setaffinity(0, aff)
    out["kh2d_tree_k3"] = {
        "value": cells.size * o.N / (t2 - t0), "unit": METRIC, "cores": 1, "kind": "oracle",
        "sample": f"one limited SSP-RK3 stage (RHS + update {t1 - t0:.2f} s, limiters {t2 - t1:.2f} s) of "
                  f"{cells.size} seeded leaves of the {len(leaves)}-leaf quadtree KH mesh (k=3); the oracle finds "
                  f"neighbours by a brute-force search over all leaves, so its cost per leaf grows with the mesh; "
                  f"single-threaded C oracle pinned to core {core}"}
    return out


def cpu_baseline_2d(wl, budget_s: float = 8.0):
    """The oracle on whole-mesh SSP-RK3 stages of the 2D vortex (256^2, k=2)."""
    import oracle
    o = oracle.Oracle(wl)
    w0 = o.initial_state()
    dt = o.max_dt(w0)
    aff = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {min(aff)})
    try:
        t0 = time.perf_counter()
        stages = 0
        u = w0
        while True:
            stage = stages % 3 + 1
            u = o.rk3_stage(stage, dt, w0, u if stage > 1 else w0)
            stages += 1
            if time.perf_counter() - t0 > budget_s and stages >= 3:
                break
        el = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, aff)
    return {"value": o.ncell * o.N * stages / el, "unit": METRIC, "cores": 1, "kind": "oracle",
            "sample": f"{stages} SSP-RK3 stages of the full 256^2 k=2 vortex state, {el:.1f} s"}


def time_steps(s, wl, steps, warmup, graph=True):
    """Time `steps` SSP-RK3 steps (time step + 3 stages [+ limiters]) of the
    workload on solver `s`; returns ms per step.  The state is built by the
    library's projection (and limited first if the workload limits)."""
    import torch
    A = build_state(s, wl)
    if s.limited:
        s.limit(A)
    B = s.empty()
    stage_bufs = [s.empty() for _ in range(s.stages - 1)]
    dtbuf, rate = s.scalar(), s.rate_state()
    stream = torch.cuda.current_stream()
    s.max_rate(A, rate)

    def two_steps():
        # one library call per step; the signal rate of the new state is
        # carried in `rate` to the next step's time step
        s.rk_step(A, stage_bufs + [B], dtbuf, rate)
        s.rk_step(B, stage_bufs + [A], dtbuf, rate)

    steps = steps + (steps % 2)
    for _ in range((warmup + 1) // 2):
        two_steps()
    torch.cuda.synchronize()
    g = None
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            two_steps()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            two_steps()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // 2):
        g.replay() if g is not None else two_steps()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = s.status()
    if st != 0:
        raise RuntimeError(f"device error flag {st} in {wl['name']}")
    return el / steps * 1e3, A


def variants():
    """The other figures of the metric: FP32 vs FP64, the 3D limited
    workload, and the adjoint/forward time ratio."""
    import torch
    import paper_1506_06140_amd as dg
    from paper_1506_06140_amd import adjoint
    out = {}
    # the refined-box blast in reduced precision needs a positivity floor above
    # the FP32 rounding of the energy (node pressures are formed in FP32)
    # (the *_char runs: the same workloads with the characteristic limiter;
    # DG-4 and DG-5: the vortex at k = 3 and k = 4 with the five-stage RK_4)
    runs = [("vortex", "vortex", 400, {}, ("fp32", "bf16")),
            ("vortex_dg4_rk4", "vortex", 200, {"k": 3, "rk": "rk4"}, ("fp64", "fp32")),
            ("vortex_dg5_rk4", "vortex", 200, {"k": 4, "rk": "rk4"}, ("fp64", "fp32")),
            ("kh3d", "kh3d", 10, {}, ("fp32", "bf16")),
            ("kh3d_char", "kh3d", 10, {"limiter": 2}, ("fp64",)),
            ("blast_amr", "blast_amr", 10, {"eps": 1e-4}, ("fp64", "fp32", "bf16")),
            ("blast_amr_char", "blast_amr", 10, {"eps": 1e-4, "limiter": 2}, ("fp64",))]
    for label, name, steps, over, precs in runs:
        wl = workloads.workload(name, **over)
        for prec in precs:
            s = dg.Solver(wl, prec)
            ms, _ = time_steps(s, wl, steps, 4)
            cells = (s.ncoarse - s.nhole + s.nfine) if s.amr else s.ncell
            b, f = alg_work(wl["dim"], wl["k"])
            peak = FP64_PEAK_TFLOPS if prec == "fp64" else FP32_PEAK_TFLOPS
            # fractions of one step's algorithmic work (all stages) over the
            # whole step time (time step and limiters included)
            ns = s.stages
            out[f"{label}_{prec}"] = {"ms_per_step": ms, "dof_updates_per_s": cells * s.N * ns / (ms * 1e-3),
                                     "cells": cells, "k": wl["k"], "dim": wl["dim"], "stages": ns,
                                     "limiter": wl["limiter"], "positivity": wl["positivity"],
                                     "eps": wl["eps"], "status": s.status(),
                                     "hbm_frac": ns * b * cells / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                                     "alu_frac": ns * f * cells / (ms * 1e-3) / (peak * 1e12),
                                     "alu_peak_tflops": peak}
            del s
            torch.cuda.empty_cache()
    # the stage kernels of the two 3D workloads per precision and path (one
    # fused RHS + stage launch, HIP events), with the limiter pass
    kinds = {
        "kh3d": ("3D shear layer 128^3, k=2", {},
                 {"fp64_mfma": "k_rhs_mfma3d<2>", "fp64_valu": "k_rhs_stage<3,2,double>",
                  "fp32_valu": "k_rhs_stage<3,2,float>", "fp32_mfma": None,
                  "bf16_mfma": "k_rhs_mfma3d<2,float,BF16 volume>"}),
        "blast_amr": ("3D blast, 64^3 base grid + refined 32^3 box (64^3 fine cells), k=3", {"eps": 1e-4},
                      {"fp64_mfma": "k_rhs_mfma3d<3,AMR>", "fp64_valu": "k_rhs_amr_quad<3>",
                       "fp32_valu": "k_rhs_amr<3,3,float>", "fp32_mfma": "k_rhs_mfma3d<3,AMR,float>",
                       "bf16_mfma": "k_rhs_mfma3d<3,AMR,float,BF16 volume>"}),
    }
    for name, (desc, over, kernels) in kinds.items():
        wl = workloads.workload(name, **over)
        rec = {"workload": desc, "kernels": {}}
        for label, kname in kernels.items():
            if kname is None:
                continue  # FP32 on a uniform k = 2 grid has no MFMA form (the VALU kernel is faster)
            prec, path = label.split("_")
            s = dg.Solver(dict(wl, path3d=dg.DG_PATH3D_VALU if path == "valu" else dg.DG_PATH3D_AUTO), prec)
            w = build_state(s, wl)
            s.limit(w)
            bufs = [s.empty(), s.empty(), s.empty(), s.scalar()]
            kms = kernel_ms(s, w, bufs, 10)
            cells = (s.ncoarse - s.nhole + s.nfine) if s.amr else s.ncell
            b3, f3 = alg_work(3, wl["k"])
            peak = FP64_PEAK_TFLOPS if prec == "fp64" else FP32_PEAK_TFLOPS
            rec["kernels"][label] = {"kernel": kname, "ms": kms, "alu_frac": f3 * cells / (kms * 1e-3) / 1e12 / peak,
                                     "alu_peak_tflops": peak}
            if label == "fp64_mfma":
                rec["limiter_ms"] = kernel_ms(s, w, bufs, 10, limiter=True)
                rec["cells"] = cells
                rec["alg_flops_per_launch"] = f3 * cells
            del s, w, bufs
            torch.cuda.empty_cache()
        out[f"{name}_stage_kernels"] = rec
    # adaptive KH (2D, 64^2 base, DG-4 with RK_4, characteristic limiter and
    # positivity): every 10 steps the flags (w_t = 0.01, alpha = 1.1), the box
    # around them with one buffer layer and, if it changed, the regrid
    wl = workloads.workload("kh2d")
    s = dg.Solver(wl)
    w = build_state(s, wl)
    s.limit(w)
    nsteps, every = 200, 10
    t_step = t_adapt = 0.0
    dof_stages = 0
    regrids = 0
    box = None
    for i in range(nsteps):
        if i % every == 0:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, nb = s.amr_flags(w, wl["wt"], wl["alpha"])
            if nb != box or i == 0:
                if nb != box:
                    s, w = s.regrid(w, nb)
                    regrids += 1
                    box = nb
                stage_bufs = [s.empty() for _ in range(s.stages - 1)]
                other, dtb, rate = s.empty(), s.scalar(), s.rate_state()
                s.max_rate(w, rate)
            torch.cuda.synchronize()
            t_adapt += time.perf_counter() - t0
        t0 = time.perf_counter()
        nxt = s.rk_step(w, stage_bufs + [other], dtb, rate)
        w, other = nxt, w
        torch.cuda.synchronize()
        t_step += time.perf_counter() - t0
        cells = (s.ncoarse - s.nhole + s.nfine) if s.amr else s.ncell
        dof_stages += cells * s.N * s.stages
    st = s.status()
    out_box = {"lo": list(box[0]), "hi": list(box[1])} if box else None
    out["kh2d_adaptive_fp64"] = {"steps": nsteps, "regrid_every": every, "regrids": regrids, "final_box": out_box,
                                 "ms_per_step": t_step / nsteps * 1e3, "dof_updates_per_s": dof_stages / t_step,
                                 "adapt_ms_per_check": t_adapt / (nsteps // every) * 1e3, "status": st}
    del s
    torch.cuda.empty_cache()
    out["kh2d_tree_fp64"] = tree_variant()
    torch.cuda.empty_cache()
    # adjoint: 512^2, k=3, J = int rho^2 after 400 steps at fixed dt, checkpoint 20
    wl = workloads.workload("vortex_adjoint")
    s = dg.Solver(wl)
    w0 = build_state(s, wl)
    dt = s.max_dt(w0)
    nsteps, ck = wl["steps"], wl["checkpoint"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = w0.clone().requires_grad_(True)
    wT = adjoint.trajectory(s, x, nsteps, dt, ck)
    J = adjoint.density_square_integral(s, wT)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = x.grad.detach()
    # central differences on the 64 seeded +-1 directions (SplitMix64 seeds
    # 1..64) scaled to |d| = |w0|, h = 1e-6, at the full size
    fd = []
    scale = float(torch.linalg.vector_norm(w0)) / w0.numel() ** 0.5
    h = 1e-6
    for seed in range(1, 65):
        d = torch.from_numpy(workloads.sign_direction(seed, w0.numel()).reshape(tuple(w0.shape))).to(w0.device) * scale
        with torch.no_grad():
            jp = float(adjoint.density_square_integral(s, adjoint.trajectory(s, w0 + h * d, nsteps, dt, nsteps)))
            jm = float(adjoint.density_square_integral(s, adjoint.trajectory(s, w0 - h * d, nsteps, dt, nsteps)))
        dJ = float((g * d).sum())
        fd.append(abs((jp - jm) / (2 * h) - dJ) / abs(dJ))
    out["adjoint_vortex512_k3"] = {"forward_s": t1 - t0, "backward_s": t2 - t1,
                                   "adjoint_over_forward": (t2 - t1) / (t1 - t0), "steps": nsteps,
                                   "checkpoint": ck, "J": float(J.detach()),
                                   "fd_directions": len(fd), "fd_rel_err_max_h1e-6": max(fd),
                                   "fd_rel_err_median_h1e-6": float(np.median(fd))}
    return out


def tree_variant(max_level: int = 5, steps: int = 100, reps: int = 30):
    """The KH setup on the quadtree (Sec. 4): base 64^2 (the paper's level 6),
    k = 3, SSP-RK3, characteristic limiter and positivity after every stage,
    the mesh adapted to the criterion (w_t = 0.01, alpha = 1.1) down to
    max_level levels below the base (the origin shifted by 0.3 base cells in
    y, so that the sharp layers cut cells on every level).  Times the step
    (time step, three fused RHS/stage launches, three limiter passes; graph
    replay, state resident), one adaptation (criterion, plan, regrid) and the
    stage kernel alone (HIP events)."""
    import torch
    import paper_1506_06140_amd as dg
    n = 64
    wl = workloads.workload("kh2d", rk="rk3", x0=(0.0, -0.3 / n, 0.0))
    leaves = np.array([(0, x, y) for y in range(n) for x in range(n)])
    s = dg.TreeSolver(wl, leaves)
    w = s.project(torch.from_numpy(np.ascontiguousarray(np.stack(
        _tree_prims(s, wl)))).cuda())
    s.limit(w)
    for _ in range(max_level + 1):
        w = s.adapt(w, wl["wt"], wl["alpha"], max_level)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w = s.adapt(w, wl["wt"], wl["alpha"], max_level)
    torch.cuda.synchronize()
    t_adapt = time.perf_counter() - t0
    A, B = w, s.empty()
    bufs = [s.empty(), s.empty()]
    dt = s.scalar()

    def two_steps():
        s.step(A, bufs + [B, dt])
        s.step(B, bufs + [A, dt])
    two_steps()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        two_steps()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        two_steps()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // 2):
        g.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    st = s.status()
    # the stage kernel alone: HIP events around `reps` launches on the stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.rk_stage(1, dt, None, A, bufs[0])
    ev0.record()
    for _ in range(reps):
        s.rk_stage(1, dt, None, A, bufs[0])
    ev1.record()
    torch.cuda.synchronize()
    kms = ev0.elapsed_time(ev1) / reps
    lv = s.leaves[:, 0]
    _, f3 = alg_work(2, 3)
    cells = int(s.nleaf)
    area = 0.25 ** lv
    rec = {"base": [n, n], "k": 3, "max_level": max_level, "leaves": cells,
           "leaves_per_level": np.bincount(lv).tolist(),
           "refined_leaf_fraction": float((lv > 0).mean()), "refined_area_fraction": float(area[lv > 0].sum() / area.sum()),
           "uniform_equivalent_cells": (n << max_level) ** 2,
           "ms_per_step": ms, "dof_updates_per_s": cells * s.N * 3 / (ms * 1e-3),
           "adapt_ms": t_adapt * 1e3, "stage_kernel": "k_rhs_tree<3,0>", "stage_kernel_ms": kms,
           "stage_kernel_alu_frac": f3 * cells / (kms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, "status": st}
    del s, A, B, bufs
    torch.cuda.empty_cache()
    return rec


def _tree_prims(s, wl):
    """Primitive fields of the workload at every leaf's volume nodes,
    [5][Q][nleaf] (the library projects them)."""
    xi, _ = s.quadrature()
    lv = s.leaves
    h = wl["length"][0] / wl["n"][0] / (2.0 ** lv[:, 0])
    x = wl["x0"][0] + h[None, :] * (lv[:, 1][None, :] + 0.5 * (1.0 + xi[:, 0][:, None]))
    y = wl["x0"][1] + h[None, :] * (lv[:, 2][None, :] + 0.5 * (1.0 + xi[:, 1][:, None]))
    wlq = dict(wl, nq=s.Q)
    return workloads.primitives(wlq, x, y, np.zeros_like(x))


def kernel_ms(s, w, bufs, reps, limiter=False):
    """Mean duration of the fused RHS + stage kernel of solver s (stages 1, 2,
    3 in turn from the state w, `reps` launches queued back to back, HIP
    events on the stream they run on), or with limiter=True of the limiter
    pass that follows each stage (the same sequence with the limiter after
    every stage, minus the stages alone): every pass limits a fresh stage
    output, as in a step."""
    import torch
    stream = torch.cuda.current_stream()
    bufs[0].copy_(w)  # the previous stage's state of stages 2 and 3
    dt = s.max_dt(w, bufs[3])

    def run(n, with_limit):
        for i in range(n):
            stage = i % 3 + 1
            out = bufs[1] if stage == 1 else bufs[2]
            s.rk_stage(stage, dt, w, w if stage == 1 else bufs[0], out)
            if with_limit:
                s.limit(out)

    def timed(with_limit):
        run(3, with_limit)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run(reps, with_limit)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_stage = timed(False)
    return timed(True) - t_stage if limiter else t_stage


def vortex2d_line(steps=400, warmup=20, with_cpu=True, reps=300, n=256, k=2, precision="fp64"):
    """The 2D vortex (n^2, degree k, no limiter) with its stage kernel's HBM
    roofline.  256^2, k = 2 (12.6 MB) stays in the 256 MB Infinity Cache;
    512^2, k = 3 is the adjoint workload's grid (84 MB, three states 252 MB)."""
    import paper_1506_06140_amd as dg
    wl = workloads.workload("vortex", n=(n, n, 1), k=k)
    s = dg.Solver(wl, precision)
    ms, w = time_steps(s, wl, steps, warmup)
    bufs = [s.empty(), s.empty(), s.empty(), s.scalar()]
    kms = kernel_ms(s, w, bufs, reps)
    b, f = alg_work(2, k)
    alg_bytes = b * s.ncell
    achieved = alg_bytes / (kms * 1e-3) / 1e9
    base = (n, k, precision) == (256, 2, "fp64")
    out = {"workload": f"isentropic vortex 2D, {n}x{n} cells, k={k} (N={s.N}), {precision.upper()}, SSP-RK3, "
                       "CFL 0.2, no limiter, seeded 1e-3 density noise",
           "ms_per_step": ms, "dof_updates_per_s": s.ncell * s.N * 3 / (ms * 1e-3),
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("tile2d") if base else None,
                        "kernel": f"k_rhs_tile2d<{k},{'double' if precision == 'fp64' else 'float'}>",
                        "kernel_ms": kms, "alg_bytes_per_launch": alg_bytes,
                        "fp64_frac": f * s.ncell / (kms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}}
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline_2d(wl)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--graph", type=int, default=1, help="replay the step as a HIP graph")
    ap.add_argument("--variants", type=int, default=1, help="also time FP32, the 3D workload and the adjoint")
    ap.add_argument("--kernel-reps", type=int, default=30, help="launches per kernel timing")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32"), help="2D vortex lines only")
    ap.add_argument("--workload", default="kh3d", choices=("kh3d", "blast_amr", "vortex", "vortex512"),
                    help="the timed workload: the 128^3 shear layer (the headline), the 64^3 blast with its refined "
                         "box (k = 3), or the 2D vortex 256^2 (its line alone, for profiling the 2D kernel)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on a single GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_1506_06140_amd as dg

    if args.workload in ("vortex", "vortex512"):
        n, k = (256, 2) if args.workload == "vortex" else (512, 3)
        print(json.dumps(vortex2d_line(steps=args.steps, warmup=args.warmup,
                                       with_cpu=not args.no_cpu and args.workload == "vortex",
                                       reps=args.kernel_reps, n=n, k=k, precision=args.precision)), flush=True)
        return

    wl = workloads.workload(args.workload)
    kname = "stage3d" if args.workload == "kh3d" else "stage3d_amr"
    s = dg.Solver(wl)
    steps = args.steps + (args.steps % 2)
    ms_step, w = time_steps(s, wl, steps, args.warmup, graph=bool(args.graph))
    cells = (s.ncoarse - s.nhole + s.nfine) if s.amr else s.ncell
    dof = cells * s.N
    value = dof * 3 / (ms_step * 1e-3)

    # the dominant kernel (fused RHS + stage) and the limiter pass, timed alone
    bufs = [s.empty(), s.empty(), s.empty(), s.scalar()]
    k_ms = kernel_ms(s, w, bufs, args.kernel_reps)
    lim_ms = kernel_ms(s, w, bufs, args.kernel_reps, limiter=True)
    if s.status() != 0:
        raise RuntimeError("device error flag set in the kernel timing")
    b, f = alg_work(3, wl["k"])
    alg_flops = f * cells
    alg_bytes = b * cells
    achieved = alg_flops / (k_ms * 1e-3) / 1e12
    # limiter: reads every coefficient once; it writes back only the
    # variables it changed (data-dependent, few cells of a smooth flow), which
    # the figure leaves out: its HBM fraction is a lower bound
    lim_bytes = s.N * s.nvar * 8 * cells

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("3D Kelvin-Helmholtz shear layer, 128^3 cells, k=2 (N=10), FP64, SSP-RK3, CFL 0.2, "
                                "component-wise TVB minmod + positivity limiter after every stage, seeded 1e-2 "
                                "velocity noise") if args.workload == "kh3d" else
                               ("3D Sod-type blast, 64^3 base grid + refined central 32^3 base cells (64^3 fine "
                                "cells), k=3 (N=20), FP64, SSP-RK3, CFL 0.2, minmod + positivity limiter"),
                   "cells": cells, "dof": dof, "stages_per_step": 3, "graph": bool(args.graph)},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": measured_traffic(kname),
                     "kernel": KERNELS[kname]["name"], "kernel_ms": k_ms,
                     "alg_flops_per_launch": alg_flops, "alg_bytes_per_launch": alg_bytes,
                     "hbm_achieved_gbs": alg_bytes / (k_ms * 1e-3) / 1e9,
                     "hbm_frac": alg_bytes / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "limiter": {"kernel": ("k_limit<3,2,false>" if args.workload == "kh3d" else "k_limit_amr<3,3,false> (both blocks)")
                              + " + k_positivity",
                    "kernel_ms": lim_ms, "alg_bytes_per_launch": lim_bytes,
                    "hbm_frac": lim_bytes / (lim_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        # the whole step's algorithmic work over the step time
        "step_fracs": {"alu": 3 * alg_flops / (ms_step * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                       "hbm": 3 * alg_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    del s, w, bufs
    torch.cuda.empty_cache()
    # the same stage kernel on the vector ALU (one thread per cell), for comparison
    s = dg.Solver(dict(wl, path3d=dg.DG_PATH3D_VALU))
    w = build_state(s, wl)
    s.limit(w)
    bufs = [s.empty(), s.empty(), s.empty(), s.scalar()]
    kv = kernel_ms(s, w, bufs, args.kernel_reps)
    rec["roofline"]["valu_kernel"] = {"kernel": "k_rhs_stage<3,2,double>" if args.workload == "kh3d" else
                                      "k_rhs_amr_quad<3>", "kernel_ms": kv,
                                      "frac": alg_flops / (kv * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                                      "traffic": measured_traffic("stage3d_valu") if args.workload == "kh3d" else None}
    del s, w, bufs
    torch.cuda.empty_cache()
    if args.variants:
        rec["variants"] = {"vortex2d_fp64": vortex2d_line(with_cpu=not args.no_cpu)}
        rec["variants"].update(variants())
    if not args.no_cpu and args.workload == "kh3d":
        rec["cpu_baseline"] = cpu_baseline(wl)
        rec["cpu_baseline"]["other_workloads"] = cpu_other_workloads()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
