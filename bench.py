#!/usr/bin/env python3
"""Benchmark of the DG right-hand side + SSP-RK3 hot path on one MI355X.

Workload: 2D isentropic vortex (strength 5, gamma 1.4, boost (1,1), periodic
[-5,5]^2), 256^2 cells, degree k = 2 (N = 6 modes, 4 variables), FP64,
seeded +-1e-3 density noise, CFL 0.2, no limiter.  One *step* is the whole
hot path for one SSP-RK3 step: the CFL time step reduction and the three
fused RHS + stage kernels.  The metric is DOF-updates per second per RK
stage: cells * N * 3 / step time.

The initial state is built by the library itself (seeded primitives from
``workloads`` sampled at the library's Gauss nodes, L2-projected by
``dg_project``); it is resident in HBM before the timed region starts.

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
METRIC = "DOF-updates/s per RK stage"
KERNEL_SRC = os.path.join(ROOT, "paper_1506_06140_amd", "csrc", "dg_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_rhs_tile2d_vortex256_k2_traffic.txt")


_FINGERPRINT_REGIONS = [
    # reciprocal helpers, the time-step rate, the Euler flux
    ("// Reciprocal and reciprocal square root from the hardware estimates plus",
     "// HLLC numerical flux in +a between traces UL (low side) and UR (high side),"),
    ("// HLLC numerical flux in +a between traces UL (low side) and UR (high side),",
     "// ---------------------------------------------------------------------------\n// Right-hand side and fused stage."),
    ("// 2D right-hand side + SSP-RK3 stage on LDS tiles, four lanes per cell.",
     "// Discrete adjoint of the right-hand side and of the SSP-RK3 stages."),
]


FP32_PEAK_TFLOPS = 157.3


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


def kernel_hash() -> str:
    """Fingerprint of the source of the benchmarked stage kernel (the tiled 2D
    kernel, the Riemann solver and its reciprocal helpers)."""
    src = open(KERNEL_SRC).read()
    parts = []
    for a, b in _FINGERPRINT_REGIONS:
        i = src.find(a)
        j = src.find(b, i + 1) if i >= 0 else -1
        if i < 0 or j < 0:
            raise RuntimeError(f"kernel fingerprint marker not found in {KERNEL_SRC}: {a if i < 0 else b!r}")
        parts.append(src[i:j])
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the stage kernel from the committed rocprofv3
    counter summary, or None if absent or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel_source_sha256_16:\s*(\w+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_hash():
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


def cpu_baseline(wl, budget_s: float = 12.0):
    """The FP64 oracle, single-threaded, on a bounded number of RK stages of
    the same workload."""
    import oracle
    o = oracle.Oracle(wl)
    w0 = o.initial_state()
    dt = o.max_dt(w0)
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
    dof = o.ncell * o.N
    return {"value": dof * stages / el, "unit": METRIC, "cores": 1, "kind": "oracle",
            "sample": f"{stages} SSP-RK3 stages (RHS + update, no limiter) of the full 256^2 k=2 vortex "
                      f"state, single-threaded C oracle, {el:.1f} s"}


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
    runs = [("vortex", "vortex", 400, {}, ("fp64", "fp32", "bf16")),
            ("vortex_dg4_rk4", "vortex", 200, {"k": 3, "rk": "rk4"}, ("fp64", "fp32")),
            ("vortex_dg5_rk4", "vortex", 200, {"k": 4, "rk": "rk4"}, ("fp64", "fp32")),
            ("kh3d", "kh3d", 10, {}, ("fp64", "fp32", "bf16")),
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
            _, rng = s.amr_flags(w, wl["wt"], wl["alpha"])
            nb = s.box_for(rng)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--graph", type=int, default=1, help="replay the step as a HIP graph")
    ap.add_argument("--variants", type=int, default=1, help="also time FP32, the 3D workload and the adjoint")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on a single GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_1506_06140_amd as dg

    wl = workloads.workload("vortex")
    s = dg.Solver(wl)
    A = build_state(s, wl)
    B = s.empty()
    u1, u2, dtbuf, rate = s.empty(), s.empty(), s.scalar(), s.rate_state()
    stream = torch.cuda.current_stream()
    s.max_rate(A, rate)

    def two_steps():
        # ping-pong: A -> B -> A, stage buffers u1, u2, device time step
        # dtbuf; each step is one dg_rk_step call (time step, 3 stages)
        s.rk_step(A, [u1, u2, B], dtbuf, rate)
        s.rk_step(B, [u1, u2, A], dtbuf, rate)

    steps = args.steps + (args.steps % 2)
    for _ in range((args.warmup + 1) // 2):
        two_steps()
    torch.cuda.synchronize()
    if s.status() != 0:
        raise RuntimeError("device error flag set during warm-up")

    graph = None
    if args.graph:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            two_steps()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            two_steps()
        torch.cuda.synchronize()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if graph is not None:
        for _ in range(steps // 2):
            graph.replay()
    else:
        for _ in range(steps // 2):
            two_steps()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = s.status()
    if st != 0:
        raise RuntimeError(f"device error flag {st} after the timed steps")
    w = A
    bufs = [u1, u2, B, dtbuf]
    args.steps = steps

    dof = s.ncell * s.N
    ms_step = el / args.steps * 1e3
    value = dof * 3 * args.steps / el

    # average duration of the dominant kernel (fused RHS + stage): one pair of
    # HIP events on the stream the kernels run on around a batch of launches
    # queued back to back (stages 1, 2, 3 in turn)
    reps = 300
    dt = s.max_dt(w, bufs[3])
    for stage in (1, 2, 3):
        s.rk_stage(stage, dt, w, w if stage == 1 else bufs[0], bufs[1] if stage == 1 else bufs[2])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(reps):
        stage = i % 3 + 1
        s.rk_stage(stage, dt, w, w if stage == 1 else bufs[0], bufs[1] if stage == 1 else bufs[2])
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / reps
    state_bytes = s.nvar * s.N * s.ncell * 8
    alg_bytes = 8.0 / 3.0 * state_bytes  # read w_prev (+ w_n in stages 2,3), write w_out
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    alg_flops = alg_work(2, 2)[1] * s.ncell

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "isentropic vortex 2D, 256x256 cells, k=2 (N=6), FP64, SSP-RK3, CFL 0.2, "
                               "no limiter, seeded 1e-3 density noise",
                   "cells": s.ncell, "dof": dof, "stages_per_step": 3, "graph": bool(graph)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_rhs_tile2d<2,double> (8x8 tiles)", "kernel_ms": k_ms,
                     "alg_bytes_per_launch": alg_bytes},
        # the same launch against the FP64 vector peak (algorithmic flops)
        "roofline_fp64": {"bound": "alu", "achieved": alg_flops / (k_ms * 1e-3) / 1e12,
                          "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": alg_flops / (k_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                          "alg_flops_per_launch": alg_flops},
    }
    if args.variants:
        rec["variants"] = variants()
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
