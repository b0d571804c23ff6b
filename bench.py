#!/usr/bin/env python3
"""Throughput of the reacting-flow RK3 step on one MI355X.

A step is one SSP-RK3 step of the full hot path on the 128^3 periodic
multicomponent Taylor-Green box (9 species, 20 reversible reactions,
mixture-averaged transport, Mach 0.3): per stage the per-cell kernel
(primitives, Newton T, transport, chemistry, source, heat release; the first
stage also reduces the stable dt), the dilatation sensor, and the fused flux
sweep with the stage update; the time-integrated heat release accumulates on
the device.  Inputs are seeded synthetic fields resident in HBM.

Prints one JSON line.  `value` = cells x 3 stages x steps / time.  The same
line carries, under their own keys, the 256x128x128 mixing layer with laser
deposition over its 100 steps, the 64-member ensemble over 50 steps (one
captured graph against per-member launches), the 64^3 adjoint workload over
50 steps (backward/forward time), the 128^3 curvilinear grid, and the
oracle timed on the host cores (a baseline, not the target).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector, TFLOP/s
def point_flops_per_cell(ns, nr, laser_on, newton_iters=3):
    """Algorithmic FP64 operations of the per-cell kernel (one stage), from
    the operation counts of its formulas (+, -, *, /, sqrt = 1, FMA = 2);
    exponentials, logarithms and powers are not counted here but in
    point_transcendentals_per_cell."""
    newton = newton_iters * (ns * 25 + 2)
    thermo = ns * 13 + ns * 2 + 8
    transport = ns * 20 + ns * ns * 6 + ns * 5 + (ns * (ns - 1) // 2) * 17 + ns * 2
    chem = ns * 21 + nr * (5 + 2 * ns + 2 + 4 + 1 + 2 * ns) + ns * 14
    laser = 30 if laser_on else 0
    misc = 40
    return newton + thermo + transport + chem + laser + misc


def point_transcendentals_per_cell(ns, nr, laser_on):
    """exp/log/pow evaluations of the per-cell kernel per cell and stage:
    three per species for mu_s (Omega(2,2) fit), four per pair for D_ij
    (Omega(1,1) fit), two for the mixture, two per reaction (k_f, K_c)
    plus ln T, and nine for the laser's Gaussians."""
    return 3 * ns + 4 * (ns * (ns - 1) // 2) + 2 + 2 * nr + 1 + (9 if laser_on else 0)


def sweep_bytes_per_cell(ns):
    """Algorithmic HBM bytes of the flux sweep (sensor, convective and
    diffusive flux differences, stage update) per cell and stage, by the
    item list of the measurement plan: read U (nv), the per-cell fields the
    fluxes need (p, c, mu, lambda, T, D_s: 5 + ns), the sources (wdot_s,
    q_L: ns + 1) and, in stages 2-3 (2/3 on average), U^n (nv); write
    U^(k+1) (nv).  469 B at ns = 9 (the plan's estimate: about 460 B)."""
    nv = ns + 4
    return 8 * (nv + (5 + ns) + (ns + 1) + nv * 2.0 / 3.0 + nv)


def point_bytes_per_cell(ns):
    """Algorithmic HBM bytes of the per-cell kernel per cell and stage: read
    U and T; write T, c, mu, lambda, D_s and the sources (the plan's item
    list: 296 B at ns = 9, about 300 B)."""
    nv = ns + 4
    return 8 * (nv + 1) + 8 * (1 + 3 + ns + (ns + 1))


CSRC = os.path.join(ROOT, "paper_2202_02319_amd", "csrc")
KERNEL_SOURCES = {
    "k_point": ("htr_point.hip", "htr_dev.h", "htr_flux.h"),
    "k_sensor": ("htr_point.hip", "htr_dev.h", "htr_flux.h"),
    "k_conv": ("htr_sweep.hip", "htr_dev.h", "htr_flux.h"),
    "k_diff": ("htr_sweep.hip", "htr_dev.h", "htr_flux.h"),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_tgv128.md")


def curv_conv_bytes_per_cell(ns):
    """Curvilinear convective face kernel, per cell and direction, each array
    read once (perfect stencil reuse): U (ns+4), p, c, u, v, w (5), the face
    metric vector (3), the sensor flag (1 byte); write the face flux (ns+4)."""
    return 8 * (2 * (ns + 4) + 5 + 3) + 1


def curv_diff_bytes_per_cell(ns):
    """Curvilinear diffusive face kernel, per cell and direction: U (ns),
    T, mu, lambda, u, v, w, D_s (6+ns), mole fractions (ns), the two
    tangential index-space differences of (u, v, w, T, X_s) (2 (4+ns)),
    node metric terms and J (10), face metric vector (3); write the face
    flux (ns+4)."""
    return 8 * (ns + 1 + (5 + ns) + ns + 2 * (4 + ns) + 10 + 3 + (ns + 4))


def curv_update_bytes_per_cell(ns):
    """Curvilinear update: the three directions' convective and diffusive
    face fluxes (6 (ns+4)), U, U^n (stages 2 and 3: 2/3 on average),
    sources (ns+1) and J in; U^(k+1) out."""
    nv = ns + 4
    return 8 * (6 * nv + nv + (2.0 / 3.0) * nv + (ns + 1) + 1 + nv)


def kernel_source_hash(kernel):
    """Short SHA-256 of the source files a kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, each scaled by the
    same counter's reading on a plain copy of known size) from the committed
    counter summary; None if there is none for this kernel and workload or
    if the kernel's sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if not line.startswith("traffic:"):
                continue
            kv = dict(tok.split("=", 1) for tok in line.split()[1:])
            if kv.get("kernel") == kernel and kv.get("workload") == workload:
                if kv.get("sha") != kernel_source_hash(kernel):
                    return None
                return float(kv["fetch_bytes"]) + float(kv["write_bytes"])
    return None


def calibration_copy(nbytes=1 << 30):
    """A plain device copy of known size (read nbytes, write nbytes) that a
    counter run uses to scale FETCH_SIZE and WRITE_SIZE to bytes."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    return nbytes


def cpu_baseline(case, seconds_target=15.0):
    """The oracle (test infrastructure) timed on the host cores on a bounded
    sample of the same workload: repeated right-hand-side evaluations (one
    stage each) of the whole grid, or of a leading slab if one evaluation of
    the whole grid would take more than the target, for about
    seconds_target seconds of work."""
    from oracle import Oracle
    import synth
    nz = case.grid.n[2]
    # probe on a 4-layer slab, then size the sample
    kz = min(4, nz)
    probe = None
    while True:
        n = (case.grid.n[0], case.grid.n[1], kz)
        g = synth.Grid(n=n, xnode=[case.grid.xnode[0], case.grid.xnode[1], case.grid.xnode[2][:kz]],
                       xin=[case.grid.xin[0], case.grid.xin[1], case.grid.xin[2][:kz]],
                       xif=[case.grid.xif[0], case.grid.xif[1], case.grid.xif[2][:kz]], L=case.grid.L)
        N = g.N
        sub = synth.Case(case.name, case.mech, g, case.Y[:, :N], case.T[:N], case.p[:N], case.vel[:, :N],
                         laser=case.laser, flags=case.flags)
        o = Oracle(sub)
        U = o.prim_to_cons()
        T = sub.T.copy()
        if probe is None:
            t0 = time.perf_counter()
            o.rhs(U, T, t=0.0)
            probe = (time.perf_counter() - t0) / kz        # seconds per z layer
            kz = nz if probe * nz <= seconds_target else max(1, int(seconds_target / probe))
            continue
        break
    reps = max(1, int(round(seconds_target / (probe * kz))))
    t0 = time.perf_counter()
    for _ in range(reps):
        o.rhs(U, T, t=0.0)
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": reps * sub.grid.N / el, "unit": "cell-stage updates/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{reps} RHS evaluations (one stage each) of a {sub.grid.n[0]}x{sub.grid.n[1]}x{sub.grid.n[2]} "
                      f"{'grid' if kz == nz else 'slab of the grid'}, {el:.1f} s"}


def cpu_baseline_curvilinear(n=64, seconds_target=10.0, amp=0.25):
    """The oracle (test infrastructure) on the curvilinear workload's recipe
    at n^3 (the Taylor-Green state on a wavy grid): repeated right-hand-side
    evaluations of the whole grid for about seconds_target seconds (the
    metric set-up is not timed)."""
    from oracle import Oracle
    import synth
    c2 = synth.case_c2(n=n)
    grid = synth.wavy_grid(c2.grid.n, c2.grid.spacing(), amp=amp, seed=11)
    case = synth.Case("tgv-curv", c2.mech, grid, c2.Y, c2.T, c2.p, c2.vel, flags=c2.flags)
    o = Oracle(case)
    U = o.prim_to_cons()
    T = case.T.copy()
    t0 = time.perf_counter()
    o.rhs(U, T, t=0.0)
    one = time.perf_counter() - t0
    reps = max(1, int(round(seconds_target / one)))
    t0 = time.perf_counter()
    for _ in range(reps):
        o.rhs(U, T, t=0.0)
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": reps * grid.N / el, "unit": "cell-stage updates/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{reps} RHS evaluations (one stage each) of the {n}^3 wavy-grid Taylor-Green state, {el:.1f} s"}


def ensemble_measure(steps, warm=1, sizes=None):
    """The 64-member ensemble (N^3 members, N uniform on {32, 40, ..., 96}
    unless `sizes` gives the N of each member; perturbed deposition energy,
    kernel centre and ln A): `steps` RK3 steps of all members as one captured
    HIP-graph launch (one launch per kernel over all members' tiles), against
    the same steps driven member by member (one htr_rk3_step per member and
    step, one stream)."""
    import torch
    import synth
    from paper_2202_02319_amd import htr
    e = synth.ensemble_c4(sizes=sizes)
    Ns = sorted({int(round(c.grid.N ** (1 / 3))) for c in e.members})
    ctx = htr.Context(e.mech, e.members[0].grid)
    b = htr.Batch.from_cases(ctx, e.members, e.dlnA)
    U, T = htr.batch_state_from_cases(b, e.members)
    z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")  # noqa: E731
    t, dt, J = z(b.nmem), z(b.nmem), z(b.nmem)
    work = b.new_work()
    shapes, grid = htr.htr_batch_autotune(b, U, T.clone(), work)
    stream = torch.cuda.current_stream()
    htr.htr_rk3_steps_batched(b, U, T, t, dt, 1, steps, work, J, use_graph=True)   # capture + warm-up
    torch.cuda.synchronize()
    htr.htr_batch_check(b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    htr.htr_rk3_steps_batched(b, U, T, t, dt, 1, steps, work, J, use_graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    htr.htr_batch_check(b)
    t_b = e0.elapsed_time(e1) / 1e3
    del U, T, work
    # member by member
    mems = []
    for m, c in enumerate(e.members):
        g = htr.Context(e.mech, c.grid)
        htr.htr_set_tiling(g, shapes[m], 0)     # the shape tuned for its size class
        mems.append((g, htr.cons_from_case(g, c), htr.to_dev(c.T), z(1), z(1), z(1), g.new_work(),
                     htr.to_dev(e.dlnA[m]), c.laser))

    def per_member(nst):
        for _ in range(nst):
            for (g, Um, Tm, tm, dtm, Jm, wm, dl, las) in mems:
                htr.htr_rk3_step(g, Um, Tm, tm, dtm, 1, las, dl, wm, Jm)
    per_member(warm)
    torch.cuda.synchronize()
    e0.record(stream)
    per_member(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    for g, *_ in mems:
        htr.htr_check(g)
    t_m = e0.elapsed_time(e1) / 1e3
    cs = b.N * 3 * steps
    return {"workload": f"{len(e.members)}-member mixing-layer ensemble, N^3 members with N in "
                        f"{{{','.join(map(str, Ns))}}}, {b.N} cells, {steps} RK3 steps", "cells": b.N, "steps": steps,
            "batched_value": cs / t_b, "per_member_value": cs / t_m, "unit": "cell-stage updates/s",
            "batched_over_per_member": t_m / t_b, "batched_ms_per_step": 1e3 * t_b / steps,
            "per_member_ms_per_step": 1e3 * t_m / steps,
            "tiles": {f"{n}^3": "x".join(map(str, shapes[[int(round(c.grid.N ** (1 / 3))) for c in e.members].index(n)]))
                      for n in Ns}, "persistent_grid": grid, "conv_split": htr.htr_batch_get_conv_split(b)}


def curvilinear_measure(steps, warm=2, n=128, amp=0.25):
    """The 128^3 Taylor-Green state (9 species, 20 reactions) on a 128^3 wavy
    curvilinear grid (every metric term varying along every axis): `steps`
    SSP-RK3 steps with the in-step CFL dt through the curvilinear kernels,
    per-kernel HIP-event durations, and the face and update kernels priced
    against HBM with their algorithmic bytes."""
    import torch
    import synth
    from paper_2202_02319_amd import htr
    c2 = synth.case_c2(n=n)
    grid = synth.wavy_grid(c2.grid.n, c2.grid.spacing(), amp=amp, seed=11)
    case = synth.Case("tgv-curv", c2.mech, grid, c2.Y, c2.T, c2.p, c2.vel, flags=c2.flags)
    ctx = htr.Context.from_case(case)
    N = ctx.N
    U = htr.cons_from_case(ctx, case)
    T = htr.to_dev(case.T)
    z = lambda: torch.zeros(1, dtype=torch.float64, device="cuda")  # noqa: E731
    t, dt = z(), z()
    work = ctx.new_work()

    def step():
        htr.htr_rk3_step(ctx, U, T, t, dt, 1, None, None, work, None)
    for _ in range(warm):
        step()
    torch.cuda.synchronize()
    htr.htr_check(ctx)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    htr.htr_check(ctx)
    ms = e0.elapsed_time(e1) / steps
    htr.htr_timing(ctx, 1)
    for _ in range(steps):
        step()
    kt = htr.htr_timing_read(ctx)
    htr.htr_timing(ctx, 0)
    htr.htr_check(ctx)
    avg = {k: v[0] / max(v[1], 1) for k, v in kt.items()}
    ns = case.mech.ns
    kern = {}
    for k, name, bpc in (("conv", "k_curv_conv", 3 * curv_conv_bytes_per_cell(ns)),
                         ("diff", "k_curv_diff", 3 * curv_diff_bytes_per_cell(ns)),
                         ("update", "k_curv_update", curv_update_bytes_per_cell(ns))):
        ach = bpc * N / (avg[k] / 1e3) / 1e9
        kern[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_cell": round(bpc, 1),
                      "avg_ms": round(avg[k], 4)}
    return {"workload": f"{n}^3 multicomponent Taylor-Green state on a {n}^3 wavy curvilinear grid, 9 species, "
                        f"20 reactions, SSP-RK3 with in-step CFL dt", "cells": N, "steps": steps,
            "value": N * 3 / (ms / 1e3), "unit": "cell-stage updates/s", "ms_per_step": ms,
            "kernel_ms": {"point": round(avg["point"], 4), "molefrac+igrad+sensor": round(avg["sensor"], 4),
                          "conv_faces": round(avg["conv"], 4), "diff_faces": round(avg["diff"], 4),
                          "update": round(avg["update"], 4), "reduce": round(avg["reduce"], 4)},
            "kernels": kern}


def multifidelity_measure(hf_steps, nlf=64, n_lf=16):
    """Multi-fidelity co-processing: the 64^3 mixing layer (HF) for hf_steps
    SSP-RK3 steps and an LF ensemble of nlf members of n_lf^3 (the same
    recipe, coarse grids, perturbed deposition) for 3 hf_steps steps, alone
    and at once on two HIP streams."""
    import synth
    from paper_2202_02319_amd.multifidelity import Fidelities, co_process
    hf_case = synth.case_c5()
    e = synth.ensemble_c4(nmem=nlf, sizes=[n_lf] * nlf)
    fid = Fidelities(hf_case, e.members, e.dlnA)
    run = co_process(fid, hf_steps, 3 * hf_steps)
    return {"workload": f"HF: 64^3 mixing layer, {hf_steps} RK3 steps; LF: {nlf} members of {n_lf}^3, "
                        f"{3 * hf_steps} RK3 steps (captured graph); two HIP streams",
            "hf_ms": round(run.hf_ms, 3), "lf_ms": round(run.lf_ms, 3), "both_ms": round(run.both_ms, 3),
            "overlap": round(run.overlap(), 3)}


def adjoint_measure(nsteps=50, every=10, n=64):
    """The adjoint workload: the 64^3 mixing layer, `nsteps` RK3 steps with a
    frozen dt, checkpoints every `every` steps; gradient of the time-
    integrated heat release with respect to (E, centre, ln A_1..20).
    Returns forward time (with checkpointing) and backward time (segment
    re-runs + reverse sweep) and their ratio."""
    import torch
    import synth
    from paper_2202_02319_amd import htr
    from paper_2202_02319_amd.adjoint import HeatReleaseProblem
    case = synth.case_c5(n=n, steps=nsteps)
    ctx = htr.Context.from_case(case)
    U0 = htr.cons_from_case(ctx, case)
    T0 = htr.to_dev(case.T)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    htr.htr_autotune(ctx, U0, T0.clone(), ctx.new_work())
    htr.htr_stable_dt(ctx, U0, T0.clone(), dt)
    prob = HeatReleaseProblem(ctx, U0, T0, case.laser, float(dt.item()), nsteps, checkpoint_every=every)
    theta = torch.tensor([case.laser.E, *case.laser.center] + [0.0] * case.mech.nr, dtype=torch.float64,
                         device="cuda")
    J, ck = prob.forward(theta, keep_last=True)            # warm-up
    prob.backward(theta, ck)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, ck = prob.forward(theta, keep_last=True)   # as the autograd function runs it
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g, _ = prob.backward(theta, ck)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gh = g.cpu().numpy()
    return {"workload": f"{n}^3 mixing layer, {nsteps} RK3 steps, frozen dt, checkpoints every {every}; "
                        "dJ/d(E, centre, ln A_1..20)",
            "forward_ms": 1e3 * (t1 - t0), "backward_ms": 1e3 * (t2 - t1),
            "adjoint_over_forward": (t2 - t1) / (t1 - t0), "J": float(J.item()),
            "dJ_dE": float(gh[0]), "dJ_dcentre": [float(v) for v in gh[1:4]]}


def single_measure(case, steps, warmup, autotune=True, conv_split=None, tile=None):
    """`steps` timed SSP-RK3 steps (in-step CFL dt, J accumulated) of one
    grid after `warmup` untimed ones, HIP events on the launch stream; then
    the same number of steps again with per-kernel event timing.  Returns
    the throughput, the per-kernel launch averages and the roofline of the
    per-cell kernel and of the flux sweep."""
    import torch
    from paper_2202_02319_amd import htr
    ctx = htr.Context.from_case(case)
    N = ctx.N
    U = htr.cons_from_case(ctx, case)
    T = htr.to_dev(case.T)
    z = lambda: torch.zeros(1, dtype=torch.float64, device="cuda")  # noqa: E731
    t_dev, dt_dev, J_dev = z(), z(), z()
    work = ctx.new_work()
    laser = case.laser if case.laser.on else None
    if conv_split is not None:
        htr.htr_set_conv_split(ctx, conv_split)
    if tile is not None:
        htr.htr_set_tiling(ctx, tile, 0)
    tile, grid = htr.htr_autotune(ctx, U, T.clone(), work) if autotune else htr.htr_get_tiling(ctx)

    U0, T0 = U.clone(), T.clone()

    def step():
        htr.htr_rk3_step(ctx, U, T, t_dev, dt_dev, 1, laser, None, work, J_dev)

    def restart():
        # every pass starts from the initial state, so no pass runs the
        # workload past its configured number of steps
        U.copy_(U0)
        T.copy_(T0)
        t_dev.zero_()
        J_dev.zero_()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    htr.htr_check(ctx)
    restart()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    htr.htr_check(ctx)
    ms = e0.elapsed_time(e1) / steps
    J_timed = float(J_dev.item())
    # per-kernel durations, HIP events on the launch stream, the same steps again
    restart()
    htr.htr_timing(ctx, 1)
    for _ in range(steps):
        step()
    kt = htr.htr_timing_read(ctx)
    htr.htr_timing(ctx, 0)
    htr.htr_check(ctx)
    ns, nr = case.mech.ns, case.mech.nr
    avg = {k: v[0] / max(v[1], 1) for k, v in kt.items()}
    # the per-cell kernel against the FP64 vector peak (formula FLOPs, the
    # exponentials counted apart), the flux sweep (sensor + convective +
    # diffusive kernels, one stage) against HBM with its algorithmic bytes
    fl = point_flops_per_cell(ns, nr, laser is not None)
    ach = fl * N / (avg["point"] / 1e3) / 1e12
    point = {"kernel": "k_point", "bound": "alu", "achieved": round(ach, 2), "peak": FP64_PEAK_TFLOPS,
             "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4), "flops_per_cell": fl,
             "transcendentals_per_cell": point_transcendentals_per_cell(ns, nr, laser is not None),
             "bytes_per_cell": point_bytes_per_cell(ns), "avg_ms": round(avg["point"], 4)}
    sweep_ms = avg["sensor"] + avg["conv"] + avg["diff"]
    bpc = sweep_bytes_per_cell(ns)
    ach = bpc * N / (sweep_ms / 1e3) / 1e9
    sweep = {"kernel": "sweep (k_sensor + k_conv + k_diff)", "bound": "hbm", "achieved": round(ach, 1),
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
             "bytes_per_cell": round(bpc, 1), "avg_ms": round(sweep_ms, 4),
             "parts_ms": {"k_sensor": round(avg["sensor"], 4), "k_conv": round(avg["conv"], 4),
                          "k_diff": round(avg["diff"], 4)}}
    return {"ctx": ctx, "N": N, "ms": ms, "wall": wall, "value": N * 3 / (ms / 1e3), "tile": tile, "grid": grid,
            "conv_split": htr.htr_get_conv_split(ctx),
            "avg": avg, "kt": kt, "point": point, "sweep": sweep, "J": J_timed}


def roofline_of(meas, workload, steps):
    """The dominant one of the per-cell kernel and the flux sweep (longer
    per-stage time), with HBM traffic from the committed counter summary."""
    dom = "sweep" if meas["sweep"]["avg_ms"] >= meas["point"]["avg_ms"] else "point"
    roof = {k: v for k, v in meas[dom].items() if k in ("kernel", "bound", "achieved", "peak", "unit", "frac")}
    kernels = ("k_sensor", "k_conv", "k_diff") if dom == "sweep" else ("k_point",)
    tb = [measured_traffic(k, workload) for k in kernels]
    tb = None if any(b is None for b in tb) else float(sum(tb))
    roof["traffic"] = round(tb / (meas[dom]["avg_ms"] / 1e3) / 1e9, 1) if tb is not None else None
    roof["traffic_bytes_per_stage"] = tb
    roof["avg_ms_per_stage"] = meas[dom]["avg_ms"]
    roof["point"] = meas["point"]
    roof["sweep"] = meas["sweep"]
    roof["kernel_ms"] = {k: round(v, 4) for k, v in meas["avg"].items()}
    roof["step_ms_by_kernel"] = {k: round(v[0] / steps, 4) for k, v in meas["kt"].items()}
    return roof


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["tgv128", "mixing256"], default="tgv128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--mix-steps", type=int, default=100,
                    help="RK3 steps of the 256x128x128 mixing-layer measurement (0: skip)")
    ap.add_argument("--ens-steps", type=int, default=50, help="RK3 steps of the ensemble measurement (0: skip)")
    ap.add_argument("--adj-steps", type=int, default=50, help="RK3 steps of the adjoint measurement (0: skip)")
    ap.add_argument("--mf-steps", type=int, default=10,
                    help="HF steps of the multi-fidelity co-processing measurement (0: skip)")
    ap.add_argument("--curv-steps", type=int, default=5,
                    help="RK3 steps of the curvilinear-grid measurement (0: skip)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tiles (no autotuning)")
    ap.add_argument("--conv-split", type=int, choices=(0, 1), default=None,
                    help="with --no-autotune: 1 runs central tiles in the lean convective sweep (the default), "
                         "0 every tile in the full sweep")
    ap.add_argument("--tile", type=str, default=None,
                    help="with --no-autotune: the convective tile shape, e.g. 8x8x4 (default 16x4x4)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with a plain 1 GiB device copy (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (ensemble members or grid blocks "
              "would shard across GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth

    case = synth.case_c2() if args.workload == "tgv128" else synth.case_c3()
    tile = tuple(int(x) for x in args.tile.split("x")) if args.tile else None
    meas = single_measure(case, args.steps, args.warmup, autotune=not args.no_autotune, conv_split=args.conv_split,
                          tile=tile)
    ns, nr = case.mech.ns, case.mech.nr
    out = {
        "metric": "FP64 cell-stage updates/s (plain vs batched ensemble); adjoint/forward time",
        "value": meas["value"],
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": meas["ms"],
        "wall_s": meas["wall"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3-D periodic multicomponent Taylor-Green box 128^3, 9 species, 20 reactions, "
                               "Mach 0.3, SSP-RK3 with in-step CFL dt"
                   if args.workload == "tgv128" else
                   "3-D periodic double mixing layer 256x128x128, 9 species, 20 reactions, laser",
                   "cells": meas["N"], "species": ns, "reactions": nr, "stages_per_step": 3,
                   "tile": "x".join(map(str, meas["tile"])), "persistent_grid": meas["grid"],
                   "conv_split": meas["conv_split"]},
        "roofline": roofline_of(meas, args.workload, args.steps),
    }
    del meas
    torch.cuda.empty_cache()
    if args.mix_steps > 0 and args.workload == "tgv128":
        c3 = synth.case_c3()
        m3 = single_measure(c3, args.mix_steps, 2, autotune=not args.no_autotune, conv_split=args.conv_split)
        out["mixing256"] = {
            "workload": "3-D periodic double mixing layer 256x128x128, 9 species, 20 reactions, laser deposition, "
                        f"{args.mix_steps} SSP-RK3 steps with in-step CFL dt",
            "cells": m3["N"], "steps": args.mix_steps, "value": m3["value"], "unit": "cell-stage updates/s",
            "ms_per_step": m3["ms"], "tile": "x".join(map(str, m3["tile"])), "conv_split": m3["conv_split"],
            "J": m3["J"],
            "roofline": roofline_of(m3, "mixing256", args.mix_steps)}
        del m3
        torch.cuda.empty_cache()
    if args.ens_steps > 0:
        out["ensemble"] = ensemble_measure(args.ens_steps)
        torch.cuda.empty_cache()
        # small members (N = 12..24): each member alone fills a few CUs, so
        # per-member launches are latency-bound and batching pays most
        small = np.random.default_rng(12).choice(np.arange(12, 25, 4), size=64)
        out["ensemble_small"] = ensemble_measure(args.ens_steps, sizes=small)
    if args.mf_steps > 0:
        torch.cuda.empty_cache()
        out["multifidelity"] = multifidelity_measure(args.mf_steps)
    if args.adj_steps > 0:
        torch.cuda.empty_cache()
        out["adjoint"] = adjoint_measure(args.adj_steps)
    if args.curv_steps > 0:
        torch.cuda.empty_cache()
        out["curvilinear"] = curvilinear_measure(args.curv_steps)
        if not args.no_cpu_baseline:
            out["curvilinear"]["cpu_baseline"] = cpu_baseline_curvilinear()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    if args.calib_copy:
        out["calibration_copy_bytes"] = calibration_copy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
