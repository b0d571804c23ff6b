"""Writes the oracle's state after each benchmark workload's configured
number of SSP-RK3 steps at a fixed set of sampled cells (plus the
normalisation scales and the time-integrated heat release), the expected
values of the after-steps parity tests.

TEST INFRASTRUCTURE: calls only the oracle (oracle/) and the seeded input
generators (synth/).  Run from the repository root, one workload per call:

    python tests/golden/make_step_fixtures.py tgv128      # 128^3 Taylor-Green box, 10 steps
    python tests/golden/make_step_fixtures.py mixing256   # 256x128x128 mixing layer, 100 steps
    python tests/golden/make_step_fixtures.py ensemble    # 3 members of the 64-member ensemble, 50 steps
    python tests/golden/make_step_fixtures.py adjoint64   # 64^3 mixing layer, 50 steps, frozen dt, + tangent

Each writes tests/golden/steps_<workload>.json.  The oracle takes each step
with its own stable dt (the in-step CFL rule), except the adjoint workload,
whose dt is frozen at the initial state's and which also records the
tangent dJ of one parameter direction over the same steps.
"""
from __future__ import annotations

import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import Oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
NSAMPLE = 256


def sample_cells(case, seed):
    """NSAMPLE seeded cells spread over the grid, plus a 4x4x4 block at the
    laser centre when the case has a laser."""
    N = case.grid.N
    rng = np.random.default_rng(seed)
    cells = set(int(q) for q in rng.choice(N, size=NSAMPLE, replace=False))
    if case.laser.on:
        n = case.grid.n
        c = [int(np.argmin(np.abs(case.grid.xnode[a] - case.laser.center[a]))) for a in range(3)]
        for k in range(-2, 2):
            for j in range(-2, 2):
                for i in range(-2, 2):
                    q = ((c[2] + k) % n[2] * n[1] + (c[1] + j) % n[1]) * n[0] + (c[0] + i) % n[0]
                    cells.add(int(q))
    return sorted(cells)


def run(o, case, nsteps, lnA=None, dt_frozen=None, log=""):
    U = o.prim_to_cons()
    T = case.T.copy()
    t, J, dts = 0.0, 0.0, []
    t0 = time.time()
    for n in range(nsteps):
        dt = dt_frozen if dt_frozen is not None else o.stable_dt(U, T)
        J = o.rk3_step(U, T, t, dt, lnA=lnA, J=J)
        t += dt
        dts.append(dt)
        print(f"{log} step {n + 1}/{nsteps} dt {dt:.6e} ({time.time() - t0:.0f} s)", flush=True)
    return U, T, t, J, dts


def record(o, case, U, T, t, J, dts, cells, **extra):
    c = o.cells(U, T.copy())[2]
    ns = o.ns
    return {
        "n": list(case.grid.n), "ns": ns, "steps": len(dts), "t": t, "J": J, "dts": dts,
        "max_abs": [float(v) for v in np.abs(U).max(axis=1)],
        "rho_c": float(U[:ns].sum(axis=0).max() * c.max()),
        "cells": cells,
        "U": [[float(U[v, q]) for q in cells] for v in range(U.shape[0])],
        "T": [float(T[q]) for q in cells],
        **extra,
    }


def write(name, about, body):
    path = os.path.join(HERE, f"steps_{name}.json")
    body = {"about": about, "command": f"python tests/golden/make_step_fixtures.py {name}", **body}
    with open(path, "w") as fh:
        json.dump(body, fh)
        fh.write("\n")
    print("wrote", path)


def tgv128():
    case = synth.case_c2()
    o = Oracle(case)
    U, T, t, J, dts = run(o, case, 10, log="tgv128")
    write("tgv128", "oracle state after 10 SSP-RK3 steps (in-step CFL 0.5 dt) of the 128^3 multicomponent "
          "Taylor-Green box (9 species, 20 reactions), at sampled cells",
          record(o, case, U, T, t, J, dts, sample_cells(case, 102)))


def mixing256():
    case = synth.case_c3()
    o = Oracle(case)
    U, T, t, J, dts = run(o, case, case.steps, log="mixing256")
    write("mixing256", "oracle state after 100 SSP-RK3 steps (in-step CFL 0.5 dt) of the 256x128x128 double "
          "mixing layer with laser deposition (9 species, 20 reactions), at sampled cells",
          record(o, case, U, T, t, J, dts, sample_cells(case, 103)))


def ensemble():
    e = synth.ensemble_c4()
    sizes = [c.grid.n[0] for c in e.members]
    order = np.argsort(sizes, kind="stable")
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    out = {}
    for m in picks:
        c = e.members[m]
        mech_m = dataclasses.replace(e.mech, lnA=e.mech.lnA + e.dlnA[m])
        cm = synth.Case(c.name, mech_m, c.grid, c.Y, c.T, c.p, c.vel, laser=c.laser)
        o = Oracle(cm)
        U, T, t, J, dts = run(o, cm, e.steps, log=f"member {m} ({sizes[m]}^3)")
        out[str(m)] = record(o, cm, U, T, t, J, dts, sample_cells(cm, 104 + m))
    write("ensemble", "oracle states after 50 SSP-RK3 steps (each member its own in-step CFL 0.5 dt, its own "
          "ln A offsets and laser) of the smallest, the median-size and the largest member of the 64-member "
          "mixing-layer ensemble, at sampled cells", {"members": out})


def adjoint64():
    case = synth.case_c5()
    o = Oracle(case)
    U0 = o.prim_to_cons()
    dt = o.stable_dt(U0, case.T.copy())
    U, T, t, J, dts = run(o, case, case.steps, dt_frozen=dt, log="adjoint64")
    body = record(o, case, U, T, t, J, dts, sample_cells(case, 105))
    # tangent of J along one direction of theta = (E, centre, ln A offsets)
    rng = np.random.default_rng(5)
    las = case.laser.as_array()
    dth = np.concatenate([[0.2 * las[0]], 0.1 * case.laser.sigma_r * rng.normal(size=3),
                          rng.normal(size=case.mech.nr)])
    U = U0.copy()
    dU = np.zeros_like(U)
    T = case.T.copy()
    Jt, dJ = 0.0, 0.0
    t0 = time.time()
    for n in range(case.steps):
        Jt, dJ = o.rk3_tangent(U, dU, T, n * dt, dt, las, dth[:4], case.mech.lnA, dth[4:], Jt, dJ)
        print(f"adjoint64 tangent step {n + 1}/{case.steps} ({time.time() - t0:.0f} s)", flush=True)
    body["tangent"] = {"dtheta": [float(v) for v in dth], "J": Jt, "dJ": dJ}
    write("adjoint64", "oracle state after 50 SSP-RK3 steps with the dt frozen at the initial state's stable dt "
          "of the 64^3 mixing layer (9 species, 20 reactions, laser), at sampled cells; and the oracle's "
          "forward-mode (dual-number) tangent dJ of the time-integrated heat release along dtheta over the "
          "same steps", body)


if __name__ == "__main__":
    {"tgv128": tgv128, "mixing256": mixing256, "ensemble": ensemble, "adjoint64": adjoint64}[sys.argv[1]]()
