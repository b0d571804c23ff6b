"""GPU against the oracle after each benchmark workload's configured number
of SSP-RK3 steps, at the workloads' full sizes and in the benchmark's launch
configuration (autotuned tiles; the ensemble as one captured graph):

- the 128^3 Taylor-Green box after 10 steps;
- the 256x128x128 mixing layer with laser deposition after 100 steps;
- the smallest, the median-size and the largest member of the 64-member
  ensemble after 50 steps of the whole ensemble;
- the 64^3 adjoint workload after 50 steps at its frozen dt, and the
  adjoint gradient along one parameter direction against the oracle's
  forward-mode tangent over the same 50 steps.

Expected values: tests/golden/steps_*.json, written by
tests/golden/make_step_fixtures.py from the oracle alone: every conserved
variable at 256 seeded cells (plus a block at the laser centre), the full
field's max|U_v|, the acoustic momentum scale rho*c, t and J.  The bar is
1e-9 normwise per conserved variable, the momentum rows measured against
max(max|rho u|, rho c) (the oracle's own spread under one-ulp input
perturbations is shown in test_oracle_spread.py).
"""
import json
import os

import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, host
from paper_2202_02319_amd import htr

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-9
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fixture(name):
    path = os.path.join(GOLDEN, f"steps_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet (tests/golden/make_step_fixtures.py {name})")
    with open(path) as fh:
        return json.load(fh)


def _check(U_host, fx):
    ns = fx["ns"]
    cells = np.array(fx["cells"])
    ref = np.array(fx["U"])
    den = np.array(fx["max_abs"])
    den[ns:ns + 3] = np.maximum(den[ns:ns + 3], fx["rho_c"])
    err = np.abs(U_host[:, cells] - ref).max(axis=1) / den
    assert err.max() <= STEP_TOL, err
    return err


def _single(case, nsteps, fx):
    ctx = htr.Context.from_case(case)
    U = htr.cons_from_case(ctx, case)
    T = dev(case.T)
    work = ctx.new_work()
    htr.htr_autotune(ctx, U, T.clone(), work)
    z = lambda: torch.zeros(1, dtype=torch.float64, device="cuda")  # noqa: E731
    t, dt, J = z(), z(), z()
    laser = case.laser if case.laser.on else None
    for _ in range(nsteps):
        htr.htr_rk3_step(ctx, U, T, t, dt, 1, laser, None, work, J)
    htr.htr_check(ctx)
    _check(host(U), fx)
    assert float(host(t)[0]) == pytest.approx(fx["t"], rel=1e-12)
    assert float(host(J)[0]) == pytest.approx(fx["J"], rel=STEP_TOL)


def test_taylor_green_128_after_10_steps():
    fx = _fixture("tgv128")
    _single(synth.case_c2(), fx["steps"], fx)


def test_mixing_layer_256x128x128_after_100_steps():
    fx = _fixture("mixing256")
    case = synth.case_c3()
    assert fx["steps"] == case.steps
    _single(case, fx["steps"], fx)


def test_ensemble_after_50_steps():
    fx = _fixture("ensemble")["members"]
    e = synth.ensemble_c4()
    ctx = htr.Context(e.mech, e.members[0].grid)
    b = htr.Batch.from_cases(ctx, e.members, e.dlnA)
    U, T = htr.batch_state_from_cases(b, e.members)
    work = b.new_work()
    htr.htr_batch_autotune(b, U, T.clone(), work)
    z = lambda: torch.zeros(b.nmem, dtype=torch.float64, device="cuda")  # noqa: E731
    t, dt, J = z(), z(), z()
    htr.htr_rk3_steps_batched(b, U, T, t, dt, 1, e.steps, work, J, use_graph=True)
    htr.htr_batch_check(b)
    Uh, th, Jh = host(U), host(t), host(J)
    sizes = sorted(e.members[int(m)].grid.n[0] for m in fx)
    assert sizes[0] == 32 and sizes[-1] == 96
    for m, f in fx.items():
        m = int(m)
        assert f["steps"] == e.steps
        _check(b.unpack(Uh, ctx.nv, m), f)
        assert float(th[m]) == pytest.approx(f["t"], rel=1e-12)
        assert float(Jh[m]) == pytest.approx(f["J"], rel=STEP_TOL)


def test_adjoint_workload_after_50_steps_and_tangent():
    from paper_2202_02319_amd.adjoint import HeatReleaseObjective, HeatReleaseProblem
    fx = _fixture("adjoint64")
    case = synth.case_c5()
    ctx = htr.Context.from_case(case)
    U0 = htr.cons_from_case(ctx, case)
    T0 = dev(case.T)
    work = ctx.new_work()
    htr.htr_autotune(ctx, U0, T0.clone(), work)
    dtv = fx["dts"][0]
    assert all(d == dtv for d in fx["dts"])          # frozen
    U, T = U0.clone(), T0.clone()
    z = lambda: torch.zeros(1, dtype=torch.float64, device="cuda")  # noqa: E731
    t, dt, J = z(), z(), z()
    dt.fill_(dtv)
    for _ in range(case.steps):
        htr.htr_rk3_step(ctx, U, T, t, dt, 0, case.laser, None, work, J)
    htr.htr_check(ctx)
    _check(host(U), fx)
    assert float(host(J)[0]) == pytest.approx(fx["J"], rel=STEP_TOL)
    # the adjoint gradient along the oracle tangent's direction
    prob = HeatReleaseProblem(ctx, U0, T0, case.laser, dtv, case.steps,
                              checkpoint_every=case.meta["checkpoint_every"])
    theta = torch.tensor([case.laser.E, *case.laser.center] + [0.0] * case.mech.nr, dtype=torch.float64,
                         device="cuda")
    th = theta.clone().requires_grad_(True)
    Jt = HeatReleaseObjective.apply(th, prob)
    Jt.backward()
    grad = host(th.grad)
    tg = fx["tangent"]
    assert float(Jt.item()) == pytest.approx(tg["J"], rel=STEP_TOL)
    assert float((grad * np.array(tg["dtheta"])).sum()) == pytest.approx(tg["dJ"], rel=STEP_TOL)
