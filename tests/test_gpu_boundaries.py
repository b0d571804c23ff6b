"""GPU parity with non-periodic boundaries (Methods › Diffusion flame ›
Physical model and numerical setup; Methods › Model rocket combustor ›
Numerical setup): characteristic inflow/outflow and isothermal no-slip
walls, the HIP path through the C interface against the oracle on the same
seeded inputs.  Per RHS <= 1e-12 normwise per conserved variable, after
three SSP-RK3 steps with the in-step dt <= 1e-9 (momentum against the
acoustic scale rho*c).  1-D, 2-D and 3-D grids, walls on one axis with
inflow/outflow or outflow on another, hybrid, TENO6 on every face, WENO3-Z
and inviscid schemes, and a grid of several ragged tiles along every axis
(the tiled sweeps and the boundary kernel meet)."""
import numpy as np
import pytest
import torch

import synth
from conftest import normwise, normwise_state
from gpu_util import both, dev, gpu_rhs, host
from paper_2202_02319_amd import _lib, htr

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-12
STEP_TOL = 1e-9
W, I, O = synth.BC_WALL, synth.BC_INFLOW, synth.BC_OUTFLOW
P0 = 101325.0

CASES = [
    ("2d-walls", (16, 12, 1), ((0, 0), (W, W), (0, 0)), 0),
    ("3d-in-out-walls", (14, 10, 9), ((I, O), (W, W), (0, 0)), 0),
    ("3d-walls-outflow-teno", (12, 9, 10), ((0, 0), (W, W), (O, O)), synth.FORCE_TENO),
    ("1d-outflow", (20, 1, 1), ((O, O), (0, 0), (0, 0)), 0),
    ("2d-out-walls-weno", (18, 11, 1), ((O, O), (W, W), (0, 0)), synth.FORCE_TENO | synth.WENO3Z),
    ("3d-walls-inviscid", (12, 10, 8), ((0, 0), (W, W), (0, 0)), synth.VISC_OFF),
    ("3d-multitile", (40, 24, 20), ((O, O), (W, W), (0, 0)), 0),
]


def _case(n, bc, flags, seed=5):
    c = synth.small_case(n=n, seed=seed, mech=synth.case_c1().mech, flags=flags)
    c.laser.t0 = 0.0
    c.bc = bc
    c.pinf = ((P0, P0),) * 3
    c.relax = ((0.25, 0.25),) * 3
    g = c.grid
    idx = np.arange(g.N)
    stride = [1, g.n[0], g.n[0] * g.n[1]]
    for a in range(3):
        if bc[a][0] == W:   # the walls are at rest
            ca = (idx // stride[a]) % g.n[a]
            c.vel[:, (ca == 0) | (ca == g.n[a] - 1)] = 0.0
    return c


@pytest.mark.parametrize("name,n,bc,flags", CASES)
def test_rhs_parity(name, n, bc, flags):
    case = _case(n, bc, flags)
    o, g = both(case)
    U = o.prim_to_cons()
    ref, hrr_o = o.rhs(U, case.T.copy(), t=2e-8, want_hrr=True)
    got, _, hrr_g = gpu_rhs(g, U, case.T.copy(), 2e-8, case.laser, want_hrr=True)
    err = normwise(got, ref)
    assert err.max() <= RHS_TOL, err
    assert normwise(hrr_g[None], hrr_o[None]).max() <= RHS_TOL


@pytest.mark.parametrize("name,n,bc,flags", CASES)
def test_steps_parity(name, n, bc, flags):
    case = _case(n, bc, flags)
    o, g = both(case)
    U0 = o.prim_to_cons()
    U, T, t, J = U0.copy(), case.T.copy(), 0.0, 0.0
    for _ in range(3):
        dt = o.stable_dt(U, T)
        J = o.rk3_step(U, T, t, dt, J=J)
        t += dt
    Ug, Tg = dev(U0), dev(case.T)
    z = lambda: torch.zeros(1, dtype=torch.float64, device="cuda")  # noqa: E731
    td, dtd, Jd = z(), z(), z()
    work = g.new_work()
    for _ in range(3):
        htr.htr_rk3_step(g, Ug, Tg, td, dtd, 1, case.laser, None, work, Jd)
    htr.htr_check(g)
    assert float(host(td)[0]) == pytest.approx(t, rel=1e-12)
    rho_c = float(U[:o.ns].sum(axis=0).max() * o.cells(U, T.copy())[2].max())
    assert normwise_state(host(Ug), U, o.ns, rho_c).max() <= STEP_TOL
    assert float(host(Jd)[0]) == pytest.approx(J, rel=STEP_TOL, abs=1e-30)


def test_acoustic_pulse_through_outflow_matches_the_oracle():
    """The outflow pin's set-up (a pulse leaving through a characteristic
    outflow) on the GPU: the state after the pulse has left equals the
    oracle's, and little of the pulse is left.  Central fluxes: in 1-D the
    dilatation sensor is one wherever the velocity varies at all, so the
    hybrid scheme switches on roundoff in the quiet part of the domain, and
    the oracle run against itself from inputs one ulp apart already spreads
    by 3e-7 in the density after these steps (5e-15 with central fluxes)."""
    n, L, eps = 121, 1e-3, 1e-3
    W_AIR, RU = 0.02897, 8.31446261815324
    g = synth.uniform_grid((n, 1, 1), L / (n - 1))
    g.xnode[0] = np.arange(n) * L / (n - 1)
    x = g.xnode[0]
    T0 = 300.0
    rho0 = P0 * W_AIR / (RU * T0)
    c0 = np.sqrt(1.4 * P0 / rho0)
    pp = eps * P0 * np.exp(-((x - 0.6 * L) / (0.05 * L)) ** 2)
    rho, p = rho0 + pp / c0 ** 2, P0 + pp
    vel = np.zeros((3, n))
    vel[0] = pp / (rho0 * c0)
    case = synth.Case("pulse", synth.single_species(W_AIR, 3.5), g, np.ones((1, n)), p * W_AIR / (RU * rho), p, vel,
                      flags=synth.CHEM_OFF | synth.VISC_OFF | synth.FORCE_CENTRAL, bc=((O, O), (0, 0), (0, 0)),
                      pinf=((P0, P0),) * 3,
                      relax=((0.25, 0.25),) * 3)
    o, gc = both(case)
    U0 = o.prim_to_cons()
    U, T, t, dts = U0.copy(), case.T.copy(), 0.0, []
    while t < 0.8 * L / c0:
        dt = o.stable_dt(U, T)
        o.rk3_step(U, T, t, dt)
        t += dt
        dts.append(dt)
    Ug, Tg = dev(U0), dev(case.T)
    z = lambda: torch.zeros(1, dtype=torch.float64, device="cuda")  # noqa: E731
    td, dtd = z(), z()
    work = gc.new_work()
    for dt in dts:
        dtd.fill_(dt)
        htr.htr_rk3_step(gc, Ug, Tg, td, dtd, 0, None, None, work, None)
    htr.htr_check(gc)
    rho_c = float(U[0].max() * o.cells(U, T.copy())[2].max())
    assert normwise_state(host(Ug), U, 1, rho_c).max() <= STEP_TOL
    pres = o.cells(host(Ug), host(Tg))[1]
    assert np.abs(pres - P0).max() < 0.02 * eps * P0


def test_refusals():
    case = _case((16, 12, 1), ((0, 0), (W, W), (0, 0)), 0)
    g = htr.Context.from_case(case)
    bad = [((0, 0), (W, 0), (0, 0)), ((0, 0), (W, 7), (0, 0))]
    for bc in bad:
        with pytest.raises(htr.HTRError, match="EINVAL"):
            htr.htr_set_boundaries(g, bc, case.pinf, case.relax)
    with pytest.raises(htr.HTRError, match="EINVAL"):      # a bounded axis of 4 nodes
        g4 = htr.Context.from_case(_case((16, 4, 1), ((0, 0), (0, 0), (0, 0)), 0))
        htr.htr_set_boundaries(g4, ((0, 0), (W, W), (0, 0)), case.pinf, case.relax)
    with pytest.raises(htr.HTRError, match="EINVAL"):      # outflow without a far-field pressure
        htr.htr_set_boundaries(g, ((O, O), (W, W), (0, 0)), ((0.0, 0.0),) * 3, case.relax)
    U = htr.cons_from_case(g, case)
    T = dev(case.T)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.full((1,), 1e-9, dtype=torch.float64, device="cuda")
    with pytest.raises(htr.HTRError, match="UNSUPPORTED"):
        htr.htr_rk3_step_taped(g, U, T, t, dt, 0, None, None, g.new_work(), None, htr.new_tape(g))
    with pytest.raises(htr.HTRError, match="UNSUPPORTED"):
        htr.Batch.from_cases(g, [case])
    curv = synth.Case("c", case.mech, synth.wavy_grid((16, 12, 1), 5e-5, amp=0.25, seed=3), case.Y, case.T, case.p,
                      case.vel)
    gcv = htr.Context.from_case(curv)
    with pytest.raises(htr.HTRError, match="UNSUPPORTED"):
        htr.htr_set_boundaries(gcv, ((0, 0), (W, W), (0, 0)), case.pinf, case.relax)
    # all-periodic restores the periodic grid: the RHS equals a fresh periodic context's
    htr.htr_set_boundaries(g, ((0, 0),) * 3, case.pinf, case.relax)
    gp = htr.Context(case.mech, case.grid)
    a, b = torch.empty_like(U), torch.empty_like(U)
    htr.htr_rhs(g, U, dev(case.T), 0.0, None, a)
    htr.htr_rhs(gp, U, dev(case.T), 0.0, None, b)
    htr.htr_check(g)
    assert torch.equal(a, b)
    assert _lib.HTR_BC_WALL == synth.BC_WALL
