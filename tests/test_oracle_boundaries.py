"""Pins of the oracle's non-periodic boundaries (Methods › Diffusion flame ›
Physical model and numerical setup: characteristic in/outflow boundaries
and no-slip walls; Methods › Model rocket combustor › Numerical setup:
isothermal walls at 300 K).  On a bounded axis the first and last nodes lie
on the boundary; faces whose six-point stencil does not fit take the
widest centred interpolation that does (Rusanov where the hybrid switch
marks them); boundary nodes take the locally one-dimensional characteristic
treatment of Poinsot & Lele with the entering waves prescribed.

- plane Couette flow between no-slip walls (one moving): the exact linear
  profile is a steady state of the discrete operator;
- a shear mode between resting walls decays at the exact viscous rate
  nu (pi/L)^2, at second order in the spacing;
- conduction between isothermal walls: the energy rate of a sine
  temperature mode at rest converges at second order to lambda T'';
- an acoustic pulse leaves through an outflow, through either side, with
  less than 1e-4 of it left at sigma = 0 and about 1% at sigma = 0.25 (a
  relaxation that holds the boundary pressure reflects most of it; the
  leaving wave taken for the entering one, planted in a copy of the
  oracle, fails this); a wall reflects it with its sign and amplitude, the
  wall pressure doubling, and a closed box keeps its mass;
- a uniform flow from a held inflow to an outflow at the far-field
  pressure is steady.
"""
import numpy as np
import pytest

import synth
from oracle import Oracle

W_AIR = 0.02897
RU = 8.31446261815324


def _gas(**kw):
    return synth.single_species(W_AIR, 3.5, **kw)


def _line(n, L, axis=1):
    """n nodes along one axis with the first and last on the boundaries."""
    dims = [1, 1, 1]
    dims[axis] = n
    d = L / (n - 1)
    g = synth.uniform_grid(tuple(dims), d)
    g.xnode[axis] = np.arange(n) * d
    return g


def _case(mech, g, T, p, vel, bc, flags=synth.CHEM_OFF, pinf=((0.0, 0.0),) * 3, relax=((0.0, 0.0),) * 3):
    N = g.N
    return synth.Case("bnd", mech, g, np.ones((1, N)), np.asarray(T, float) * np.ones(N),
                      np.asarray(p, float) * np.ones(N), np.asarray(vel, float).reshape(3, -1) * np.ones((3, N)),
                      flags=flags, bc=bc, pinf=pinf, relax=relax)


def _walls(axis=1):
    bc = [(0, 0), (0, 0), (0, 0)]
    bc[axis] = (synth.BC_WALL, synth.BC_WALL)
    return tuple(bc)


def test_couette_profile_is_steady():
    n, L, U = 24, 1e-4, 20.0
    g = _line(n, L)
    y = g.xnode[1]
    vel = np.zeros((3, n))
    vel[0] = U * y / L                      # wall at y = 0 at rest, wall at y = L moving at U
    case = _case(_gas(), g, 300.0, 101325.0, vel, _walls())
    o = Oracle(case)
    U0 = o.prim_to_cons()
    r = o.rhs(U0, case.T.copy())
    mu = o.cells(U0, case.T.copy())[3][0]
    scale = mu * U / L * (n - 1) / L          # one face's shear stress over the spacing
    assert np.abs(r[1]).max() <= 1e-10 * scale     # x-momentum: steady
    rho_c = U0[0][0] * 347.0 * (n - 1) / L
    assert np.abs(r[0]).max() <= 1e-13 * rho_c     # no mass moves (rounding of a uniform p)
    assert np.abs(r[2]).max() <= 1e-10 * scale     # no wall-normal momentum
    # viscous heating is the only energy change: mu (U/L)^2 inside
    assert np.allclose(r[4][1:-1], mu * (U / L) ** 2, rtol=1e-8)


def _shear_decay_rate(n, L=5e-5, U=1.0, nsteps_frac=0.05):
    g = _line(n, L)
    y = g.xnode[1]
    vel = np.zeros((3, n))
    vel[0] = U * np.sin(np.pi * y / L)
    case = _case(_gas(), g, 300.0, 101325.0, vel, _walls())
    o = Oracle(case)
    U0 = o.prim_to_cons()
    c = o.cells(U0, case.T.copy())
    nu = c[3][0] / U0[0][0]
    rate = nu * (np.pi / L) ** 2
    Uc, T = U0.copy(), case.T.copy()
    t = 0.0
    tend = nsteps_frac / rate
    dt = o.stable_dt(Uc, T)
    nst = int(np.ceil(tend / dt))
    dt = tend / nst
    for _ in range(nst):
        o.rk3_step(Uc, T, t, dt)
        t += dt
    mid = n // 2
    A0 = U0[1][mid] / U0[0][mid]
    A1 = Uc[1][mid] / Uc[0][mid]
    return -np.log(A1 / A0) / t, rate


def test_shear_mode_decays_at_the_viscous_rate_second_order():
    e = []
    for n in (17, 33):
        got, exact = _shear_decay_rate(n)
        e.append(abs(got - exact) / exact)
    assert e[1] < 2e-3
    assert np.log2(e[0] / e[1]) > 1.8, e


def _conduction_error(n, L=1e-4, dT=0.05):
    g = _line(n, L)
    y = g.xnode[1]
    T = 300.0 + dT * np.sin(np.pi * y / L)
    case = _case(_gas(), g, T, 101325.0, np.zeros((3, n)), _walls())
    o = Oracle(case)
    U0 = o.prim_to_cons()
    r = o.rhs(U0, case.T.copy())
    lam = o.cells(U0, case.T.copy())[4]
    exact = -lam * (np.pi / L) ** 2 * dT * np.sin(np.pi * y / L)
    inner = slice(1, n - 1)
    return np.abs(r[4][inner] - exact[inner]).max() / np.abs(exact).max()


def test_conduction_between_isothermal_walls_second_order():
    e = [_conduction_error(n) for n in (17, 33, 65)]
    assert e[2] < 2e-3
    assert np.log2(e[1] / e[2]) > 1.8, e


def _pulse(side, n=121, L=1e-3, eps=1e-3, relax=0.25, wall=False, tend_L=None, probe=None):
    """A right-running (side 1) or left-running (side 0) Gaussian acoustic
    pulse leaving through an outflow (or reflected by a wall); returns the
    pressure perturbation left in the domain over the pulse amplitude, at
    tend_L domain-crossing times (default: after it has gone) and the nodes."""
    g = _line(n, L, axis=0)
    x = g.xnode[0]
    p0, T0 = 101325.0, 300.0
    rho0 = p0 * W_AIR / (RU * T0)
    c0 = np.sqrt(1.4 * p0 / rho0)
    xc = 0.6 * L if side == 1 else 0.4 * L
    w = 0.05 * L
    pp = eps * p0 * np.exp(-((x - xc) / w) ** 2)
    sgn = 1.0 if side == 1 else -1.0
    rho = rho0 + pp / c0 ** 2
    p = p0 + pp
    T = p * W_AIR / (RU * rho)
    vel = np.zeros((3, n))
    vel[0] = sgn * pp / (rho0 * c0)
    kind = synth.BC_WALL if wall else synth.BC_OUTFLOW
    bc = ((kind, kind), (0, 0), (0, 0))
    case = _case(_gas(), g, T, p, vel, bc, flags=synth.CHEM_OFF | synth.VISC_OFF,
                 pinf=((p0, p0), (0, 0), (0, 0)), relax=((relax, relax), (0, 0), (0, 0)))
    o = Oracle(case)
    U = o.prim_to_cons()
    Tc = case.T.copy()
    t = 0.0
    tend = (tend_L if tend_L is not None else 0.8) * L / c0
    peak = 0.0
    while t < tend:
        dt = min(o.stable_dt(U, Tc), tend - t)
        o.rk3_step(U, Tc, t, dt)
        t += dt
        if probe is not None:
            peak = max(peak, (o.cells(U, Tc)[1][probe] - p0) / (eps * p0))
    pres = o.cells(U, Tc)[1]
    if probe is not None:
        return peak
    return (pres - p0) / (eps * p0), x / L


def check_outflow_absorbs():
    for side in (0, 1):
        for relax, bound in ((0.0, 1e-4), (0.25, 2e-2)):
            R = np.abs(_pulse(side, relax=relax)[0]).max()
            assert R < bound, (side, relax, R)


def check_wall_reflects():
    # at 0.8 crossing times the pulse has hit the wall at 0.4 and come back
    # 0.4 domain lengths: same sign, same amplitude (inviscid), at x = 0.4 L
    # from the wall it hit; during the reflection the wall pressure doubles
    for side in (0, 1):
        dp, x = _pulse(side, wall=True)
        k = int(np.argmax(np.abs(dp)))
        assert dp[k] > 0.9, (side, dp[k])
        assert abs(x[k] - (0.4 if side == 0 else 0.6)) < 0.02, (side, x[k])
        assert dp.min() > -0.05, (side, dp.min())
    peak = _pulse(0, wall=True, tend_L=0.6, probe=0)
    assert 1.8 < peak < 2.05, peak


def _closed_box_mass_drift(n=121, L=1e-3, eps=1e-3):
    """Total mass (trapezoidal weights, half at the wall nodes) of a closed
    box with an acoustic pulse reflecting from a wall, change after 0.8
    crossing times over the pulse's own mass excess."""
    g = _line(n, L, axis=0)
    x = g.xnode[0]
    p0, T0 = 101325.0, 300.0
    rho0 = p0 * W_AIR / (RU * T0)
    c0 = np.sqrt(1.4 * p0 / rho0)
    pp = eps * p0 * np.exp(-((x - 0.4 * L) / (0.05 * L)) ** 2)
    rho = rho0 + pp / c0 ** 2
    p = p0 + pp
    vel = np.zeros((3, n))
    vel[0] = -pp / (rho0 * c0)
    bc = ((synth.BC_WALL, synth.BC_WALL), (0, 0), (0, 0))
    case = _case(_gas(), g, p * W_AIR / (RU * rho), p, vel, bc, flags=synth.CHEM_OFF | synth.VISC_OFF)
    o = Oracle(case)
    U = o.prim_to_cons()
    Tc = case.T.copy()
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    m0 = (w * U[0]).sum()
    excess = (w * (rho - rho0)).sum()
    t, tend = 0.0, 0.8 * L / c0
    while t < tend:
        dt = min(o.stable_dt(U, Tc), tend - t)
        o.rk3_step(U, Tc, t, dt)
        t += dt
    return ((w * U[0]).sum() - m0) / excess


def check_wall_mass():
    # the wall node's density follows the continuity equation (no entropy
    # wave at u_n = 0): the box keeps its mass through the reflection
    assert abs(_closed_box_mass_drift()) < 0.02


def test_closed_box_keeps_its_mass():
    check_wall_mass()


def test_acoustic_pulse_leaves_through_the_outflow():
    """Perfectly non-reflecting (sigma = 0): below 1e-4 of the pulse left;
    sigma = 0.25: the pressure relaxation reflects about 1%; a relaxation
    so fast that it holds the boundary pressure reflects most of it."""
    check_outflow_absorbs()
    assert np.abs(_pulse(1, relax=300.0)[0]).max() > 0.8


def test_acoustic_pulse_reflects_from_a_wall():
    check_wall_reflects()


MUTANTS = {
    # the leaving acoustic wave taken for the entering one at an outflow
    "outflow_incoming_sign": [("if (sgn * val(un - cc) < 0) L1 = relaxp;", "if (sgn * val(un - cc) > 0) L1 = relaxp;"),
                              ("if (sgn * val(un + cc) < 0) L5 = relaxp;", "if (sgn * val(un + cc) > 0) L5 = relaxp;")],
}


def test_pins_catch_planted_boundary_mistake(tmp_path):
    import oracle.oracle as oo
    lib = oo.build_variant(MUTANTS["outflow_incoming_sign"], str(tmp_path), name="liboracle_outflow_sign.so")
    with oo.use_library(lib):
        with pytest.raises((AssertionError, oo.OracleError)):
            check_outflow_absorbs()


def test_uniform_inflow_to_outflow_is_steady():
    n = 24
    g = _line(n, 1e-3, axis=0)
    bc = ((synth.BC_INFLOW, synth.BC_OUTFLOW), (0, 0), (0, 0))
    vel = np.zeros((3, n))
    vel[0] = 40.0
    vel[1] = 5.0
    case = _case(_gas(), g, 350.0, 101325.0, vel, bc, flags=synth.CHEM_OFF,
                 pinf=((0.0, 101325.0), (0, 0), (0, 0)), relax=((0.0, 0.3), (0, 0), (0, 0)))
    o = Oracle(case)
    U0 = o.prim_to_cons()
    r = o.rhs(U0, case.T.copy())
    flux = np.abs(U0).max(axis=1) * 40.0 * (n - 1) / 1e-3
    assert np.all(np.abs(r).max(axis=1) <= 1e-12 * (flux + 101325.0 * (n - 1) / 1e-3)), np.abs(r).max(axis=1)
