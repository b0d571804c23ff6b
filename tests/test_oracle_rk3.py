"""Pins of the oracle's time integration (SSP-RK3 in Shu-Osher form,
Gottlieb et al. 2001, cited in Methods › Numerical method), of the time-integrated heat
release and of the forward-mode tangent."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import synth
from oracle import Oracle


def _single_cell(mech, T, p, Y, dx=1e-4):
    g = synth.uniform_grid((1, 1, 1), dx)
    return synth.Case("cell", mech, g, np.asarray(Y, float)[:, None].copy(), np.array([T]), np.array([p]),
                      np.zeros((3, 1)))


def test_stage_combination_is_simpson():
    """For a right-hand side that depends on t only (a laser pulse in one
    quiescent cell) one step adds dt/6 (f(t) + 4 f(t+dt/2) + f(t+dt)):
    the stage times t, t+dt, t+dt/2 and weights 1/6, 1/6, 2/3."""
    mech = synth.single_species(0.028, 3.5)
    case = _single_cell(mech, 400.0, 1e5, [1.0])
    case.flags = synth.CHEM_OFF | synth.VISC_OFF
    case.laser = synth.Laser(E=3.0e4, center=(0, 0, 0), sigma_r=1.0, t0=2e-6, sigma_t=2.5e-7, on=True)
    o = Oracle(case)
    U = o.prim_to_cons()
    T = case.T.copy()

    def f(t):
        return o.cells(U, T.copy(), t=t)[5 + 2 + 1, 0]
    t, dt = 1.1e-6, 3e-7
    E0 = U[4, 0]
    o.rk3_step(U, T, t, dt)
    assert U[4, 0] - E0 == pytest.approx(dt / 6 * (f(t) + 4 * f(t + dt / 2) + f(t + dt)), rel=1e-12)
    # over the whole pulse the deposited energy converges to E (composite
    # Simpson on a decaying Gaussian converges faster than any power)
    errs = []
    for nst in (8, 16, 24):
        U = o.prim_to_cons()
        T = case.T.copy()
        dt = 4e-6 / nst
        for k in range(nst):
            o.rk3_step(U, T, k * dt, dt)
        errs.append(abs(U[4, 0] - o.prim_to_cons()[4, 0] - 3.0e4))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-12 * 3.0e4 * 1e3, errs


def test_homogeneous_reactor_third_order_and_heat_release():
    """A single closed cell with chemistry: RK3 converges at third order to
    a tight implicit (Radau) solution of the same right-hand side, and the
    accumulated heat release J converges to the time integral of HRR."""
    case = synth.case_c1()
    mech = case.mech
    Y = case.Y[:, 0]
    cell = _single_cell(mech, 1500.0, 101325.0, Y)
    cell.flags = synth.VISC_OFF
    o = Oracle(cell)
    U0 = o.prim_to_cons()
    T0 = cell.T.copy()
    ns = mech.ns
    vol = 1e-4 ** 3
    t_end = 2e-6

    def fun(t, z):
        U = z[:-1].reshape(ns + 4, 1)
        d, h = o.rhs(U, np.array([1500.0]), t=t, want_hrr=True)
        return np.concatenate([d.ravel(), [vol * h[0]]])
    ref = solve_ivp(fun, (0, t_end), np.concatenate([U0.ravel(), [0.0]]), method="Radau", rtol=1e-12,
                    atol=1e-14)
    Uref = ref.y[:-1, -1]
    Jref = ref.y[-1, -1]
    assert abs(Jref) > 0
    eU, eJ = [], []
    for nst in (40, 80, 160):
        U = U0.copy()
        T = T0.copy()
        dt = t_end / nst
        J = 0.0
        for k in range(nst):
            J = o.rk3_step(U, T, k * dt, dt, J=J)
        eU.append(np.max(np.abs(U.ravel()[:ns] - Uref[:ns])) / np.max(np.abs(Uref[:ns])))
        eJ.append(abs(J - Jref) / abs(Jref))
    oU = np.log2(np.array(eU[:-1]) / np.array(eU[1:]))
    oJ = np.log2(np.array(eJ[:-1]) / np.array(eJ[1:]))
    assert oU.min() > 2.7, (eU, oU)
    assert oJ.min() > 2.7, (eJ, oJ)


def test_tangent_matches_central_differences():
    """The Dual-number tangent of one RK3 step (state and parameter
    directions: E, centre, ln A) against central finite differences."""
    mech = synth.case_c1().mech                # explicitly stable chemistry at 1500 K
    case = synth.small_case(n=(6, 5, 4), seed=17, T_base=1500.0, mech=mech)
    case.laser.t0 = 1e-8
    o = Oracle(case)
    U0 = o.prim_to_cons()
    rng = np.random.default_rng(3)
    dU = rng.normal(size=U0.shape) * np.abs(U0).max(axis=1, keepdims=True) * 1e-3
    las = case.laser.as_array()
    dlas = np.array([las[0] * 0.3, 0.2 * las[4], -0.1 * las[4], 0.3 * las[4]])
    dlnA = rng.normal(size=case.mech.nr)
    dt = 0.5 * o.stable_dt(U0, case.T.copy())

    def run(eps):
        U = U0 + eps * dU
        T = case.T.copy()
        l2 = las.copy()
        l2[:4] += eps * dlas
        J = o.rk3_step(U, T, 0.0, dt, laser=l2, lnA=case.mech.lnA + eps * dlnA)
        return U, J
    U = U0.copy()
    dUt = dU.copy()
    J, dJ = o.rk3_tangent(U, dUt, case.T.copy(), 0.0, dt, las, dlas, case.mech.lnA, dlnA)
    h = 1e-6
    Up, Jp = run(h)
    Um, Jm = run(-h)
    fd = (Up - Um) / (2 * h)
    err = np.abs(fd - dUt).max(axis=1) / np.abs(dUt).max(axis=1)
    assert err.max() < 1e-6, err
    assert (Jp - Jm) / (2 * h) == pytest.approx(dJ, rel=1e-6)
