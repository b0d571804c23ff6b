"""Pins of the energy row of the oracle's diffusive flux (paper: Methods ›
Solver, eqs. (3), (5), (6)): the enthalpy carried by the diffusing species
(the sum of J_s h_s in the heat flux) and the work of the viscous stress
(the divergence of tau . u).  Neither can be seen by conservation, which
holds for any face flux, and both are checked here against properties
fixed by the equations, not against the oracle's own formulas.

- Enthalpy diffusion.  A mixture at rest with uniform T and p and a varying
  composition has no stress, no pressure gradient and no conduction, so the
  energy equation carries only -div(sum_s h_s J_s).  With every h_s uniform
  that is sum_s h_s (-div J_s) = sum_s h_s d(rho_s)/dt, exactly, also in the
  discrete conservative form.  The energy rate must therefore equal the
  enthalpy-weighted species rates to rounding.
- Viscous heating.  At uniform T, p and rho, the viscous part of the energy
  rate minus u . (viscous part of the momentum rate) is the rate of
  internal-energy production, which tends to the dissipation function
  Phi = tau : grad u.  The face-centred work term gives it at second order;
  a work term formed with a node velocity instead of the face velocity is
  only first order, a dropped work term gives -u . div tau, and a flipped one
  gives the wrong sign.

`check_*` raise AssertionError; the tests call them, and the planted-mistake
tests (test_oracle_mutants.py) call them on deliberately broken oracle
builds to show that they fail there."""
import numpy as np
import pytest

import synth
from oracle import Oracle

RU = 8.31446261815324


def _case(mech, g, Y, T, p, vel, flags):
    return synth.Case("energy", mech, g, np.asarray(Y, float), np.asarray(T, float), np.asarray(p, float),
                      np.asarray(vel, float), flags=flags)


def _enthalpies(o, mech, T):
    """h_s(T) in J/kg from the (separately pinned) NASA-7 evaluation."""
    return np.array([o.thermo(s, T)[1] * RU / mech.W[s] * T for s in range(mech.ns)])


def check_enthalpy_diffusion(n=(10, 8, 6), seed=7, stretched=True):
    """dE/dt == sum_s h_s d(rho_s)/dt for a mixture at rest with uniform T, p."""
    mech = synth.make_mechanism(3, 1, seed)
    g = synth.stretched_grid(n, 4e-5, amp=0.15) if stretched else synth.uniform_grid(n, 4e-5)
    N = g.N
    x, y, z = (c.ravel() for c in g.mesh())
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 6)
    s = 0.5 + 0.35 * np.sin(2 * np.pi * x / g.L[0] + ph[0]) * np.cos(2 * np.pi * y / g.L[1] + ph[1]) \
        * np.cos(2 * np.pi * z / g.L[2] + ph[2])
    Ya = np.array([0.7, 0.2, 0.1])
    Yb = np.array([0.05, 0.25, 0.7])
    Y = s[None] * Ya[:, None] + (1 - s[None]) * Yb[:, None]
    T0, p0 = 900.0, 2e5
    o = Oracle(_case(mech, g, Y, np.full(N, T0), np.full(N, p0), np.zeros((3, N)), synth.CHEM_OFF))
    U = o.prim_to_cons()
    d = o.rhs(U, np.full(N, T0))
    h = _enthalpies(o, mech, T0)
    ns = mech.ns
    expect = (h[:, None] * d[:ns]).sum(axis=0)
    scale = np.max(np.abs(h[:, None] * d[:ns]).sum(axis=0))
    # the species really diffuse, with distinct enthalpies
    assert scale > 0 and np.ptp(h) > 0.1 * np.max(np.abs(h))
    assert np.max(np.abs(expect)) > 1e-3 * scale
    assert np.max(np.abs(d[ns + 3] - expect)) <= 1e-10 * scale, np.max(np.abs(d[ns + 3] - expect)) / scale
    # nothing else moves: no stress, no pressure gradient, no mass change
    assert np.max(np.abs(d[:ns].sum(axis=0))) <= 1e-12 * np.max(np.abs(d[:ns]))


def _shear_state(plane, nn, L, amp):
    """Uniform T, p; velocity u_a = A sin(k x_b) + C sin(k x_a), u_b = B sin(k x_a),
    u_c = D sin(k x_a) on the 2-D grid spanning axes plane = (a, b)."""
    a, b = plane
    c = 3 - a - b
    n = [1, 1, 1]
    n[a] = n[b] = nn
    g = synth.uniform_grid(tuple(n), L / nn)
    X = [m.ravel() for m in g.mesh()]
    k = 2 * np.pi / L
    A, B, C, D = amp
    vel = np.zeros((3, g.N))
    vel[a] = A * np.sin(k * X[b]) + C * np.sin(k * X[a])
    vel[b] = B * np.sin(k * X[a])
    vel[c] = D * np.sin(k * X[a])
    phi = (2 * (C * k * np.cos(k * X[a])) ** 2 + (A * k * np.cos(k * X[b]) + B * k * np.cos(k * X[a])) ** 2
           + (D * k * np.cos(k * X[a])) ** 2 - (2.0 / 3.0) * (C * k * np.cos(k * X[a])) ** 2)
    return g, vel, phi


def viscous_heating_errors(plane=(0, 1), sizes=(16, 32, 64)):
    """Relative max error of the discrete viscous internal-energy rate
    against mu Phi, per grid size."""
    mech = synth.single_species(0.028, 3.5, sigma=3.7e-10, epsk=90.0)
    L = 4e-4
    T0, p0 = 400.0, 1e5
    amp = (2.0, 1.5, 0.8, 1.2)
    errs = []
    for nn in sizes:
        g, vel, phi = _shear_state(plane, nn, L, amp)
        N = g.N
        case = _case(mech, g, np.ones((1, N)), np.full(N, T0), np.full(N, p0), vel, synth.CHEM_OFF)
        o = Oracle(case)
        U = o.prim_to_cons()
        d_on = o.rhs(U, np.full(N, T0))
        o.set_flags(synth.CHEM_OFF | synth.VISC_OFF)
        d_off = o.rhs(U, np.full(N, T0))
        dv = d_on - d_off                       # the diffusive part alone
        assert np.max(np.abs(dv[0])) <= 1e-6 * np.max(np.abs(dv[1:4]))   # one species: no mass diffusion
        mu = o.cells(U, np.full(N, T0))[3]
        assert np.ptp(mu) <= 1e-13 * mu[0]
        ev = dv[4] - (vel * dv[1:4]).sum(axis=0)
        ex = mu[0] * phi
        errs.append(np.max(np.abs(ev - ex)) / np.max(np.abs(ex)))
    return errs


def check_viscous_heating(plane=(0, 1)):
    errs = viscous_heating_errors(plane)
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert errs[-1] < 5e-3, errs
    assert min(orders) > 1.8, (errs, orders)


def test_enthalpy_diffusion_energy_row():
    check_enthalpy_diffusion()


def test_enthalpy_diffusion_energy_row_uniform_1d():
    check_enthalpy_diffusion(n=(24, 1, 1), seed=3, stretched=False)


@pytest.mark.parametrize("plane", [(0, 1), (1, 2), (2, 0)])
def test_viscous_heating_energy_row(plane):
    check_viscous_heating(plane)
