"""Brute force of the whole right-hand side: the oracle's dU/dt and heat
release on tiny periodic grids against a straight-line 40-digit evaluation
(tests/mp_rhs.py) of everything the step computes: Newton temperature,
NASA-7 thermodynamics, Chapman-Enskog/Wilke/Eucken/Bird transport, species
fluxes with the correction velocity, the heat flux with the species
enthalpy transport, the viscous stress with its cross terms and its work,
reversible Arrhenius chemistry with K_c, the laser source, the hybrid
switch, central and TENO6 convective fluxes (paper: Methods › Solver, eqs.
(1)-(6); Methods › Numerical method).

The two evaluations share no code (the one-face TENO6 reconstruction
aside, pinned on its own), so agreement to ~1e-13 bounds the oracle's
rounding and rules out a dropped, mis-signed or mis-indexed term anywhere
in the right-hand side."""
import numpy as np
import pytest

import synth
from mp_rhs import rhs as mp_rhs
from oracle import Oracle


def _mech(ns, nr, seed):
    """Seeded mechanism; three species admit one element-balanced reaction
    of the enumerated kind, so a second one is added as the same reaction
    written the other way round with its own seeded Arrhenius parameters
    (a duplicate reaction in the CHEMKIN sense)."""
    if not (ns == 3 and nr == 2):
        return synth.make_mechanism(ns, nr, seed)
    m = synth.make_mechanism(3, 1, seed)
    rng = np.random.default_rng(seed + 1000)
    order = int(m.nu_r[0].sum())
    m.lnA = np.append(m.lnA, rng.uniform(6, 12) * np.log(10) + (order - 1) * np.log(1e-6))
    m.beta = np.append(m.beta, rng.uniform(-1, 1))
    m.Ea = np.append(m.Ea, rng.uniform(50e3, 200e3))
    m.nu_f = np.vstack([m.nu_f, m.nu_r[:1]]).astype(np.int32)
    m.nu_r = np.vstack([m.nu_r, m.nu_f[:1]]).astype(np.int32)
    return m


def check_whole_rhs(n, ns, nr, seed, flags, tol=1e-12):
    case = synth.small_case(n=n, seed=seed, flags=flags, laser=True, T_base=1400.0, noise=0.08,
                            mech=_mech(ns, nr, seed))
    case.laser.t0 = 2e-8
    t = 1e-8
    o = Oracle(case)
    U = o.prim_to_cons()
    ref, hrr = o.rhs(U, case.T.copy(), t=t, want_hrr=True)
    bf, bf_hrr = mp_rhs(case, U, t=t, flags=flags)
    scale = np.abs(bf).max(axis=1)
    # a velocity component along an inactive axis may be zero throughout;
    # its row must then be exactly zero on both sides
    zero = scale == 0
    assert np.all(ref[zero] == 0) and zero.sum() <= 1
    err = np.abs(ref - bf).max(axis=1) / np.where(zero, 1.0, scale)
    assert err.max() < tol, err
    if not flags & synth.CHEM_OFF:
        assert np.abs(bf_hrr).max() > 0
        assert np.abs(hrr - bf_hrr).max() <= tol * np.abs(bf_hrr).max()
    return err


GRIDS = [(4, 1, 1), (4, 4, 4), (3, 4, 5)]


@pytest.mark.parametrize("flags", [synth.FORCE_CENTRAL, synth.FORCE_TENO, 0])
@pytest.mark.parametrize("n", GRIDS)
def test_whole_rhs_brute_force(n, flags):
    check_whole_rhs(n, ns=3, nr=2, seed=sum(n) + 17, flags=flags)


@pytest.mark.parametrize("n", [(4, 1, 1), (3, 4, 5)])
def test_whole_rhs_brute_force_two_species(n):
    check_whole_rhs(n, ns=2, nr=1, seed=23, flags=0)
