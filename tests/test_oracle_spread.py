"""The oracle against itself on inputs perturbed by one ulp: the spread that
rounding alone produces, which is what the parity tolerances must admit.

- After the 200 SSP-RK3 steps of the 1-D 256-cell reacting case, the
  momentum of a flow that starts at rest differs by more than 1e-9 of its
  own maximum between two oracle runs one ulp apart, while the species
  differ by ~1e-11.  Measured against the acoustic scale rho*c (the
  after-steps measure of the parity tests) the momentum spread is far below
  1e-9.
- A right-hand side of the 128^3 Taylor-Green box and of the 256x128x128
  mixing layer (windows of them) differs, between inputs one ulp apart, by
  more than 1e-12 of max|dU/dt| on some rows, and by well under the
  flux-difference rounding floor 100 eps xi max|F| of the per-RHS parity
  tests.
"""
import numpy as np
import pytest

import synth
from conftest import flux_floor, normwise, normwise_state
from gpu_util import sub_window
from oracle import Oracle


def _perturb(U, seed):
    r = np.random.default_rng(seed)
    return U * (1 + r.choice([-1.0, 1.0], size=U.shape) * 2.0 ** -53)


def _run(o, case, U0, nsteps):
    U = U0.copy()
    T = case.T.copy()
    t = 0.0
    for _ in range(nsteps):
        dt = o.stable_dt(U, T)
        o.rk3_step(U, T, t, dt)
        t += dt
    return U


def test_c1_momentum_spread_after_200_steps():
    case = synth.case_c1()
    o = Oracle(case)
    U0 = o.prim_to_cons()
    ns = o.ns
    Ua = _run(o, case, U0, case.steps)
    rho_c = float(Ua[:ns].sum(axis=0).max() * o.cells(Ua, case.T.copy())[2].max())
    plain, scaled = [], []
    for seed in (1, 2, 3):
        Ub = _run(o, case, _perturb(U0, seed), case.steps)
        e = normwise(Ub, Ua)
        assert e[:ns].max() < 1e-9          # species: far inside the bar
        plain.append(e[ns])                 # x-momentum against its own maximum
        scaled.append(normwise_state(Ub, Ua, ns, rho_c)[ns])
    # rounding alone exceeds the plain 1e-9 bar on the momentum of this near-rest flow
    assert min(plain) > 1e-9, plain
    # against the acoustic scale it is two orders of magnitude inside it
    assert max(scaled) < 1e-11, scaled


@pytest.mark.parametrize("which", ["C2", "C3"])
def test_full_size_rhs_spread_within_flux_floor(which):
    case = synth.case_c2() if which == "C2" else synth.case_c3()
    n = case.grid.n
    rng = np.random.default_rng(0)
    over_plain = False
    for trial in range(2):
        lo = [int(rng.integers(0, n[a])) for a in range(3)]
        sub, flat, inner = sub_window(case, lo, (8, 8, 8), 5)
        o = Oracle(sub)
        U = o.prim_to_cons()
        a = o.rhs(U, sub.T.copy(), t=3e-8)[:, inner]
        b = o.rhs(_perturb(U, trial + 5), sub.T.copy(), t=3e-8)[:, inner]
        p = o.cells(U, sub.T.copy())[1]
        xi_max = max(float(np.max(case.grid.xin[ax])) for ax in range(3) if n[ax] > 1)
        d = np.abs(a - b).max(axis=1)
        over_plain |= bool(np.any(d > 1e-12 * np.abs(a).max(axis=1)))
        assert np.all(d <= 0.5 * flux_floor(U, p, xi_max, o.ns)), d / flux_floor(U, p, xi_max, o.ns)
    assert over_plain
