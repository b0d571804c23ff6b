"""GPU parity: the HIP path through the C interface against the oracle on
the same seeded inputs (normwise per conserved variable, max|a-b|/max|b|):
<= 1e-12 per RHS and per-cell quantity, <= 1e-9 after the configured steps."""
import numpy as np
import pytest
import torch

import synth
from conftest import flux_floor, normwise, normwise_state, rhs_close
from gpu_util import both, dev, gpu_cells, gpu_rhs, host, sub_window
from oracle import Oracle
from paper_2202_02319_amd import htr

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-12
STEP_TOL = 1e-9

CASES = [
    ("3d-ragged", dict(n=(13, 7, 6), ns=5, nr=4, seed=21)),
    ("3d-stretched", dict(n=(9, 8, 7), ns=4, nr=3, seed=22, stretched=True)),
    ("2d", dict(n=(17, 11, 1), ns=5, nr=4, seed=23)),
    ("1d", dict(n=(37, 1, 1), ns=3, nr=1, seed=24)),
    ("tiny-wrap", dict(n=(4, 5, 3), ns=4, nr=3, seed=25)),
    ("ns12", dict(n=(10, 6, 5), ns=12, nr=30, seed=26)),
]


def _case(kw, flags=0):
    c = synth.small_case(**kw, flags=flags)
    c.laser.t0 = 0.0
    return c


@pytest.mark.parametrize("name,kw", CASES)
def test_prim_to_cons_parity(name, kw):
    case = _case(kw)
    o, g = both(case)
    U_o = o.prim_to_cons()
    U_g = host(htr.cons_from_case(g, case))
    assert normwise(U_g, U_o).max() <= 1e-14


@pytest.mark.parametrize("name,kw", CASES)
def test_cells_parity(name, kw):
    case = _case(kw)
    o, g = both(case)
    U = o.prim_to_cons()
    ref = o.cells(U, case.T.copy(), t=1e-8)
    got = gpu_cells(g, U, case.T.copy(), 1e-8, case.laser)
    err = normwise(got, ref)
    assert err.max() <= RHS_TOL, err


@pytest.mark.parametrize("flags", [0, synth.FORCE_CENTRAL, synth.FORCE_TENO, synth.CHEM_OFF,
                                   synth.VISC_OFF, synth.VISC_OFF | synth.FORCE_TENO,
                                   synth.WENO3Z, synth.FORCE_TENO | synth.WENO3Z])
@pytest.mark.parametrize("name,kw", CASES)
def test_rhs_parity(name, kw, flags):
    case = _case(kw, flags)
    o, g = both(case)
    U = o.prim_to_cons()
    ref, hrr_o = o.rhs(U, case.T.copy(), t=2e-8, want_hrr=True)
    got, T_g, hrr_g = gpu_rhs(g, U, case.T.copy(), 2e-8, case.laser, want_hrr=True)
    err = normwise(got, ref)
    assert err.max() <= RHS_TOL, err
    assert normwise(hrr_g[None], hrr_o[None]).max() <= RHS_TOL


def test_free_stream_bitwise_on_gpu():
    n = (9, 8, 7)
    for grid in (synth.uniform_grid(n, 1e-4), synth.stretched_grid(n, 1e-4)):
        mech = synth.make_mechanism(5, 4, 3)
        N = grid.N
        Y = np.repeat(np.array([0.1, 0.2, 0.3, 0.15, 0.25])[:, None], N, axis=1)
        vel = np.array([120.0, -80.0, 45.0])[:, None] * np.ones(N)
        for fl in (synth.CHEM_OFF, synth.CHEM_OFF | synth.FORCE_TENO):
            case = synth.Case("fs", mech, grid, Y, np.full(N, 900.0), np.full(N, 2e5), vel, flags=fl)
            o, g = both(case)
            U = o.prim_to_cons()
            got, _ = gpu_rhs(g, U, np.full(N, 900.0), 0.0, None)
            assert np.all(got == 0.0)


def test_stable_dt_parity():
    for case in (synth.case_c1(), _case(CASES[0][1]), _case(CASES[1][1])):
        o, g = both(case)
        U = o.prim_to_cons()
        ref = o.stable_dt(U, case.T.copy())
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        htr.htr_stable_dt(g, dev(U), dev(case.T), dt)
        htr.htr_check(g)
        assert host(dt)[0] == pytest.approx(ref, rel=1e-13)


def _run_gpu_steps(g, case, U0, nsteps, dts=None):
    """Steps on the GPU: dt from the fused in-step CFL reduction, or given."""
    U = dev(U0)
    T = dev(case.T)
    work = g.new_work()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k in range(nsteps):
        if dts is not None:
            dt.fill_(dts[k])
        htr.htr_rk3_step(g, U, T, t, dt, dts is None, case.laser if case.laser.on else None, None, work, J)
    htr.htr_check(g)
    return host(U), float(host(J)[0]), float(host(t)[0])


def _rho_c(o, U, case):
    """Acoustic momentum scale max(rho) * max(c) of a state."""
    c = o.cells(U, case.T.copy())[2]
    return float(U[:o.ns].sum(axis=0).max() * c.max())


def _run_oracle_steps(o, case, U0, nsteps):
    U = U0.copy()
    T = case.T.copy()
    t, J, dts = 0.0, 0.0, []
    for _ in range(nsteps):
        dt = o.stable_dt(U, T)
        J = o.rk3_step(U, T, t, dt, J=J)
        t += dt
        dts.append(dt)
    return U, J, t, dts


def test_c1_after_200_steps():
    """C1 (256 cells, 5 species / 4 reactions, 200 SSP-RK3 steps at CFL 0.5)."""
    case = synth.case_c1()
    o, g = both(case)
    U0 = o.prim_to_cons()
    Uo, Jo, to, dts = _run_oracle_steps(o, case, U0, case.steps)
    Ug, Jg, tg = _run_gpu_steps(g, case, U0, case.steps)
    assert tg == pytest.approx(to, rel=1e-12)
    assert normwise_state(Ug, Uo, o.ns, _rho_c(o, Uo, case)).max() <= STEP_TOL
    assert Jg == pytest.approx(Jo, rel=STEP_TOL)


@pytest.mark.parametrize("name,kw", CASES[:3])
def test_steps_with_laser(name, kw):
    case = _case(kw)
    case.mech = synth.case_c1().mech if case.mech.ns == 5 else case.mech
    case.laser.t0 = 3e-8
    o, g = both(case)
    U0 = o.prim_to_cons()
    Uo, Jo, _, dts = _run_oracle_steps(o, case, U0, 5)
    Ug, Jg, _ = _run_gpu_steps(g, case, U0, 5, dts=dts)
    assert normwise_state(Ug, Uo, o.ns, _rho_c(o, Uo, case)).max() <= STEP_TOL
    assert Jg == pytest.approx(Jo, rel=STEP_TOL, abs=1e-30)


@pytest.mark.parametrize("which", ["C2", "C3"])
def test_full_size_rhs_sampled(which):
    """Full-size workloads: the GPU RHS of the whole grid (the launch the
    benchmark times) against the oracle on periodic windows with a 5-cell
    halo around sampled blocks."""
    case = synth.case_c2() if which == "C2" else synth.case_c3()
    g = htr.Context.from_case(case)
    Ud = htr.cons_from_case(g, case)
    Td = dev(case.T)
    out = torch.empty_like(Ud)
    htr.htr_rhs(g, Ud, Td, 3e-8, case.laser if case.laser.on else None, out)
    htr.htr_check(g)
    got = host(out)
    U_full = host(Ud)
    from oracle import Oracle
    n = case.grid.n
    rng = np.random.default_rng(0)
    for trial in range(3):
        lo = [int(rng.integers(0, n[a])) for a in range(3)]
        if which == "C3" and trial == 0:      # a block on the laser kernel
            lo = [int(np.argmin(np.abs(case.grid.xnode[a] - case.laser.center[a]))) - 4 for a in range(3)]
        sub, flat, inner = sub_window(case, lo, (8, 8, 8), 5)
        o = Oracle(sub)
        Uw = U_full[:, flat]
        ref = o.rhs(Uw, sub.T.copy(), t=3e-8)[:, inner]
        p = o.cells(Uw, sub.T.copy())[1]
        xi_max = max(float(np.max(case.grid.xin[a])) for a in range(3) if n[a] > 1)
        ok, ratio = rhs_close(got[:, flat][:, inner], ref, flux_floor(Uw, p, xi_max, o.ns), rel=RHS_TOL)
        assert ok, (trial, ratio, normwise(got[:, flat][:, inner], ref))


@pytest.mark.parametrize("what", ["nan", "negative_rho", "newton", "hot", "cold"])
def test_device_errors_match_the_oracle(what):
    """A bad cell (NaN, rho <= 0, an energy the Newton iteration cannot
    reach, a temperature outside [Tmin, Tmax]) is latched on the device and
    reported by htr_check with the error the oracle returns for the same
    state; the report clears the status, so the next good call passes.  The
    kernels run to completion on such input (bounded Newton iteration)."""
    from oracle import OracleError
    names = {4: "ENONFINITE", 5: "ENEWTON", 6: "ETRANGE"}
    case = _case(CASES[0][1])
    q, ns = 17, case.mech.ns
    if what in ("hot", "cold"):
        case.T = case.T.copy()
        case.T[q] = 7000.0 if what == "hot" else 150.0
    o, g = both(case)
    U = o.prim_to_cons()
    if what == "nan":
        U[2, q] = np.nan
    elif what == "negative_rho":
        U[:ns, q] = -np.abs(U[:ns, q])
    elif what == "newton":
        U[ns + 3, q] *= 6.0
    T = case.T.copy()
    T[q] = 1500.0                      # the Newton guess
    with pytest.raises(OracleError) as oe:
        o.rhs(U, T.copy())
    expect = names[oe.value.code]
    out = torch.empty((o.nv, o.N), dtype=torch.float64, device="cuda")
    htr.htr_rhs(g, dev(U), dev(T), 0.0, case.laser, out)
    with pytest.raises(htr.HTRError, match=expect):
        htr.htr_check(g)
    clean = _case(CASES[0][1])
    htr.htr_rhs(g, dev(Oracle(clean).prim_to_cons()), dev(clean.T), 0.0, clean.laser, out)
    htr.htr_check(g)
