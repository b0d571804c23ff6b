"""GPU parity on general curvilinear grids (Methods › Numerical method, the mapped
equations): the HIP path through the C interface against the oracle on the
same seeded inputs, normwise per row (max|a-b|/max|b|): metric terms,
per-cell quantities and the RHS <= 1e-12, steps <= 1e-9.  Grids: a wavy
grid (every metric term varies along every axis), a rotated lattice, the
skewed grid of the convergence tests; ragged sizes, 2-D and 1-D cases,
short periods that wrap the stencils more than once, 12 species, and grids
that span several ragged face tiles along every direction.  At the
benchmark's size (128^3 wavy grid) the checks are properties that hold at
any size: free-stream preservation and discrete conservation."""
import numpy as np
import pytest
import torch

import synth
from conftest import normwise, normwise_state
from gpu_util import both, dev, gpu_cells, gpu_rhs, host
from oracle import Oracle
from paper_2202_02319_amd import htr

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-12
STEP_TOL = 1e-9

CASES = [
    ("3d-ragged", dict(n=(13, 7, 6), ns=5, nr=4, seed=21)),
    ("2d", dict(n=(17, 11, 1), ns=5, nr=4, seed=23)),
    ("tiny-wrap", dict(n=(4, 5, 3), ns=4, nr=3, seed=25)),
    ("ns12", dict(n=(10, 6, 5), ns=12, nr=30, seed=26)),
    ("1d", dict(n=(37, 1, 1), ns=3, nr=1, seed=24)),
]
GRIDS = ["wavy", "rotated", "skewed"]


def _grid(kind, n, d):
    if kind == "wavy":
        return synth.wavy_grid(n, d, amp=0.25, seed=7)
    if kind == "skewed":
        return synth.skewed_grid(n, d, beta=0.2)
    if n[1] == 1 and n[2] == 1:   # 1-D: a rotation would tilt the inactive axes; a scaled lattice instead
        return synth.affine_grid(n, d, np.diag([1.3, 1.0, 1.0]))
    R = synth.rotation(0.3, -0.5, 0.9) if n[2] > 1 else synth.rotation(0.0, 0.0, 0.6)
    return synth.affine_grid(n, d, R)


def _case(kw, kind, flags=0, c1_mech=False):
    c = synth.small_case(**kw, flags=flags)
    c.laser.t0 = 0.0
    if c1_mech and c.mech.ns == 5:   # a mechanism valid over the laser-heated range
        c.mech = synth.case_c1().mech
    g = _grid(kind, c.grid.n, c.grid.spacing())
    return synth.Case(c.name + "-" + kind, c.mech, g, c.Y, c.T, c.p, c.vel, laser=c.laser, flags=flags)


@pytest.mark.parametrize("kind", GRIDS)
@pytest.mark.parametrize("name,kw", CASES)
def test_metric_parity(name, kw, kind):
    case = _case(kw, kind)
    o, g = both(case)
    mt_o, mf_o, jac_o = o.metrics()
    mt = torch.empty((10, g.N), dtype=torch.float64, device="cuda")
    mf = torch.empty((9, g.N), dtype=torch.float64, device="cuda")
    htr.htr_grid_metrics(g, mt, mf)
    htr.htr_check(g)
    mt, mf = host(mt), host(mf)
    scale = np.abs(mt_o).max()
    assert np.abs(mt[:9] - mt_o.reshape(9, -1)).max() <= 1e-13 * scale
    assert np.abs(mf - mf_o.reshape(9, -1)).max() <= 1e-13 * scale
    assert normwise(mt[9:], jac_o[None]).max() <= 1e-13


@pytest.mark.parametrize("kind", GRIDS)
@pytest.mark.parametrize("name,kw", CASES)
def test_cells_parity(name, kw, kind):
    case = _case(kw, kind)
    o, g = both(case)
    U = o.prim_to_cons()
    ref = o.cells(U, case.T.copy(), t=1e-8)
    got = gpu_cells(g, U, case.T.copy(), 1e-8, case.laser)
    err = normwise(got, ref)
    assert err.max() <= RHS_TOL, err


@pytest.mark.parametrize("flags", [0, synth.FORCE_CENTRAL, synth.FORCE_TENO, synth.CHEM_OFF,
                                   synth.VISC_OFF, synth.VISC_OFF | synth.FORCE_TENO,
                                   synth.WENO3Z, synth.FORCE_TENO | synth.WENO3Z])
@pytest.mark.parametrize("kind", GRIDS)
@pytest.mark.parametrize("name,kw", CASES)
def test_rhs_parity(name, kw, kind, flags):
    case = _case(kw, kind, flags)
    o, g = both(case)
    U = o.prim_to_cons()
    ref, hrr_o = o.rhs(U, case.T.copy(), t=2e-8, want_hrr=True)
    got, T_g, hrr_g = gpu_rhs(g, U, case.T.copy(), 2e-8, case.laser, want_hrr=True)
    err = normwise(got, ref)
    assert err.max() <= RHS_TOL, err
    assert normwise(hrr_g[None], hrr_o[None]).max() <= RHS_TOL


# grids spanning several ragged face tiles along every stencil direction of
# the convective face kernel (64 x 4 faces per tile along x, 16 x 16 along y
# and z): 70 = 64 + 6, 37 = 2 x 16 + 5, 21 = 16 + 5, 130 = 2 x 64 + 2, 40 = 2 x 16 + 8
MULTITILE = [("3d-70x37x21", (70, 37, 21)), ("2d-130x40", (130, 40, 1))]


@pytest.mark.parametrize("flags", [0, synth.FORCE_TENO, synth.VISC_OFF | synth.FORCE_TENO])
@pytest.mark.parametrize("kind", ["wavy", "skewed"])
@pytest.mark.parametrize("name,n", MULTITILE)
def test_rhs_parity_multitile(name, n, kind, flags):
    """The RHS where face tiles meet along every direction (halo values staged
    by neighbouring tiles) against the oracle, normwise per row <= 1e-12."""
    case = _case(dict(n=n, ns=5, nr=4, seed=27), kind, flags)
    o, g = both(case)
    U = o.prim_to_cons()
    ref, hrr_o = o.rhs(U, case.T.copy(), t=2e-8, want_hrr=True)
    got, T_g, hrr_g = gpu_rhs(g, U, case.T.copy(), 2e-8, case.laser, want_hrr=True)
    err = normwise(got, ref)
    assert err.max() <= RHS_TOL, err
    assert normwise(hrr_g[None], hrr_o[None]).max() <= RHS_TOL
    if flags == 0:   # the hybrid switch picks both schemes on these grids
        _, mask = o.rhs(U, case.T.copy(), t=2e-8, want_mask=True)
        assert 0 < mask.mean() < 1


@pytest.mark.parametrize("name,n", MULTITILE)
def test_steps_multitile(name, n):
    """Three SSP-RK3 steps with the in-step dt on the multi-tile wavy grids."""
    case = _case(dict(n=n, ns=5, nr=4, seed=28), "wavy", c1_mech=True)
    o, g = both(case)
    U0 = o.prim_to_cons()
    U, T, t = U0.copy(), case.T.copy(), 0.0
    for _ in range(3):
        dt = o.stable_dt(U, T)
        o.rk3_step(U, T, t, dt)
        t += dt
    Ug, Tg = dev(U0), dev(case.T)
    work = g.new_work()
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    td = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        htr.htr_rk3_step(g, Ug, Tg, td, dtd, 1, case.laser, None, work, None)
    htr.htr_check(g)
    assert float(host(td)[0]) == pytest.approx(t, rel=1e-12)
    c = o.cells(U, T)[2]
    rho_c = float(U[:o.ns].sum(axis=0).max() * c.max())
    assert normwise_state(host(Ug), U, o.ns, rho_c).max() <= STEP_TOL


@pytest.mark.parametrize("kind", GRIDS)
def test_stable_dt_parity(kind):
    for _, kw in CASES:
        case = _case(kw, kind)
        o, g = both(case)
        U = o.prim_to_cons()
        ref = o.stable_dt(U, case.T.copy())
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        htr.htr_stable_dt(g, dev(U), dev(case.T), dt)
        htr.htr_check(g)
        assert host(dt)[0] == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("kind", GRIDS)
@pytest.mark.parametrize("name,kw", CASES[:2])
def test_steps_with_laser(name, kw, kind):
    """Five SSP-RK3 steps (the oracle's dt sequence), laser on, J accumulated."""
    case = _case(kw, kind, c1_mech=True)
    case.laser.t0 = 3e-8
    o, g = both(case)
    U0 = o.prim_to_cons()
    U, T = U0.copy(), case.T.copy()
    t, J, dts = 0.0, 0.0, []
    for _ in range(5):
        dt = o.stable_dt(U, T)
        J = o.rk3_step(U, T, t, dt, J=J)
        t += dt
        dts.append(dt)
    Ug, Tg = dev(U0), dev(case.T)
    work = g.new_work()
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    td = torch.zeros(1, dtype=torch.float64, device="cuda")
    Jd = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k in range(5):
        dtd.fill_(dts[k])
        htr.htr_rk3_step(g, Ug, Tg, td, dtd, 0, case.laser, None, work, Jd)
    htr.htr_check(g)
    c = o.cells(U, T)[2]
    rho_c = float(U[:o.ns].sum(axis=0).max() * c.max())
    assert normwise_state(host(Ug), U, o.ns, rho_c).max() <= STEP_TOL
    assert float(host(Jd)[0]) == pytest.approx(J, rel=STEP_TOL, abs=1e-30)


def test_in_step_dt_matches_oracle():
    """The fused in-step CFL step on a curvilinear grid: three steps with the
    step computed on the device."""
    case = _case(CASES[0][1], "wavy", c1_mech=True)
    o, g = both(case)
    U0 = o.prim_to_cons()
    U, T, t = U0.copy(), case.T.copy(), 0.0
    for _ in range(3):
        dt = o.stable_dt(U, T)
        o.rk3_step(U, T, t, dt)
        t += dt
    Ug, Tg = dev(U0), dev(case.T)
    work = g.new_work()
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    td = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        htr.htr_rk3_step(g, Ug, Tg, td, dtd, 1, case.laser, None, work, None)
    htr.htr_check(g)
    assert float(host(td)[0]) == pytest.approx(t, rel=1e-12)
    c = o.cells(U, T)[2]
    rho_c = float(U[:o.ns].sum(axis=0).max() * c.max())
    assert normwise_state(host(Ug), U, o.ns, rho_c).max() <= STEP_TOL


def _uniform_state_case(grid, flags):
    mech = synth.make_mechanism(5, 4, 3)
    N = grid.N
    Y = np.repeat(np.array([0.1, 0.2, 0.3, 0.15, 0.25])[:, None], N, axis=1)
    vel = np.array([120.0, -80.0, 45.0 if grid.n[2] > 1 else 0.0])[:, None] * np.ones(N)
    return synth.Case("fs", mech, grid, Y, np.full(N, 900.0), np.full(N, 2e5), vel, flags=flags)


@pytest.mark.parametrize("flags", [synth.CHEM_OFF, synth.CHEM_OFF | synth.FORCE_TENO,
                                   synth.CHEM_OFF | synth.FORCE_TENO | synth.WENO3Z])
def test_free_stream_on_gpu(flags):
    for grid in (synth.wavy_grid((10, 9, 8), 1e-4, amp=0.25, seed=4), synth.skewed_grid((12, 10, 1), 1e-4)):
        case = _uniform_state_case(grid, flags)
        o, g = both(case)
        U = o.prim_to_cons()
        got, _ = gpu_rhs(g, U, np.full(grid.N, 900.0), 0.0, None)
        mt, _, jac = o.metrics()
        scale = (np.abs(U).max(axis=1) + 2e5) * 600.0 * np.abs(mt).max() * jac.max()
        assert (np.abs(got).max(axis=1) / scale).max() < 1e-13


def test_full_size_properties():
    """128^3 wavy grid, 9 species (the benchmark's curvilinear launch):
    a uniform flow stays uniform, and without sources sum (1/J) dU/dt
    vanishes for the mixing-layer state of the same size."""
    n = (128, 128, 128)
    grid = synth.wavy_grid(n, 50e-6, amp=0.25, seed=11)
    mech = synth.case_c3(n=(8, 8, 8)).mech
    N = grid.N
    Y = np.repeat(synth.cases.dirichlet_Y(np.random.default_rng(3), mech.ns)[:, None], N, axis=1)
    vel = np.array([120.0, -80.0, 45.0])[:, None] * np.ones(N)
    case = synth.Case("fs128", mech, grid, Y, np.full(N, 900.0), np.full(N, 2e5), vel,
                      flags=synth.CHEM_OFF)
    g = htr.Context.from_case(case)
    U = htr.cons_from_case(g, case)
    T = dev(case.T)
    out = torch.empty_like(U)
    htr.htr_rhs(g, U, T, 0.0, None, out)
    htr.htr_check(g)
    mt = torch.empty((10, N), dtype=torch.float64, device="cuda")
    mf = torch.empty((9, N), dtype=torch.float64, device="cuda")
    htr.htr_grid_metrics(g, mt, mf)
    Uh, got, mth = host(U), host(out), host(mt)
    scale = (np.abs(Uh).max(axis=1) + 2e5) * 600.0 * np.abs(mth[:9]).max() * mth[9].max()
    assert (np.abs(got).max(axis=1) / scale).max() < 1e-12
    # a non-uniform state: the mixing layer's fields on the wavy grid
    c3 = synth.case_c3(n=n)
    c3 = synth.Case("ml128", c3.mech, grid, c3.Y, c3.T, c3.p, c3.vel, flags=synth.CHEM_OFF)
    g3 = htr.Context.from_case(c3)
    U3 = htr.cons_from_case(g3, c3)
    out3 = torch.empty_like(U3)
    htr.htr_rhs(g3, U3, dev(c3.T), 0.0, None, out3)
    htr.htr_check(g3)
    d = host(out3)
    vol = 1.0 / mth[9]
    tot = (d * vol[None]).sum(axis=1)
    mag = (np.abs(d) * vol[None]).sum(axis=1)
    assert np.all(np.abs(tot) <= 1e-11 * mag), np.abs(tot) / mag


def test_refusals_and_bad_grids():
    case = _case(CASES[0][1], "wavy")
    g = htr.Context.from_case(case)
    U = htr.cons_from_case(g, case)
    T = dev(case.T)
    with pytest.raises(htr.HTRError, match="UNSUPPORTED"):
        htr.htr_set_tiling(g, (16, 4, 4), 0)
    with pytest.raises(htr.HTRError, match="UNSUPPORTED"):
        htr.htr_autotune(g, U, T, g.new_work())
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.full((1,), 1e-9, dtype=torch.float64, device="cuda")
    with pytest.raises(htr.HTRError, match="UNSUPPORTED"):
        htr.htr_rk3_step_taped(g, U, T, t, dt, 0, None, None, g.new_work(), None, htr.new_tape(g))
    # a folded grid: det(d x / d xi) < 0 somewhere
    bad = synth.wavy_grid(case.grid.n, 1e-4, amp=3.0, seed=4)
    with pytest.raises(htr.HTRError, match="EINVAL"):
        htr.Context.from_case(synth.Case("bad", case.mech, bad, case.Y, case.T, case.p, case.vel))
