"""Pins of the oracle's per-cell physics (paper Methods › Solver): NASA thermo
identities, the ideal-gas closure (eq. 4), Chapman-Enskog transport against
the practical-unit textbook formulas, Wilke/Eucken special cases, mass and
element conservation of the chemistry, detailed balance at equilibrium, and
the laser kernel normalisation (eq. laser-qs)."""
import numpy as np
import pytest

import synth
from oracle import Oracle
from conftest import golden
from oracle.oracle import omega11, omega22

RU = 8.31446261815324


def one_cell_case(mech, T=1500.0, p=101325.0, Y=None, vel=(0.0, 0.0, 0.0), dx=1e-4):
    g = synth.uniform_grid((1, 1, 1), dx)
    Y = np.full(mech.ns, 1.0 / mech.ns) if Y is None else np.asarray(Y, float)
    return synth.Case("cell", mech, g, Y[:, None].copy(), np.array([T]), np.array([p]),
                      np.array(vel, float)[:, None].copy())


# ----------------------------------------------------------------- thermo
def test_thermo_identities():
    """c_p = d h / dT and c_p / T = d s / dT (molar, divided by R)."""
    mech = synth.make_mechanism(9, 20, 7)
    o = Oracle(one_cell_case(mech))
    for s in range(mech.ns):
        for T in (300.0, 1234.5, 4000.0):
            h = 1e-3 * T
            # Richardson-extrapolated central differences of T*h/RT and s/R
            def d(fun):
                d1 = (fun(T + h) - fun(T - h)) / (2 * h)
                d2 = (fun(T + h / 2) - fun(T - h / 2)) / h
                return (4 * d2 - d1) / 3
            cp = o.thermo(s, T)[0]
            dh = d(lambda t: t * o.thermo(s, t)[1])
            ds = d(lambda t: o.thermo(s, t)[2])
            assert dh == pytest.approx(cp, rel=1e-9)
            assert ds == pytest.approx(cp / T, rel=1e-9)


def test_calorically_perfect_gas_closed_forms():
    """c_p/R = 7/2: gamma = 7/5, c = sqrt(1.4 R T / W), e = (5/2) R T / W."""
    W = 0.028
    mech = synth.single_species(W, 3.5)
    T, p, u = 700.0, 2.0e5, (30.0, -20.0, 10.0)
    case = one_cell_case(mech, T=T, p=p, Y=[1.0], vel=u)
    case.flags = synth.CHEM_OFF
    o = Oracle(case)
    U = o.prim_to_cons()
    rho = p * W / (RU * T)
    assert U[0, 0] == pytest.approx(rho, rel=1e-15)
    ke = 0.5 * rho * sum(v * v for v in u)
    assert U[4, 0] == pytest.approx(rho * 2.5 * RU / W * T + ke, rel=1e-14)
    cells = o.cells(U, np.array([300.0]))
    assert cells[0, 0] == pytest.approx(T, rel=1e-13)                     # Newton recovers T
    assert cells[1, 0] == pytest.approx(p, rel=1e-13)                     # eq. (4)
    assert cells[2, 0] == pytest.approx(np.sqrt(1.4 * RU * T / W), rel=1e-13)


def test_newton_round_trip_and_guess_independence():
    mech = synth.make_mechanism(9, 20, 3)
    case = synth.small_case(n=(6, 5, 4), ns=4, nr=3)
    o = Oracle(case)
    U = o.prim_to_cons()
    for guess in (300.0, 1500.0, 3000.0):
        c = o.cells(U, np.full(case.grid.N, guess))
        assert np.max(np.abs(c[0] - case.T) / case.T) < 1e-13
    del mech


# --------------------------------------------------------------- transport
def test_collision_integral_fits_against_table():
    """Neufeld-Janzen-Aziz fits against the Hirschfelder-Curtiss-Bird table
    (Lennard-Jones 12-6; tests/golden/collision_integrals.csv): Omega(2,2)*
    and Omega(1,1)* within the fits' 0.2%."""
    rows = golden("collision_integrals.csv")
    assert len(rows) >= 4
    for Ts, o22, o11 in rows:
        assert omega22(float(Ts)) == pytest.approx(float(o22), rel=2e-3), Ts
        assert omega11(float(Ts)) == pytest.approx(float(o11), rel=2e-3), Ts


def _two_species(W1, W2, s1, s2, e1, e2, cp1=3.5, cp2=3.5):
    m1 = synth.single_species(W1, cp1, sigma=s1, epsk=e1)
    m2 = synth.single_species(W2, cp2, sigma=s2, epsk=e2)
    mech = synth.Mechanism(
        names=["A", "B"], elem=np.zeros((3, 2), np.int32), W=np.array([W1, W2]),
        nasa7=np.vstack([m1.nasa7, m2.nasa7]), lj_sigma=np.array([s1, s2]), lj_epsk=np.array([e1, e2]),
        lnA=np.zeros(0), beta=np.zeros(0), Ea=np.zeros(0), nu_f=np.zeros((0, 2), np.int32),
        nu_r=np.zeros((0, 2), np.int32))
    return mech


def test_viscosity_and_binary_diffusion_practical_units():
    """Chapman-Enskog viscosity, eta[uP] = 26.69 sqrt(M T)/(sigma^2 Omega_v),
    and binary diffusion, D[cm^2/s] = 0.00266 T^1.5/(P[bar] M_AB^0.5 sigma^2
    Omega_D), M_AB = 2/(1/M_A + 1/M_B) (practical-unit forms, Poling et al.)."""
    mech = _two_species(0.028014, 0.031999, 3.798e-10, 3.467e-10, 71.4, 106.7)
    o = Oracle(one_cell_case(mech, T=300.0))
    for s, (M, sg, ek) in enumerate([(28.014, 3.798, 71.4), (31.999, 3.467, 106.7)]):
        for T in (300.0, 1000.0):
            eta = 26.69 * np.sqrt(M * T) / (sg ** 2 * omega22(T / ek)) * 1e-7
            assert o.mu_species(s, T) == pytest.approx(eta, rel=5e-4)   # 26.69 is rounded (26.696)
    for T, P in ((300.0, 101325.0), (1200.0, 5e5)):
        MAB = 2.0 / (1 / 28.014 + 1 / 31.999)
        sg = 0.5 * (3.798 + 3.467)
        ek = np.sqrt(71.4 * 106.7)
        D = 0.00266 * T ** 1.5 / (P / 1e5 * np.sqrt(MAB) * sg ** 2 * omega11(T / ek)) * 1e-4
        assert o.D_binary(0, 1, T, P) == pytest.approx(D, rel=2e-3)
    # order of magnitude against the measured N2-O2 value at 1 atm, ~293 K: 0.20 cm^2/s
    assert o.D_binary(0, 1, 293.0, 101325.0) == pytest.approx(2.0e-5, rel=0.1)
    assert o.mu_species(0, 300.0) == pytest.approx(1.78e-5, rel=0.03)    # N2, measured


def _cells(mech, T, p, Y):
    o = Oracle(one_cell_case(mech, T=T, p=p, Y=Y))
    U = o.prim_to_cons()
    c = o.cells(U, np.array([T]))
    ns = mech.ns
    return dict(T=c[0, 0], p=c[1, 0], c=c[2, 0], mu=c[3, 0], lam=c[4, 0], D=c[5:5 + ns, 0]), o


def test_wilke_identical_and_pure_species():
    # two copies of one molecule: the mixture viscosity equals the species value
    mech = _two_species(0.028, 0.028, 3.7e-10, 3.7e-10, 90.0, 90.0)
    for y in (0.1, 0.5, 0.93):
        c, o = _cells(mech, 800.0, 101325.0, [y, 1 - y])
        assert c["mu"] == pytest.approx(o.mu_species(0, 800.0), rel=1e-14)
    # a pure species inside a multicomponent table
    mech = synth.make_mechanism(5, 4, 9)
    Y = np.zeros(5)
    Y[2] = 1.0
    c, o = _cells(mech, 1100.0, 101325.0, Y)
    assert c["mu"] == pytest.approx(o.mu_species(2, 1100.0), rel=1e-14)


def test_eucken_reduces_to_monatomic_kinetic_theory():
    """For c_p = (5/2) R/W the Eucken conductivity is lambda = (15/4)(R/W) mu."""
    W = 0.039948
    mech = synth.single_species(W, 2.5, sigma=3.4e-10, epsk=120.0)
    c, o = _cells(mech, 600.0, 101325.0, [1.0])
    assert c["lam"] == pytest.approx(15.0 / 4.0 * RU / W * c["mu"], rel=1e-14)


def test_mixture_diffusivity_binary_and_blanc():
    """Binary mixture: D_1 = D_12 W_2 / W (so that J_1 = -rho D_12 grad Y_1);
    trace species: D_s -> 1 / sum_j X_j / D_sj (Blanc's law)."""
    mech = _two_species(0.004, 0.032, 2.6e-10, 3.5e-10, 10.0, 110.0, 2.5, 3.5)
    T, p = 900.0, 2e5
    for y1 in (0.05, 0.3, 0.8):
        c, o = _cells(mech, T, p, [y1, 1 - y1])
        W = 1 / (y1 / 0.004 + (1 - y1) / 0.032)
        D12 = o.D_binary(0, 1, T, p)
        assert c["D"][0] == pytest.approx(D12 * 0.032 / W, rel=1e-13)
        assert c["D"][1] == pytest.approx(D12 * 0.004 / W, rel=1e-13)
    mech = synth.make_mechanism(5, 4, 2)
    Y = np.array([1e-12, 0.3, 0.2, 0.25, 0.25])
    c, o = _cells(mech, T, p, Y)
    W = 1 / np.sum(Y / mech.W)
    X = Y * W / mech.W
    blanc = 1 / sum(X[j] / o.D_binary(0, j, T, p) for j in range(1, 5))
    assert c["D"][0] == pytest.approx(blanc, rel=1e-10)


# --------------------------------------------------------------- chemistry
def _wdot(o, U, T):
    ns = o.ns
    c = o.cells(U, T.copy())
    return c[5 + ns:5 + 2 * ns], c[5 + 2 * ns]


@pytest.mark.parametrize("seed,ns,nr", [(1, 5, 4), (2, 9, 20), (13, 6, 10)])
def test_chemistry_conserves_mass_and_elements(seed, ns, nr):
    case = synth.small_case(n=(5, 4, 3), ns=ns, nr=nr, seed=seed, T_base=1800.0)
    o = Oracle(case)
    U = o.prim_to_cons()
    w, _ = _wdot(o, U, case.T)
    scale = np.abs(w).sum(axis=0)
    assert np.all(scale > 0)
    assert np.max(np.abs(w.sum(axis=0)) / scale) < 1e-14
    elem = case.mech.elem
    moles = w / case.mech.W[:, None]
    for e in range(3):
        tot = (elem[e][:, None] * moles).sum(axis=0)
        ref = (elem[e][:, None] * np.abs(moles)).sum(axis=0)
        assert np.max(np.abs(tot) / np.maximum(ref, 1e-300)) < 1e-13


def test_detailed_balance_at_equilibrium():
    """At ln c_s = -g_s/(R T) + ln(p0/(R T)) + sum_e lambda_e a_es (any
    element potentials lambda_e) every element-balanced reaction has zero net
    rate: k_f prod c^nu' = k_b prod c^nu''."""
    mech = synth.make_mechanism(9, 20, 21)
    T = 1700.0
    o = Oracle(one_cell_case(mech, T=T))
    G = np.array([o.thermo(s, T)[1] - o.thermo(s, T)[2] for s in range(mech.ns)])
    lam = np.array([-6.0, -9.0, -3.0])
    lnc = -G + np.log(101325.0 / (RU * T)) + lam @ mech.elem
    c = np.exp(lnc)
    Y = c * mech.W / np.sum(c * mech.W)
    p = np.sum(c) * RU * T
    case = one_cell_case(mech, T=T, p=p, Y=Y)
    o = Oracle(case)
    U = o.prim_to_cons()
    w, _ = _wdot(o, U, np.array([T]))
    # reference magnitude: the forward production of the fastest species
    case2 = one_cell_case(mech, T=T, p=p, Y=np.where(np.arange(mech.ns) == 0, 0.5, 0.5 / (mech.ns - 1)))
    o2 = Oracle(case2)
    w2, _ = _wdot(o2, o2.prim_to_cons(), np.array([T]))
    rel = np.abs(w[:, 0]) / (np.abs(w2[:, 0]).max() + np.abs(w[:, 0]).max() * 0 + 1e-300)
    # compare with the unbalanced rates scaled to the same concentrations
    assert np.max(np.abs(w[:, 0])) < 1e-9 * np.max(np.abs(w2[:, 0])), rel


def test_rate_law_scalings():
    """Law of mass action and the Arrhenius form, as invariants: with no
    products present, scaling every concentration by s scales the net rate by
    s^order; shifting ln A_j by ln 2 doubles reaction j's contribution."""
    mech = synth.make_mechanism(4, 1, 31, inert_bath=False)
    order = int(mech.nu_f.sum())
    Y = np.where(mech.nu_f[0] > 0, 1.0, 0.0)
    Y = Y / Y.sum()
    T = 1500.0
    r = []
    for p in (1e5, 2e5):
        c, o = _cells(mech, T, p, Y)
        w, _ = _wdot(o, o.prim_to_cons(), np.array([T]))
        r.append(w[:, 0])
    assert np.allclose(r[1], r[0] * 2.0 ** order, rtol=1e-12, atol=0)
    case = one_cell_case(mech, T=T, p=1e5, Y=Y)
    o = Oracle(case)
    U = o.prim_to_cons()
    w0, _ = _wdot(o, U, np.array([T]))
    case.mech = synth.Mechanism(**{**mech.__dict__, "lnA": mech.lnA + np.log(2.0)})
    o2 = Oracle(case)
    w1, _ = _wdot(o2, U, np.array([T]))
    assert np.allclose(w1, 2 * w0, rtol=1e-13, atol=0)


def test_heat_release_sign_and_definition():
    """HRR = -sum_s h_s wdot_s: with the per-species enthalpies from the
    oracle's own thermo (pinned above)."""
    case = synth.small_case(n=(4, 3, 2), ns=5, nr=4, seed=3, T_base=1800.0)
    o = Oracle(case)
    U = o.prim_to_cons()
    c = o.cells(U, case.T.copy())
    ns = 5
    w = c[5 + ns:5 + 2 * ns]
    hrr = c[5 + 2 * ns]
    T = c[0]
    h = np.array([[o.thermo(s, Tq)[1] * RU / case.mech.W[s] * Tq for Tq in T] for s in range(ns)])
    assert np.allclose(hrr, -(h * w).sum(axis=0), rtol=1e-12, atol=1e-12 * np.abs(hrr).max())


# ------------------------------------------------------------------- laser
@pytest.mark.parametrize("n", [(64, 1, 1), (32, 24, 1), (16, 20, 12)])
def test_laser_space_integral(n):
    """The spatial integral of q_L equals E exp(-(t-t0)^2/(2 st^2))/(sqrt(2 pi) st)
    in any dimension (the paper's 2-D normalisation generalised), so the
    space-time integral is E."""
    dx = 1e-4
    case = synth.small_case(n=n, ns=2, nr=0, seed=4)
    case.laser = synth.Laser(E=2.5e-3, center=tuple(0.37 * L for L in case.grid.L), sigma_r=2.5 * dx, t0=1e-6,
                             sigma_t=3e-7, on=True)
    g = synth.uniform_grid(n, dx)
    case.grid = g
    case.laser.center = tuple(0.37 * L for L in g.L)
    o = Oracle(case)
    U = o.prim_to_cons()
    act = [a for a in range(3) if n[a] > 1]
    area = np.prod([dx for _ in act])
    for t in (1e-6, 1.3e-6):
        qL = o.cells(U, case.T.copy(), t=t)[5 + 2 * 2 + 1]
        tot = qL.sum() * area
        st = 3e-7
        ref = 2.5e-3 * np.exp(-0.5 * ((t - 1e-6) / st) ** 2) / (np.sqrt(2 * np.pi) * st)
        assert tot == pytest.approx(ref, rel=1e-12)
    # circular mean over the period = centre (exact for a wrapped Gaussian)
    qL = o.cells(U, case.T.copy(), t=1e-6)[5 + 2 * 2 + 1]
    for a in act:
        xs = g.mesh()[a].ravel()
        ang = np.angle((qL * np.exp(2j * np.pi * xs / g.L[a])).sum())
        assert (ang % (2 * np.pi)) * g.L[a] / (2 * np.pi) == pytest.approx(case.laser.center[a], rel=1e-12)
