"""Pins of the oracle's TENO6 reconstruction against definitions derived here
independently (sympy): candidate stencils and smoothness indicators as the
Jiang-Shu integrals of interpolating polynomials, the sixth-order
scale-separation measure, and the ENO cut-off on discontinuities.
Scheme: TENO6 (Fu et al. 2016), cited by the paper in Methods › Numerical method."""
import numpy as np
import pytest
import sympy as sp

from oracle.oracle import teno6, teno6_detail

X = sp.symbols("x")
F = sp.symbols("f0:6")          # cell averages at i-2..i+3


def _poly(nodes):
    n = len(nodes)
    a = sp.symbols("a0:%d" % n)
    p = sum(a[k] * X ** k for k in range(n))
    eqs = [sp.integrate(p, (X, j - sp.Rational(1, 2), j + sp.Rational(1, 2))) - F[j + 2] for j in nodes]
    return sp.expand(p.subs(sp.solve(eqs, a)))


def _beta(p, n):
    h = sp.Rational(1, 2)
    return sp.expand(sum(sp.integrate(sp.diff(p, X, l) ** 2, (X, -h, h)) for l in range(1, n)))


@pytest.fixture(scope="module")
def sym():
    st = {0: [-1, 0, 1], 1: [0, 1, 2], 2: [-2, -1, 0], 3: [0, 1, 2, 3]}
    P = {k: _poly(v) for k, v in st.items()}
    P6 = _poly([-2, -1, 0, 1, 2, 3])
    Bx = {k: _beta(P[k], len(st[k])) for k in st}
    B6x = _beta(P6, 6)
    B = {k: sp.lambdify(F, Bx[k]) for k in st}
    B6 = sp.lambdify(F, B6x)
    Q = {k: sp.lambdify(F, P[k].subs(X, sp.Rational(1, 2))) for k in st}
    Q6 = P6.subs(X, sp.Rational(1, 2))
    return dict(B=B, B6=B6, Q=Q, Q6=Q6, Bx=Bx, B6x=B6x)


def test_linear_weights_give_central6(sym):
    """d = (9/20, 3/10, 1/20, 1/5) combine the candidates into the six-point
    central interpolation (1, -8, 37, 37, -8, 1)/60."""
    d = [sp.Rational(9, 20), sp.Rational(3, 10), sp.Rational(1, 20), sp.Rational(1, 5)]
    st = {0: [-1, 0, 1], 1: [0, 1, 2], 2: [-2, -1, 0], 3: [0, 1, 2, 3]}
    comb = sum(d[k] * _poly(st[k]).subs(X, sp.Rational(1, 2)) for k in range(4))
    assert sp.simplify(comb - sym["Q6"]) == 0
    coeffs = [sym["Q6"].coeff(F[i]) for i in range(6)]
    assert coeffs == [sp.Rational(c, 60) for c in (1, -8, 37, 37, -8, 1)]


def test_smoothness_indicators_match_definition(sym):
    rng = np.random.default_rng(0)
    for _ in range(50):
        f = rng.normal(size=6) * 10 ** rng.uniform(-3, 3)
        _, det = teno6_detail(f)
        for k in range(4):
            ref = sym["B"][k](*f)
            assert abs(det["beta"][k] - ref) <= 1e-12 * max(abs(ref), 1e-300) + 1e-300
        ref6 = sym["B6"](*f)
        assert abs(det["beta6"] - ref6) <= 1e-11 * abs(ref6)


def test_smoothness_indicators_of_nearly_uniform_data(sym):
    """Data that varies by 1e-9 of its size: the indicators (~1e-18 f^2)
    keep their relative accuracy against the exact value of the definition
    at the same (exactly represented) data, because they are formed from the
    differences of the stencil values, which are exact here.  Sums of
    multiples of the values themselves (-11 f_i + 18 f_{i+1} - ...) carry the
    rounding of those products: 1e-8 to 1e-6 of the four-point indicator and
    of beta6 on this data."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        f = 1.0 + 1e-9 * rng.normal(size=6)
        _, det = teno6_detail(f)
        exact = {F[i]: sp.Rational(float(f[i])) for i in range(6)}
        for k in range(4):
            ref = float(sym["Bx"][k].subs(exact))
            assert abs(det["beta"][k] - ref) <= 1e-12 * ref, (k, det["beta"][k], ref)
        ref6 = float(sym["B6x"].subs(exact))
        assert abs(det["beta6"] - ref6) <= 1e-12 * ref6


def test_smooth_data_uses_all_stencils_and_is_sixth_order(sym):
    """On smooth data every candidate survives the cut-off, the result is the
    central six-point value, and tau (the global smoothness measure) scales
    as h^6 while the candidate betas scale as h^2."""
    taus, betas, errs = [], [], []
    for h in (0.2, 0.1, 0.05):
        x0 = 0.37
        # cell averages of sin over cells of width h centred at (j + 1/2... ) x0 + j h
        f = np.array([(np.cos(x0 + (j - 0.5) * h) - np.cos(x0 + (j + 0.5) * h)) / h for j in range(-2, 4)])
        v, det = teno6_detail(f)
        assert np.allclose(det["omega"], [9 / 20, 3 / 10, 1 / 20, 1 / 5], rtol=0, atol=1e-15)
        taus.append(det["tau"])
        betas.append(det["beta"][0])
        errs.append(abs(v - np.sin(x0 + 0.5 * h)))
    r_tau = np.log2(taus[0] / taus[1]), np.log2(taus[1] / taus[2])
    r_err = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert min(r_tau) > 5.6, r_tau
    assert min(r_err) > 5.6, r_err
    assert abs(np.log2(betas[0] / betas[1]) - 2) < 0.1


@pytest.mark.parametrize("f,expect", [
    ([0, 0, 0, 1, 1, 1], 0.0),      # jump between i and i+1: only the upwind stencil survives
    ([0, 0, 1, 1, 1, 1], 1.0),      # jump between i-1 and i: stencils right of i survive
    ([1, 1, 1, 1, 5, 5], 1.0),      # jump between i+1 and i+2: S0 and S2 survive
])
def test_cutoff_on_discontinuities(f, expect):
    v, det = teno6_detail(np.array(f, float))
    assert v == pytest.approx(expect, abs=1e-14)


def test_cutoff_selects_smooth_candidates_only():
    v, det = teno6_detail(np.array([1, 1, 1, 1, 5, 5], float))
    assert list(det["omega"] > 0) == [True, False, True, False]
    v, det = teno6_detail(np.array([0, 0, 1, 1, 1, 1], float))
    assert list(det["omega"] > 0) == [False, True, False, True]


def test_constant_and_linear_data_exact():
    assert teno6(np.full(6, 3.25)) == 3.25
    f = 2.0 + 0.5 * np.arange(-2, 4)          # cell averages of a linear function
    assert teno6(f) == pytest.approx(2.0 + 0.5 * 0.5, abs=1e-14)


def test_no_overflow_for_large_jumps():
    v = teno6(np.array([0, 0, 0, 1e20, 1e20, 1e20]))
    assert np.isfinite(v) and v == 0.0
