"""Brute force: the convective right-hand side of tiny periodic grids
written out straight-line in 40-digit arithmetic (mpmath), apart from the
oracle's assembly, and compared with the oracle (Methods › Numerical method: conservative
finite differences; the central six-point flux, or TENO6 / WENO3-Z on a
local Lax-Friedrichs split; the hybrid switch).

Recomputed here:
- the primitives of a calorically perfect gas;
- the dilatation sensor and the pressure-jump switch;
- the node fluxes and the splitting speed;
- the mirrored minus-side stencil;
- the face difference and the metric.

Only the one-face reconstructions come from the oracle: TENO6 and WENO3-Z
of six values, pinned on their own in the TENO and WENO tests.  One
calorically perfect species, no chemistry, no viscosity, on 1-D, 2-D and
3-D grids, uniform and stretched, with a jump so that cut-offs occur."""
import mpmath as mp
import numpy as np
import pytest

import oracle.oracle as oo
import synth
from oracle import Oracle

RU = 8.31446261815324
CC = (1, -8, 37, 37, -8, 1)


def _state(g, seed):
    """rho, u (3 components) and p per node, smooth plus a jump in x."""
    rng = np.random.default_rng(seed)
    x, y, z = g.mesh()
    Lx = g.L[0]
    ph = rng.uniform(0, 2 * np.pi, 6)
    jump = np.where((x > 0.3 * Lx) & (x < 0.6 * Lx), 1.0, 0.0)
    rho = (1.0 + 0.2 * np.sin(2 * np.pi * x / Lx + ph[0]) + 0.5 * jump).ravel()
    p = (1e5 * (1 + 0.1 * np.cos(2 * np.pi * y / g.L[1] + ph[1]) + 0.8 * jump)).ravel()
    vel = np.stack([30 * np.sin(2 * np.pi * x / Lx + ph[2]), 20 * np.cos(2 * np.pi * y / g.L[1] + ph[3]),
                    10 * np.sin(2 * np.pi * z / g.L[2] + ph[4])]).reshape(3, -1)
    for a in range(3):
        if g.n[a] == 1:
            vel[a] = 0.0
    return rho, vel, p


def brute_rhs(U, g, flags, W, cpR, theta_c, psi_c, CT):
    """dU/dt of the convective terms, U [5][N] (rho, rho u, rho v, rho w, E)."""
    mp.mp.dps = 40
    n = g.n
    N = g.N
    R = mp.mpf(RU) / mp.mpf(W)
    cv = (mp.mpf(cpR) - 1) * R
    gam = mp.mpf(cpR) / (mp.mpf(cpR) - 1)
    Um = [[mp.mpf(float(U[v, q])) for q in range(N)] for v in range(5)]

    def idx(i, j, k):
        return ((k % n[2]) * n[1] + (j % n[1])) * n[0] + (i % n[0])
    rho = Um[0]
    u = [[Um[1 + a][q] / rho[q] for q in range(N)] for a in range(3)]
    # e = E/rho - |u|^2/2 = c_v T for this gas (h = c_p T, no formation enthalpy)
    T = [(Um[4][q] / rho[q] - (u[0][q] ** 2 + u[1][q] ** 2 + u[2][q] ** 2) / 2) / cv for q in range(N)]
    p = [rho[q] * R * T[q] for q in range(N)]
    c = [mp.sqrt(gam * R * T[q]) for q in range(N)]
    xin = [[mp.mpf(float(v)) for v in g.xin[a]] for a in range(3)]
    # sensor: theta = div^2 / (div^2 + |curl|^2 + 1e-300), central differences
    theta = [0.0] * N
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                q = idx(i, j, k)
                gr = [[mp.mpf(0)] * 3 for _ in range(3)]
                for a in range(3):
                    if n[a] == 1:
                        continue
                    off = [0, 0, 0]
                    off[a] = 1
                    qp = idx(i + off[0], j + off[1], k + off[2])
                    qm = idx(i - off[0], j - off[1], k - off[2])
                    ca = (i, j, k)[a]
                    for m in range(3):
                        gr[a][m] = xin[a][ca] * (u[m][qp] - u[m][qm]) / 2
                div = gr[0][0] + gr[1][1] + gr[2][2]
                w2 = (gr[1][2] - gr[2][1]) ** 2 + (gr[2][0] - gr[0][2]) ** 2 + (gr[0][1] - gr[1][0]) ** 2
                theta[q] = float(div ** 2 / (div ** 2 + w2 + mp.mpf("1e-300")))

    def flux(q, v, a):
        un = u[a][q]
        if v == 0:
            return Um[0][q] * un
        if v <= 3:
            return Um[v][q] * un + (p[q] if v - 1 == a else 0)
        return (Um[4][q] + p[q]) * un
    out = [[mp.mpf(0)] * N for _ in range(5)]
    for a in range(3):
        if n[a] == 1:
            continue
        off = [0, 0, 0]
        off[a] = 1
        Fh = [[None] * N for _ in range(5)]   # face i+1/2 along a, stored at node i
        for k in range(n[2]):
            for j in range(n[1]):
                for i in range(n[0]):
                    q = idx(i, j, k)
                    st = [idx(i + (m - 2) * off[0], j + (m - 2) * off[1], k + (m - 2) * off[2]) for m in range(6)]
                    if flags & synth.FORCE_TENO:
                        teno = True
                    elif flags & synth.FORCE_CENTRAL:
                        teno = False
                    else:
                        psi = abs(p[st[3]] - p[st[2]]) / min(p[st[2]], p[st[3]])
                        teno = max(theta[s] for s in st) > theta_c or psi > psi_c
                    if not teno:
                        for v in range(5):
                            Fh[v][q] = sum(CC[m] * flux(st[m], v, a) for m in range(6)) / 60
                        continue
                    alpha = max(abs(u[a][s]) + c[s] for s in st)
                    for v in range(5):
                        fp = [(flux(st[m], v, a) + alpha * Um[v][st[m]]) / 2 for m in range(6)]
                        fm = [(flux(st[5 - m], v, a) - alpha * Um[v][st[5 - m]]) / 2 for m in range(6)]
                        rec = oo.weno3z if flags & synth.WENO3Z else (lambda f: oo.teno6(f, CT))
                        Fh[v][q] = mp.mpf(rec(np.array([float(t) for t in fp]))) + \
                            mp.mpf(rec(np.array([float(t) for t in fm])))
        for k in range(n[2]):
            for j in range(n[1]):
                for i in range(n[0]):
                    q = idx(i, j, k)
                    qm = idx(i - off[0], j - off[1], k - off[2])
                    ca = (i, j, k)[a]
                    for v in range(5):
                        out[v][q] -= xin[a][ca] * (Fh[v][q] - Fh[v][qm])
    return np.array([[float(out[v][q]) for q in range(N)] for v in range(5)])


@pytest.mark.parametrize("flags", [synth.FORCE_CENTRAL, synth.FORCE_TENO, synth.FORCE_TENO | synth.WENO3Z, 0])
@pytest.mark.parametrize("n,stretched", [((7, 1, 1), False), ((9, 1, 1), True), ((6, 5, 1), True),
                                         ((4, 3, 5), True)])
def test_convective_rhs_brute_force(n, stretched, flags):
    W, cpR = 0.029, 3.5
    mech = synth.single_species(W, cpR)
    g = synth.stretched_grid(n, 1e-4, amp=0.2) if stretched else synth.uniform_grid(n, 1e-4)
    rho, vel, p = _state(g, seed=sum(n) + flags)
    T = p / (rho * RU / W)
    case = synth.Case("bf", mech, g, np.ones((1, g.N)), T, p, vel,
                      flags=flags | synth.CHEM_OFF | synth.VISC_OFF)
    o = Oracle(case)
    U = o.prim_to_cons()
    ref = o.rhs(U, T.copy())
    bf = brute_rhs(U, g, flags, W, cpR, case.theta_c, case.psi_c, case.teno_CT)
    scale = np.abs(bf).max(axis=1)
    scale[scale == 0] = 1.0
    err = np.abs(ref - bf).max(axis=1) / scale
    assert err.max() < 1e-12, err
