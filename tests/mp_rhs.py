"""Straight-line 40-digit evaluation of the whole right-hand side on tiny
periodic grids (mpmath), written from the paper's governing equations and
the readings the oracle follows, for the brute-force pin of the oracle.

Paper: Methods › Solver, eqs. (1)-(6) (conserved variables, fluxes, the
ideal-gas closure, Wilke viscosity, NASA polynomials, the heat flux with
species enthalpy transport, mixture-averaged diffusion with a correction
velocity, finite-rate reversible Arrhenius chemistry); Methods › Numerical
method (conservative finite differences, the six-point central flux or TENO6
on a local Lax-Friedrichs split, second-order diffusive fluxes); the laser
kernel of Methods › Diffusion flame › Physical model and numerical setup.

Everything is evaluated here in 40 significant digits, cell by cell and face
by face, with no code shared with the oracle: the temperature by Newton's
method to full precision, NASA-7 thermodynamics, Chapman-Enskog species
viscosities and binary diffusivities (Neufeld-Janzen-Aziz collision
integrals), Eucken conductivities, Wilke mixing, Bird mixture diffusivities,
the Arrhenius rates with K_c from the Gibbs energies, the laser Gaussian
summed over periodic images, the dilatation sensor, the node and face
fluxes.  Only the one-face TENO6 reconstruction (six numbers in, one out,
pinned on its own against its definition) is taken from the oracle, in
double precision, as in the convective brute force."""
import mpmath as mp
import numpy as np

import oracle.oracle as oo
import synth

DPS = 40
CC = (1, -8, 37, 37, -8, 1)


def _m(x):
    return mp.mpf(float(x))


def rhs(case, U, t=0.0, flags=None):
    """dU/dt [nv][N] and HRR [N] of the case's state U (floats)."""
    mp.mp.dps = DPS
    flags = case.flags if flags is None else flags
    mech, g = case.mech, case.grid
    ns, nr = mech.ns, mech.nr
    nv = ns + 4
    n = g.n
    N = g.N
    kB = mp.mpf("1.380649e-23")
    NA = mp.mpf("6.02214076e23")
    Ru = kB * NA
    P0 = mp.mpf(101325)
    pi = mp.pi
    W = [_m(w) for w in mech.W]
    a7 = [[_m(v) for v in mech.nasa7[s]] for s in range(ns)]
    sig = [_m(v) for v in mech.lj_sigma]
    epk = [_m(v) for v in mech.lj_epsk]
    Um = [[_m(U[v, q]) for q in range(N)] for v in range(nv)]

    def idx(i, j, k):
        return ((k % n[2]) * n[1] + (j % n[1])) * n[0] + (i % n[0])

    def coords(q):
        return q % n[0], (q // n[0]) % n[1], q // (n[0] * n[1])

    # --- thermodynamics of one species (NASA-7)
    def cpR(s, T):
        a = a7[s]
        return a[0] + a[1] * T + a[2] * T ** 2 + a[3] * T ** 3 + a[4] * T ** 4

    def hRT(s, T):
        a = a7[s]
        return a[0] + a[1] * T / 2 + a[2] * T ** 2 / 3 + a[3] * T ** 3 / 4 + a[4] * T ** 4 / 5 + a[5] / T

    def sR(s, T):
        a = a7[s]
        return a[0] * mp.log(T) + a[1] * T + a[2] * T ** 2 / 2 + a[3] * T ** 3 / 3 + a[4] * T ** 4 / 4 + a[6]

    def om22(x):
        return (mp.mpf("1.16145") * x ** mp.mpf("-0.14874") + mp.mpf("0.52487") * mp.exp(mp.mpf("-0.77320") * x)
                + mp.mpf("2.16178") * mp.exp(mp.mpf("-2.43787") * x))

    def om11(x):
        return (mp.mpf("1.06036") * x ** mp.mpf("-0.15610") + mp.mpf("0.19300") * mp.exp(mp.mpf("-0.47635") * x)
                + mp.mpf("1.03587") * mp.exp(mp.mpf("-1.52996") * x)
                + mp.mpf("1.76474") * mp.exp(mp.mpf("-3.89411") * x))

    # --- per cell
    cell = []
    for q in range(N):
        rs = [Um[s][q] for s in range(ns)]
        rho = sum(rs)
        Y = [r / rho for r in rs]
        u = [Um[ns + m][q] / rho for m in range(3)]
        e = Um[ns + 3][q] / rho - (u[0] ** 2 + u[1] ** 2 + u[2] ** 2) / 2
        # e(T) = sum_s Y_s (h_s - R_s T); Newton to full precision
        T = _m(case.T[q])
        for _ in range(200):
            eT = sum(Y[s] * Ru / W[s] * T * (hRT(s, T) - 1) for s in range(ns))
            cv = sum(Y[s] * Ru / W[s] * (cpR(s, T) - 1) for s in range(ns))
            dT = (eT - e) / cv
            T -= dT
            if abs(dT) < mp.mpf(10) ** (-DPS + 5) * T:
                break
        else:
            raise RuntimeError("Newton did not converge")
        Wm = 1 / sum(Y[s] / W[s] for s in range(ns))
        p = rho * Ru * T / Wm
        X = [Y[s] * Wm / W[s] for s in range(ns)]
        h = [Ru / W[s] * T * hRT(s, T) for s in range(ns)]
        cps = [Ru / W[s] * cpR(s, T) for s in range(ns)]
        cp = sum(Y[s] * cps[s] for s in range(ns))
        c = mp.sqrt(cp / (cp - Ru / Wm) * p / rho)
        # transport
        mus = [mp.mpf(5) / 16 * mp.sqrt(pi * (W[s] / NA) * kB * T) / (pi * sig[s] ** 2 * om22(T / epk[s]))
               for s in range(ns)]
        lams = [mus[s] * (cps[s] + mp.mpf(5) / 4 * Ru / W[s]) for s in range(ns)]
        phi = [[(1 + mp.sqrt(mus[i] / mus[j]) * (W[j] / W[i]) ** mp.mpf("0.25")) ** 2
                / mp.sqrt(8 * (1 + W[i] / W[j])) for j in range(ns)] for i in range(ns)]
        mu = sum(X[i] * mus[i] / sum(X[j] * phi[i][j] for j in range(ns)) for i in range(ns))
        lam = sum(X[i] * lams[i] / sum(X[j] * phi[i][j] for j in range(ns)) for i in range(ns))

        def Dbin(i, j):
            mij = 1 / (NA * (1 / W[i] + 1 / W[j]))
            sg = (sig[i] + sig[j]) / 2
            ek = mp.sqrt(epk[i] * epk[j])
            return mp.mpf(3) / 16 * mp.sqrt(2 * pi * (kB * T) ** 3 / mij) / (p * pi * sg ** 2 * om11(T / ek))
        D = []
        for s in range(ns):
            den = sum(max(X[j], 0) / Dbin(s, j) for j in range(ns) if j != s)
            D.append(Dbin(s, s) if den < mp.mpf("1e-300") else (1 - Y[s]) / den)
        # chemistry
        wdot = [mp.mpf(0)] * ns
        if not (flags & synth.CHEM_OFF):
            conc = [rs[s] / W[s] for s in range(ns)]
            G = [hRT(s, T) - sR(s, T) for s in range(ns)]
            for j in range(nr):
                nuf = [int(v) for v in mech.nu_f[j]]
                nub = [int(v) for v in mech.nu_r[j]]
                nu = [nub[s] - nuf[s] for s in range(ns)]
                lnkf = _m(mech.lnA[j]) + _m(mech.beta[j]) * mp.log(T) - _m(mech.Ea[j]) / (Ru * T)
                lnKc = -sum(nu[s] * G[s] for s in range(ns)) + sum(nu) * mp.log(P0 / (Ru * T))
                kf = mp.exp(lnkf)
                kb = mp.exp(lnkf - lnKc)
                qj = kf * mp.fprod([conc[s] ** nuf[s] for s in range(ns)]) \
                    - kb * mp.fprod([conc[s] ** nub[s] for s in range(ns)])
                for s in range(ns):
                    wdot[s] += W[s] * nu[s] * qj
        hrr = -sum(h[s] * wdot[s] for s in range(ns))
        # laser: Gaussian in space over all periodic images, Gaussian in time
        qL = mp.mpf(0)
        las = case.laser
        if las.on:
            i, j, k = coords(q)
            dim = sum(1 for a in range(3) if n[a] > 1)
            sr, st = _m(las.sigma_r), _m(las.sigma_t)
            val = _m(las.E) / ((2 * pi) ** (mp.mpf(dim + 1) / 2) * sr ** dim * st)
            for a, ia in enumerate((i, j, k)):
                if n[a] == 1:
                    continue
                La = _m(g.L[a])
                r = _m(g.xnode[a][ia]) - _m(las.center[a])
                K = int(np.ceil(12 * float(las.sigma_r) / float(g.L[a]))) + 3
                val *= sum(mp.exp(-((r - m * La) / sr) ** 2 / 2) for m in range(-K, K + 1))
            qL = val * mp.exp(-((_m(t) - _m(las.t0)) / st) ** 2 / 2)
        cell.append(dict(rho=rho, Y=Y, u=u, T=T, p=p, c=c, W=Wm, X=X, h=h, mu=mu, lam=lam, D=D, wdot=wdot,
                         hrr=hrr, qL=qL))

    xin = [[_m(v) for v in g.xin[a]] for a in range(3)]
    xif = [[_m(v) for v in g.xif[a]] for a in range(3)]

    # --- sensor at nodes: theta = div^2 / (div^2 + |curl|^2 + 1e-300)
    def node_grad(q):
        i, j, k = coords(q)
        gr = [[mp.mpf(0)] * 3 for _ in range(3)]
        for a in range(3):
            if n[a] == 1:
                continue
            off = [0, 0, 0]
            off[a] = 1
            qp, qm = idx(i + off[0], j + off[1], k + off[2]), idx(i - off[0], j - off[1], k - off[2])
            for m in range(3):
                gr[a][m] = xin[a][(i, j, k)[a]] * (cell[qp]["u"][m] - cell[qm]["u"][m]) / 2
        return gr
    theta = []
    for q in range(N):
        gr = node_grad(q)
        div = gr[0][0] + gr[1][1] + gr[2][2]
        w2 = (gr[1][2] - gr[2][1]) ** 2 + (gr[2][0] - gr[0][2]) ** 2 + (gr[0][1] - gr[1][0]) ** 2
        theta.append(div ** 2 / (div ** 2 + w2 + mp.mpf("1e-300")))

    def nflux(q, v, d):
        z = cell[q]
        un = z["u"][d]
        if v < ns:
            return Um[v][q] * un
        if v < ns + 3:
            return Um[v][q] * un + (z["p"] if v - ns == d else 0)
        return (Um[v][q] + z["p"]) * un

    out = [[mp.mpf(0)] * N for _ in range(nv)]
    for q in range(N):
        z = cell[q]
        if not (flags & synth.CHEM_OFF):
            for s in range(ns):
                out[s][q] += z["wdot"][s]
        out[ns + 3][q] += z["qL"]
    for d in range(3):
        if n[d] == 1:
            continue
        off = [0, 0, 0]
        off[d] = 1
        Fc = [None] * N
        Fd = [None] * N
        for q in range(N):
            i, j, k = coords(q)
            st = [idx(i + (m - 2) * off[0], j + (m - 2) * off[1], k + (m - 2) * off[2]) for m in range(6)]
            # convective face flux (hybrid switch: sensor anywhere on the stencil, or a pressure jump)
            if flags & synth.FORCE_TENO:
                teno = True
            elif flags & synth.FORCE_CENTRAL:
                teno = False
            else:
                pa, pb = cell[st[2]]["p"], cell[st[3]]["p"]
                teno = max(theta[s] for s in st) > case.theta_c or abs(pb - pa) / min(pa, pb) > case.psi_c
            if not teno:
                Fc[q] = [sum(CC[m] * nflux(st[m], v, d) for m in range(6)) / 60 for v in range(nv)]
            else:
                alpha = max(abs(cell[s]["u"][d]) + cell[s]["c"] for s in st)
                Fc[q] = []
                for v in range(nv):
                    fp = [(nflux(st[m], v, d) + alpha * Um[v][st[m]]) / 2 for m in range(6)]
                    fm = [(nflux(st[5 - m], v, d) - alpha * Um[v][st[5 - m]]) / 2 for m in range(6)]
                    Fc[q].append(_m(oo.teno6(np.array([float(x) for x in fp]), case.teno_CT))
                                 + _m(oo.teno6(np.array([float(x) for x in fm]), case.teno_CT)))
            if flags & synth.VISC_OFF:
                Fd[q] = [mp.mpf(0)] * nv
                continue
            # diffusive face flux between A = node (i,j,k) and B = its neighbour along d
            A, B = cell[q], cell[st[3]]
            qA, qB = q, st[3]
            xf = xif[d][(i, j, k)[d]]
            grd = [[mp.mpf(0)] * 3 for _ in range(3)]   # grd[a][m] = d u_m / d x_a at the face
            for m in range(3):
                grd[d][m] = xf * (B["u"][m] - A["u"][m])
            for a in range(3):
                if a == d or n[a] == 1:
                    continue
                for qs in (qA, qB):
                    gs = node_grad(qs)
                    for m in range(3):
                        grd[a][m] += gs[a][m] / 2
            mu = (A["mu"] + B["mu"]) / 2
            lam = (A["lam"] + B["lam"]) / 2
            rho = (A["rho"] + B["rho"]) / 2
            Wf = (A["W"] + B["W"]) / 2
            div = grd[0][0] + grd[1][1] + grd[2][2]
            tau = [mu * (grd[d][m] + grd[m][d]) - (mp.mpf(2) / 3 * mu * div if m == d else 0) for m in range(3)]
            # J_s = -rho D_s (W_s/W) dX_s/dn + Y_s sum_j rho D_j (W_j/W) dX_j/dn  (sum_s J_s = 0)
            jd = [rho * (A["D"][s] + B["D"][s]) / 2 * (W[s] / Wf) * xf * (B["X"][s] - A["X"][s]) for s in range(ns)]
            corr = sum(jd)
            J = [-jd[s] + (A["Y"][s] + B["Y"][s]) / 2 * corr for s in range(ns)]
            qn = -lam * xf * (B["T"] - A["T"]) + sum(J[s] * (A["h"][s] + B["h"][s]) / 2 for s in range(ns))
            work = sum(tau[m] * (A["u"][m] + B["u"][m]) / 2 for m in range(3))
            Fd[q] = [-J[s] for s in range(ns)] + tau + [work - qn]
        for q in range(N):
            i, j, k = coords(q)
            qm = idx(i - off[0], j - off[1], k - off[2])
            xi = xin[d][(i, j, k)[d]]
            for v in range(nv):
                out[v][q] += xi * ((Fd[q][v] - Fd[qm][v]) - (Fc[q][v] - Fc[qm][v]))
    dUdt = np.array([[float(out[v][q]) for q in range(N)] for v in range(nv)])
    hrr = np.array([float(cell[q]["hrr"]) for q in range(N)])
    return dUdt, hrr
