"""Seeded synthetic workloads: grids, primitive initial fields, laser kernels
and ensemble tables.

The paper's applications (the 2-D diffusion flame of Application examples › Ignition of a diffusion flame and the model
combustor of Application examples › Ignition of a model combustor) need mechanisms, geometry and data that are not
available; these generators stand in for them with the shapes, sizes and
structure of the five benchmark workloads:

  C1  1-D periodic hot spot, 256 cells, 5 species / 4 reactions, 200 steps
  C2  3-D periodic Taylor-Green box, 128^3, 9 species / 20 reactions,
      1 RHS + 10 steps
  C3  3-D periodic double mixing layer with laser deposition, 256x128x128,
      9 / 20, 100 steps
  C4  64-member ensemble of C3-type boxes, N^3 with N in {32,40,...,96},
      perturbed deposition energy, kernel centre and ln A, 50 steps
  C5  64^3 mixing layer, 50 steps, checkpoints every 10 (adjoint)

Initial conditions are returned as primitive fields (Y_s, T, p, u); each side
(the oracle, the GPU library) converts them to conserved variables itself.
Velocity amplitudes use a nominal sound speed sqrt(1.4 R_u T / W); nothing
here evaluates the method's thermodynamics.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mechanism import Mechanism, make_mechanism, single_species

RU = 8.31446261815324
P_ATM = 101325.0

# scheme flags (bit values of the C interfaces)
CHEM_OFF, VISC_OFF, FORCE_CENTRAL, FORCE_TENO, WENO3Z = 1, 2, 4, 8, 16
BC_PERIODIC, BC_WALL, BC_INFLOW, BC_OUTFLOW = 0, 1, 2, 3


@dataclass
class Grid:
    n: tuple                      # (nx, ny, nz)
    xnode: list                   # three arrays of node coordinates
    xin: list                     # three arrays d(xi)/dx at nodes
    xif: list                     # three arrays d(xi)/dx at faces i+1/2
    L: tuple                      # periods

    @property
    def N(self):
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def uniform(self):
        return all(np.all(self.xin[a] == self.xin[a][0]) and np.all(self.xif[a] == self.xin[a][0])
                   for a in range(3))

    def spacing(self):
        return tuple(1.0 / self.xin[a][0] for a in range(3))

    def mesh(self):
        """Node coordinates broadcast to [nz][ny][nx]."""
        z, y, x = np.meshgrid(self.xnode[2], self.xnode[1], self.xnode[0], indexing="ij")
        return x, y, z


def uniform_grid(n, d) -> Grid:
    n = tuple(int(v) for v in n)
    d = tuple(float(v) for v in (d if np.ndim(d) else (d, d, d)))
    xnode = [(np.arange(n[a]) + 0.5) * d[a] for a in range(3)]
    xin = [np.full(n[a], 1.0 / d[a]) for a in range(3)]
    return Grid(n=n, xnode=xnode, xin=xin, xif=[v.copy() for v in xin], L=tuple(n[a] * d[a] for a in range(3)))


def stretched_grid(n, d, amp=0.2) -> Grid:
    """Periodic rectilinear grid x(xi) = d (xi + amp n/(2 pi) sin(2 pi xi/n))
    along every axis with n > 1 (xi integer at nodes, half-integer at faces);
    the metric d(xi)/dx is exact for this map."""
    n = tuple(int(v) for v in n)
    dd = tuple(float(v) for v in (d if np.ndim(d) else (d, d, d)))
    xnode, xin, xif = [], [], []
    for a in range(3):
        if n[a] == 1:
            xnode.append(np.array([0.5 * dd[a]]))
            xin.append(np.array([1.0 / dd[a]]))
            xif.append(np.array([1.0 / dd[a]]))
            continue
        k = 2 * np.pi / n[a]
        xi = np.arange(n[a]) + 0.5
        xf = np.arange(n[a]) + 1.0
        xnode.append(dd[a] * (xi + amp / k * np.sin(k * xi)))
        xin.append(1.0 / (dd[a] * (1 + amp * np.cos(k * xi))))
        xif.append(1.0 / (dd[a] * (1 + amp * np.cos(k * xf))))
    return Grid(n=n, xnode=xnode, xin=xin, xif=xif, L=tuple(n[a] * dd[a] for a in range(3)))


@dataclass
class CurvGrid:
    """General curvilinear periodic grid: node coordinates xyz[3][N] (x
    fastest, then y, then z) and the lattice periods period[3][3] (row a: the
    displacement of the node lattice when index a advances by n[a])."""
    n: tuple
    xyz: np.ndarray
    period: np.ndarray

    @property
    def N(self):
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def L(self):
        return tuple(float(np.linalg.norm(self.period[a])) for a in range(3))

    def mesh(self):
        """Node coordinates, each shaped [nz][ny][nx]."""
        sh = (self.n[2], self.n[1], self.n[0])
        return tuple(self.xyz[c].reshape(sh) for c in range(3))


def as_curvilinear(g: Grid) -> CurvGrid:
    """A rectilinear grid written as a curvilinear one (same nodes)."""
    x, y, z = g.mesh()
    return CurvGrid(n=g.n, xyz=np.stack([x.ravel(), y.ravel(), z.ravel()]), period=np.diag(np.array(g.L, float)))


def affine_grid(n, d, A, origin=(0.0, 0.0, 0.0)) -> CurvGrid:
    """Uniform lattice mapped by the matrix A: node (i, j, k) at
    origin + A ((i + 1/2) d_x, (j + 1/2) d_y, (k + 1/2) d_z); periods A L_a e_a.
    A rotation gives a rotated Cartesian grid, a shear a skewed one."""
    g = uniform_grid(n, d)
    x, y, z = g.mesh()
    A = np.asarray(A, float)
    P = np.stack([x.ravel(), y.ravel(), z.ravel()])
    return CurvGrid(n=g.n, xyz=A @ P + np.asarray(origin, float)[:, None],
                    period=np.stack([A @ (g.L[a] * np.eye(3)[a]) for a in range(3)]))


def rotation(ax, ay, az):
    """Rotation matrix R_z(az) R_y(ay) R_x(ax)."""
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def skewed_grid(n, d, beta=0.2, origin=None) -> CurvGrid:
    """Periodic skewed grid of the paper's convergence tests (Methods › Solver Performance Analysis › Accuracy):
    each coordinate is displaced by beta L/2 times the sine of the other
    active coordinates (averaged over them),
        x_c = xi_c + beta (L_c / 2) mean_{c' != c} sin(2 pi xi_c' / L_c'),
    with xi the uniform lattice position.  In 2-D this is
    x = xi + beta (L/2) sin(2 pi eta / L), y = eta + beta (L/2) sin(2 pi xi / L),
    a periodic counterpart of the printed map, whose displacement is also
    beta L/2 at most; the grid lines turn by up to atan(beta pi) (32 degrees
    at beta = 0.2; half that slope per term in 3-D)."""
    g = uniform_grid(n, d)
    x, y, z = g.mesh()
    xi = [x, y, z]
    act = [a for a in range(3) if g.n[a] > 1]
    out = []
    for c in range(3):
        v = xi[c].copy()
        others = [a for a in act if a != c]
        if c in act and others:
            v = v + beta * g.L[c] / 2 * sum(np.sin(2 * np.pi * xi[a] / g.L[a]) for a in others) / len(others)
        out.append(v.ravel())
    xyz = np.stack(out)
    if origin is not None:
        xyz = xyz + np.asarray(origin, float)[:, None]
    return CurvGrid(n=g.n, xyz=xyz, period=np.diag(np.array(g.L, float)))


def wavy_grid(n, d, amp=0.25, seed=0) -> CurvGrid:
    """Periodic wavy grid: each coordinate displaced by amp cells times a
    product of sines of all active lattice coordinates with seeded phases,
        x_c = xi_c + amp d_c prod_a sin(2 pi xi_a / L_a + phi_ca),
    so that every metric term varies along every axis (no separable
    structure for the metric differences to cancel on)."""
    g = uniform_grid(n, d)
    x, y, z = g.mesh()
    xi = [x, y, z]
    act = [a for a in range(3) if g.n[a] > 1]
    ph = np.random.default_rng(seed).uniform(0, 2 * np.pi, size=(3, 3))
    out = []
    for c in range(3):
        v = xi[c].copy()
        if c in act:
            w = np.ones_like(v)
            for a in act:
                w = w * np.sin(2 * np.pi * xi[a] / g.L[a] + ph[c, a])
            v = v + amp * g.spacing()[c] * g.n[c] / (2 * np.pi) * w
        out.append(v.ravel())
    return CurvGrid(n=g.n, xyz=np.stack(out), period=np.diag(np.array(g.L, float)))


@dataclass
class Laser:
    """Gaussian deposition kernel (Methods › Diffusion flame › Physical model and numerical setup): energy, centre, spatial and
    temporal support, delay."""
    E: float = 0.0
    center: tuple = (0.0, 0.0, 0.0)
    sigma_r: float = 1.0
    t0: float = 0.0
    sigma_t: float = 1.0
    on: bool = False

    def as_array(self):
        return np.array([self.E, *self.center, self.sigma_r, self.t0, self.sigma_t, 1.0 if self.on else 0.0])


@dataclass
class Case:
    name: str
    mech: Mechanism
    grid: Grid
    Y: np.ndarray                 # [ns][N]
    T: np.ndarray                 # [N]
    p: np.ndarray                 # [N]
    vel: np.ndarray               # [3][N]
    laser: Laser = field(default_factory=Laser)
    flags: int = 0
    cfl: float = 0.5
    theta_c: float = 0.1
    psi_c: float = 0.05
    teno_CT: float = 1e-5
    steps: int = 1
    t0: float = 0.0
    meta: dict = field(default_factory=dict)
    # boundary type per axis and side (low, high): BC_PERIODIC, BC_WALL,
    # BC_INFLOW, BC_OUTFLOW; the outflow's far-field pressure and relaxation
    bc: tuple = ((0, 0), (0, 0), (0, 0))
    pinf: tuple = ((0.0, 0.0), (0.0, 0.0), (0.0, 0.0))
    relax: tuple = ((0.0, 0.0), (0.0, 0.0), (0.0, 0.0))


def dirichlet_Y(rng, ns, size=None):
    """Flat Dirichlet draw on the simplex; redrawn while any entry < 1e-8."""
    while True:
        y = rng.dirichlet(np.ones(ns))
        if y.min() >= 1e-8:
            return y


# Fuel and oxidizer streams of the mixing layers carry only the mechanism's
# stable species: those whose enthalpy constant per unit mass (a6 R_u / W) is
# at most this in magnitude.  The others (atoms and radicals, whose seeded
# constants reach ~90 MJ/kg) start at a trace mass fraction.
STREAM_HF_CAP = 5e6       # J/kg
STREAM_TRACE = 1e-6


def stream_Y(rng, mech: Mechanism):
    """A fuel or oxidizer stream: a flat Dirichlet draw over all species
    (dirichlet_Y, same draws), then the species above STREAM_HF_CAP set to
    STREAM_TRACE and the rest rescaled to sum to one."""
    y = dirichlet_Y(rng, mech.ns)
    rad = np.abs(np.asarray(mech.nasa7)[:, 5]) * RU / np.asarray(mech.W) > STREAM_HF_CAP
    if rad.all():
        return y
    y = np.where(rad, 0.0, y)
    y = y / y.sum() * (1.0 - STREAM_TRACE * rad.sum())
    y[rad] = STREAM_TRACE
    return y


def nominal_sound_speed(mech: Mechanism, Y, T):
    W = 1.0 / np.sum(Y / mech.W)
    return float(np.sqrt(1.4 * RU * T / W))


def _streams(k):
    ss = np.random.SeedSequence(k)
    mech_s, ic_s, noise_s, ens_s = ss.spawn(4)
    return mech_s, np.random.default_rng(ic_s), np.random.default_rng(noise_s), np.random.default_rng(ens_s)


def _bandlimited_noise(rng, n, kmax_frac=1.0 / 8.0):
    """Random-phase Fourier modes with |k| <= N/8 and a flat spectrum, unit RMS."""
    nz, ny, nx = n[2], n[1], n[0]
    shape = (nz, ny, nx)
    spec = np.zeros(shape, dtype=complex)
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.fftfreq(nx) * nx
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    nn = np.array([nz, ny, nx], float)
    r = np.sqrt((KZ / nn[0]) ** 2 + (KY / nn[1]) ** 2 + (KX / nn[2]) ** 2)
    mask = (r <= kmax_frac) & (r > 0)
    phase = rng.uniform(0, 2 * np.pi, size=shape)
    spec[mask] = np.exp(1j * phase[mask])
    f = np.real(np.fft.ifftn(spec))
    f /= np.sqrt(np.mean(f * f)) + 1e-300
    return f


# Mechanism seeds of the five workloads.  Chosen among the first dozen seeds
# so that the fastest chemical destruction rate at the workload's peak
# temperature, times the initial stable time step, stays below one (explicit
# RK3 is stable to about 2.5); the test suite checks this with the oracle.
MECH_SEED = {"C1": 1, "C2": 0, "C3": 3, "C4": 3, "C5": 3}


def _mech(ns, nr, mech_seed):
    return make_mechanism(ns, nr, _streams(mech_seed)[0])


def case_c1(seed=1, n=256, mech_seed=MECH_SEED["C1"]) -> Case:
    """C1: 1-D periodic reacting gas with a Gaussian hot spot."""
    _, ic, _, _ = _streams(seed)
    mech = _mech(5, 4, mech_seed)
    dx = 20e-6
    g = uniform_grid((n, 1, 1), dx)
    x = g.xnode[0]
    L = g.L[0]
    T = 300.0 + 1200.0 * np.exp(-((x - L / 2) ** 2) / (2 * (16 * dx) ** 2))
    Y = np.repeat(dirichlet_Y(ic, mech.ns)[:, None], n, axis=1)
    return Case("C1", mech, g, Y, T, np.full(n, P_ATM), np.zeros((3, n)), steps=200)


def case_c2(seed=2, n=128, ns=9, nr=20, mech_seed=MECH_SEED["C2"]) -> Case:
    """C2: 3-D periodic multicomponent Taylor-Green box at Mach 0.3."""
    _, ic, _, _ = _streams(seed)
    mech = _mech(ns, nr, mech_seed)
    Lp = 2 * np.pi * 1e-3
    g = uniform_grid((n, n, n), Lp / n)
    x, y, z = g.mesh()
    xs, ys, zs = x / 1e-3, y / 1e-3, z / 1e-3
    T0 = 1200.0
    Yv = dirichlet_Y(ic, mech.ns)
    c0 = nominal_sound_speed(mech, Yv, T0)
    U0 = 0.3 * c0
    rho0 = P_ATM / (RU * T0 * np.sum(Yv / mech.W))
    u = U0 * np.sin(xs) * np.cos(ys) * np.cos(zs)
    v = -U0 * np.cos(xs) * np.sin(ys) * np.cos(zs)
    w = np.zeros_like(u)
    p = P_ATM + rho0 * U0 ** 2 / 16 * (np.cos(2 * xs) + np.cos(2 * ys)) * (np.cos(2 * zs) + 2)
    N = g.N
    Y = np.repeat(Yv[:, None], N, axis=1)
    vel = np.stack([u.ravel(), v.ravel(), w.ravel()])
    return Case("C2", mech, g, Y, np.full(N, T0), p.ravel(), vel, steps=10, meta={"U0": U0})


def mixing_layer(mech: Mechanism, n, dx, ic, noise_rng, *, E_mJ=None, center_shift=(0.0, 0.0, 0.0),
                 E_scale=1.0, YF=None, YO=None) -> tuple:
    """Periodic double mixing layer in y: fuel stream in the middle band,
    oxidizer outside (each of stable species, stream_Y), tanh profiles of
    thickness 4 dy, shear dU = 0.5 c0
    with 1% band-limited velocity noise, T = 300 K, p = 1 atm, and a laser
    kernel (radius 8 cells) centred on the lower layer."""
    g = uniform_grid(n, dx)
    x, y, z = g.mesh()
    Ly = g.L[1]
    dl = 4 * dx
    phi = 0.5 * (np.tanh((y - Ly / 4) / dl) - np.tanh((y - 3 * Ly / 4) / dl))
    if YF is None:
        YF = stream_Y(ic, mech)
    if YO is None:
        YO = stream_Y(ic, mech)
    Y = phi[None] * YF[:, None, None, None] + (1 - phi[None]) * YO[:, None, None, None]
    T0 = 300.0
    Ym = 0.5 * (YF + YO)
    c0 = nominal_sound_speed(mech, Ym, T0)
    dU = 0.5 * c0
    u = dU * (phi - 0.5)
    vel = np.zeros((3,) + u.shape)
    vel[0] = u
    for m in range(3):
        vel[m] += 0.01 * dU * _bandlimited_noise(noise_rng, g.n)
    if E_mJ is None:
        E_mJ = float(ic.uniform(0.1, 1.0))
    E = E_mJ * 1e-3 * (dx / 50e-6) ** 3 * E_scale
    sr = 8 * dx
    dt0 = 0.5 * dx / (3 * (c0 + dU))
    st = 5 * dt0
    center = (g.L[0] / 2 + center_shift[0] * dx, Ly / 4 + center_shift[1] * dx, g.L[2] / 2 + center_shift[2] * dx)
    las = Laser(E=E, center=center, sigma_r=sr, t0=4 * st, sigma_t=st, on=True)
    N = g.N
    return g, Y.reshape(mech.ns, N), np.full(N, T0), np.full(N, P_ATM), vel.reshape(3, N), las, dict(dU=dU, c0=c0)


def case_c3(seed=3, n=(256, 128, 128), ns=9, nr=20, steps=100, mech_seed=MECH_SEED["C3"]) -> Case:
    """C3: 3-D planar fuel/oxidizer mixing layer with laser deposition."""
    _, ic, noise, _ = _streams(seed)
    mech = _mech(ns, nr, mech_seed)
    g, Y, T, p, vel, las, meta = mixing_layer(mech, n, 50e-6, ic, noise)
    return Case("C3", mech, g, Y, T, p, vel, laser=las, steps=steps, meta=meta)


def case_c5(seed=5, n=64, ns=9, nr=20, steps=50, mech_seed=MECH_SEED["C5"]) -> Case:
    """C5: the 64^3 mixing layer for the adjoint (checkpoints every 10 steps)."""
    _, ic, noise, _ = _streams(seed)
    mech = _mech(ns, nr, mech_seed)
    g, Y, T, p, vel, las, meta = mixing_layer(mech, (n, n, n), 50e-6, ic, noise)
    meta["checkpoint_every"] = 10
    return Case("C5", mech, g, Y, T, p, vel, laser=las, steps=steps, meta=meta)


@dataclass
class Ensemble:
    mech: Mechanism
    members: list                  # list of Case (each with its own grid)
    dlnA: np.ndarray               # [nmem][nr] per-member ln A offsets
    steps: int = 50


def ensemble_c4(seed=4, nmem=64, ns=9, nr=20, sizes=None, steps=50, mech_seed=MECH_SEED["C4"]) -> Ensemble:
    """C4: 64 mixing-layer members of uneven size N^3 (N uniform on
    {32, 40, ..., 96}) with deposition energy x U[0.7, 1.3], kernel centre
    shifted by U[-10, 10] cells per axis and ln A_j + U[-0.5, 0.5]."""
    _, ic, noise, ens = _streams(seed)
    mech = _mech(ns, nr, mech_seed)
    YF = stream_Y(ic, mech)
    YO = stream_Y(ic, mech)
    E_mJ = float(ic.uniform(0.1, 1.0))
    if sizes is None:
        sizes = ens.choice(np.arange(32, 97, 8), size=nmem)
    members, dlnA = [], []
    for m in range(nmem):
        N = int(sizes[m])
        scale = float(ens.uniform(0.7, 1.3))
        shift = tuple(ens.uniform(-10, 10, size=3))
        dl = ens.uniform(-0.5, 0.5, size=nr)
        g, Y, T, p, vel, las, meta = mixing_layer(mech, (N, N, N), 50e-6, ic, noise, E_mJ=E_mJ,
                                                  center_shift=shift, E_scale=scale, YF=YF, YO=YO)
        members.append(Case(f"C4[{m}]", mech, g, Y, T, p, vel, laser=las, steps=steps, meta=meta))
        dlnA.append(dl)
    return Ensemble(mech, members, np.array(dlnA), steps=steps)


# Mechanism seed of the ignition-search base case: a 5-species, 4-reaction
# mechanism whose net heat release turns positive, and grows with the
# deposited energy, once the laser has heated the layer (the workloads'
# seeded mechanisms are net endothermic at those temperatures); explicitly
# stable by the same screen as the workloads.
IGNITION_MECH_SEED = 15


def ignition_base(n=16, mech_seed=IGNITION_MECH_SEED) -> Case:
    """One n^3 member of the mixing-layer ensemble recipe (first member's
    perturbations) with the ignition mechanism: the base case of the
    minimum-ignition-energy search."""
    return ensemble_c4(nmem=1, sizes=[n], ns=5, nr=4, mech_seed=mech_seed).members[0]


# ----------------------------------------------------------------- test cases
def sod_case(n=200, W=0.02897, axis=0) -> Case:
    """Periodic double Sod tube along one axis, single calorically perfect
    species (gamma = 1.4): high state (1 kg/m^3, 1e5 Pa) in the middle half."""
    mech = single_species(W, 3.5)
    dims = [1, 1, 1]
    dims[axis] = n
    dx = 1.0 / n
    g = uniform_grid(tuple(dims), dx)
    x = g.xnode[axis]
    hi = (x >= 0.25) & (x < 0.75)
    rho = np.where(hi, 1.0, 0.125)
    p = np.where(hi, 1e5, 1e4)
    T = p * W / (rho * RU)
    N = g.N
    return Case("sod", mech, g, np.ones((1, N)), T.ravel(), p.ravel(), np.zeros((3, N)),
                flags=CHEM_OFF | VISC_OFF, cfl=0.5, meta={"W": W, "axis": axis})


def vortex_case(n=32, L=10.0) -> Case:
    """Isentropic vortex (Methods › Solver Performance Analysis › Accuracy set-up) on a Cartesian periodic grid in
    non-dimensional units: one species with R_u/W = 1 and gamma = 1.4, so
    that p = rho T; beta = 5, alpha = 1/2, r0 = 0.5, (u0, v0, T0) = (1, 1, 1)."""
    mech = single_species(RU, 3.5, Tmin=1e-3, Tmax=1e3)
    g = uniform_grid((n, n, 1), L / n)
    x, y, _ = g.mesh()
    x = x[0] - L / 2
    y = y[0] - L / 2
    return _vortex_fields(mech, g, x, y)


def vortex_case_curv(grid: CurvGrid, L=10.0) -> Case:
    """The isentropic vortex of vortex_case on a curvilinear grid spanning
    [0, L]^2 (fields at the physical node coordinates, centred at L/2)."""
    mech = single_species(RU, 3.5, Tmin=1e-3, Tmax=1e3)
    x, y, _ = grid.mesh()
    return _vortex_fields(mech, grid, x[0] - L / 2, y[0] - L / 2)


def tgv2d_case(grid, L=2 * np.pi, u0=1.0, rho0=1.0, gamma=1.4, sigma=1.5e-11) -> Case:
    """Two-dimensional Taylor-Green vortex of the paper's viscous accuracy
    test (Methods › Solver Performance Analysis › Accuracy) in non-dimensional units: one species with R_u/W = 1
    and gamma = 1.4, u = u0 sin(kx) cos(ky), v = -u0 cos(kx) sin(ky),
    p = p0 + rho0 u0^2/4 (cos 2kx + cos 2ky) (k = 2 pi / L), rho = rho0,
    Mach number u0 / c0 = 1e-2 / sqrt(gamma).  Fields at the physical node
    coordinates of a rectilinear or curvilinear grid.  The Lennard-Jones
    well depth is the reference temperature (T* = 1 there); the diameter
    sets the viscosity, which the caller may rescale (mu scales as
    1/sigma^2)."""
    c0 = u0 * np.sqrt(gamma) / 1e-2
    p0 = rho0 * c0 ** 2 / gamma
    T0 = p0 / rho0
    mech = single_species(RU, gamma / (gamma - 1), Tmin=0.5 * T0, Tmax=2.0 * T0, sigma=sigma, epsk=T0)
    x, y, _ = grid.mesh()
    x, y = x.ravel(), y.ravel()
    k = 2 * np.pi / L
    N = grid.N
    p = p0 + rho0 * u0 ** 2 / 4 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    vel = np.stack([u0 * np.sin(k * x) * np.cos(k * y), -u0 * np.cos(k * x) * np.sin(k * y), np.zeros(N)])
    return Case("tgv2d", mech, grid, np.ones((1, N)), p / rho0, p, vel, flags=CHEM_OFF,
                meta={"u0": u0, "rho0": rho0, "k": k, "T0": T0})


def vortex_exact(x, y, t=0.0, beta=5.0, alpha=0.5, r0=0.5, gamma=1.4, u0=1.0, v0=1.0, T0=1.0, L=10.0):
    """Exact advected vortex: primitive fields at time t (periodic images
    within one period are folded in by the minimum-image shift)."""
    xs = x - u0 * t
    ys = y - v0 * t
    xs = (xs + L / 2) % L - L / 2
    ys = (ys + L / 2) % L - L / 2
    r2 = (xs ** 2 + ys ** 2) / r0 ** 2
    f = np.exp(alpha * (1 - r2))
    u = beta / (2 * np.pi) * f * ys + u0
    v = -beta / (2 * np.pi) * f * xs + v0
    # the radial momentum balance dp/dr = rho u_theta^2 / r of this velocity
    # field fixes the amplitude with a factor r0^2 (the printed form has r0 = 1)
    T = -(gamma - 1) * beta ** 2 * r0 ** 2 / (16 * alpha * gamma * np.pi ** 2) * np.exp(2 * alpha * (1 - r2)) + T0
    rho = T ** (1 / (gamma - 1))
    p = rho * T
    return rho, u, v, T, p


def _vortex_fields(mech, g, x, y):
    rho, u, v, T, p = vortex_exact(x, y)
    N = g.N
    vel = np.stack([u.ravel(), v.ravel(), np.zeros(N)])
    return Case("vortex", mech, g, np.ones((1, N)), T.ravel(), p.ravel(), vel,
                flags=CHEM_OFF | VISC_OFF, meta={})


def small_case(n=(8, 6, 5), ns=3, nr=1, seed=11, flags=0, stretched=False, dx=50e-6, laser=True,
               T_base=1500.0, noise=0.05, mech=None) -> Case:
    """Small random reacting case for brute-force and parity checks: smooth
    random perturbations of T, p, u and composition around a base state."""
    mech_s, ic, noise_rng, _ = _streams(seed)
    if mech is None:
        mech = make_mechanism(ns, nr, mech_s)
    ns = mech.ns
    g = stretched_grid(n, dx) if stretched else uniform_grid(n, dx)
    N = g.N
    x, y, z = g.mesh()
    ph = ic.uniform(0, 2 * np.pi, size=8)

    def wave(a, b, c, k):
        return (np.sin(2 * np.pi * x / g.L[0] + ph[k]) * a + np.sin(2 * np.pi * y / g.L[1] + ph[k + 1]) * b
                + np.sin(2 * np.pi * z / g.L[2] + ph[k + 2]) * c).ravel()

    T = T_base * (1 + noise * wave(1, 0.7, 0.5, 0))
    p = P_ATM * (1 + noise * wave(0.6, 0.4, 0.8, 1))
    Y0 = dirichlet_Y(ic, ns)
    Y1 = dirichlet_Y(ic, ns)
    s = 0.5 + 0.4 * np.tanh(3 * wave(1, 1, 1, 2))
    Y = s[None] * Y0[:, None] + (1 - s[None]) * Y1[:, None]
    c0 = nominal_sound_speed(mech, Y0, T_base)
    vel = np.stack([0.3 * c0 * wave(1, 0.5, 0.2, 3), 0.2 * c0 * wave(0.3, 1, 0.4, 4),
                    0.25 * c0 * wave(0.5, 0.2, 1, 5)])
    for a in range(3):
        if n[a] == 1:
            vel[a] = 0.0 if a == 2 else vel[a]
    las = Laser(E=1e-4 * (dx / 50e-6) ** 3, center=tuple(0.4 * L for L in g.L), sigma_r=2.0 * dx,
                t0=0.0, sigma_t=1e-7, on=laser)
    return Case("small", mech, g, Y, T, p, vel, laser=las, flags=flags)
