"""Seeded synthetic reaction mechanisms.

The paper's methane mechanisms (Methods › Solver) are not
available, so every mechanism here is drawn from a seed: species are small
H/O(/N) formulas, reactions are every element-balanced exchange with one or
two molecules on each side, and the thermodynamic, transport and Arrhenius
parameters are random draws in physically plausible ranges.

This module only draws numbers.  It evaluates none of the method's formulas
(no thermodynamics, no rates): the oracle and the GPU library each do that on
their own from the tables returned here.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# standard atomic masses, kg/mol
ATOMIC_MASS = {"H": 1.008e-3, "O": 15.999e-3, "N": 14.007e-3}
ELEMENTS = ("H", "O", "N")

# candidate formulas: (H, O, N) atom counts, one to three atoms
_POOL = [(h, o, n) for h in range(3) for o in range(3) for n in range(3) if 1 <= h + o + n <= 3]


def formula_name(f) -> str:
    s = ""
    for e, n in zip(ELEMENTS, f):
        if n:
            s += e + (str(n) if n > 1 else "")
    return s


@dataclass
class Mechanism:
    """Tables in SI units, laid out as the C interfaces expect them."""

    names: list
    elem: np.ndarray        # [ne][ns] atom counts
    W: np.ndarray           # [ns] kg/mol
    nasa7: np.ndarray       # [ns][7]
    lj_sigma: np.ndarray    # [ns] m
    lj_epsk: np.ndarray     # [ns] K
    lnA: np.ndarray         # [nr] ln of SI pre-exponential factor
    beta: np.ndarray        # [nr]
    Ea: np.ndarray          # [nr] J/mol
    nu_f: np.ndarray        # [nr][ns] int32
    nu_r: np.ndarray        # [nr][ns] int32
    Tmin: float = 200.0
    Tmax: float = 6000.0
    meta: dict = field(default_factory=dict)

    @property
    def ns(self):
        return len(self.W)

    @property
    def nr(self):
        return len(self.lnA)


def _enumerate_reactions(formulas, sizes=(1, 2)):
    """All element-balanced reactions with one or two molecules per side, no
    species on both sides, each unordered pair of sides listed once."""
    ns = len(formulas)
    sides = []
    for k in sizes:
        for combo in itertools.combinations_with_replacement(range(ns), k):
            sides.append(combo)

    def atoms(side):
        return tuple(sum(formulas[s][e] for s in side) for e in range(3))

    out = []
    for a, b in itertools.combinations(range(len(sides)), 2):
        ra, rb = sides[a], sides[b]
        if set(ra) & set(rb):
            continue
        if atoms(ra) != atoms(rb):
            continue
        out.append((ra, rb))
    return out


def _draw_nasa7(rng, n_atoms, Tmin, Tmax):
    """c_p/R drawn increasing at five temperatures and interpolated by a
    quartic; rejected if it leaves [1.05, hi + 2] on [Tmin, Tmax]."""
    Tk = np.array([300.0, 1000.0, 2000.0, 3500.0, 5000.0])
    lo, hi = 2.5, 3.5 + 1.5 * (n_atoms - 1)
    grid = np.linspace(Tmin, Tmax, 400)
    for _ in range(1000):
        vals = np.sort(rng.uniform(lo, hi, size=5))
        V = np.vander(Tk / 1000.0, 5, increasing=True)
        c = np.linalg.solve(V, vals)                    # in powers of T/1000
        a = c / (1000.0 ** np.arange(5))                 # in powers of T
        g = np.polynomial.polynomial.polyval(grid, a)
        if g.min() >= 1.05 and g.max() <= hi + 2.0:
            break
    else:  # pragma: no cover
        raise RuntimeError("NASA-7 draw failed")
    a6 = rng.uniform(-1.2e4, 1.2e4)                      # enthalpy constant, K
    a7 = rng.uniform(-5.0, 10.0)                         # entropy constant
    return np.concatenate([a, [a6, a7]])


def _pick_species(rng, ns):
    """Greedy seeded choice of ns formulas that admit many reactions: start
    from a random formula, then repeatedly add one (ties broken at random)
    that maximises the number of element-balanced reactions."""
    sel = [int(rng.integers(len(_POOL)))]
    while len(sel) < ns:
        best, cands = -1, []
        for i in range(len(_POOL)):
            if i in sel:
                continue
            r = len(_enumerate_reactions([_POOL[j] for j in sel + [i]]))
            if r > best:
                best, cands = r, [i]
            elif r == best:
                cands.append(i)
        sel.append(int(rng.choice(cands)))
    return [_POOL[i] for i in sel]


def make_mechanism(ns: int, nr: int, seed, *, A_range=(1e6, 1e12), beta_range=(-1.0, 1.0),
                   Ea_range=(50e3, 200e3), Tmin=200.0, Tmax=6000.0, **_ignored) -> Mechanism:
    """Seeded mechanism with ns species and nr reversible reactions.

    A is drawn log-uniform in CHEMKIN units ((cm^3/mol)^(order-1)/s) and
    converted to SI.  Orientation: a side with two molecules reacts forward
    against a side with one (recombination); between two-molecule sides the
    side with the larger enthalpy-constant sum reacts forward (nominally
    exothermic).
    """
    rng = np.random.default_rng(seed)
    for _ in range(100):
        formulas = _pick_species(rng, ns)
        rx = _enumerate_reactions(formulas)
        if len(rx) >= nr:
            break
    else:
        raise ValueError(f"no species set with {nr} reactions")
    chosen = [rx[i] for i in sorted(rng.choice(len(rx), size=nr, replace=False).tolist())]
    elem = np.array([[f[e] for f in formulas] for e in range(3)], dtype=np.int32)
    W = np.array([sum(ATOMIC_MASS[ELEMENTS[e]] * f[e] for e in range(3)) for f in formulas])
    nasa = np.array([_draw_nasa7(rng, sum(f), Tmin, Tmax) for f in formulas])
    sig = rng.uniform(2.5, 4.0, size=ns) * 1e-10
    epsk = rng.uniform(30.0, 500.0, size=ns)
    nu_f = np.zeros((nr, ns), np.int32)
    nu_r = np.zeros((nr, ns), np.int32)
    for j, (ra, rb) in enumerate(chosen):
        if len(ra) != len(rb):
            if len(ra) < len(rb):
                ra, rb = rb, ra
        elif sum(nasa[s, 5] for s in ra) < sum(nasa[s, 5] for s in rb):
            ra, rb = rb, ra
        for s in ra:
            nu_f[j, s] += 1
        for s in rb:
            nu_r[j, s] += 1
    order = nu_f.sum(axis=1)
    logA_ch = rng.uniform(np.log10(A_range[0]), np.log10(A_range[1]), size=nr)
    lnA = logA_ch * np.log(10.0) + (order - 1) * np.log(1e-6)
    beta = rng.uniform(beta_range[0], beta_range[1], size=nr)
    Ea = rng.uniform(Ea_range[0], Ea_range[1], size=nr)
    return Mechanism(
        names=[formula_name(f) for f in formulas], elem=elem, W=W, nasa7=nasa,
        lj_sigma=sig, lj_epsk=epsk, lnA=lnA, beta=beta, Ea=Ea, nu_f=nu_f, nu_r=nu_r,
        Tmin=Tmin, Tmax=Tmax, meta={"seed": str(seed), "reactions": [list(map(list, r)) for r in chosen]},
    )


def single_species(W: float, cp_over_R: float = 3.5, Tmin=200.0, Tmax=6000.0,
                   sigma=3.6e-10, epsk=100.0) -> Mechanism:
    """One calorically perfect species (constant c_p/R), no reactions."""
    a = np.zeros((1, 7))
    a[0, 0] = cp_over_R
    return Mechanism(
        names=["X"], elem=np.zeros((3, 1), np.int32), W=np.array([W]), nasa7=a,
        lj_sigma=np.array([sigma]), lj_epsk=np.array([epsk]), lnA=np.zeros(0), beta=np.zeros(0),
        Ea=np.zeros(0), nu_f=np.zeros((0, 1), np.int32), nu_r=np.zeros((0, 1), np.int32),
        Tmin=Tmin, Tmax=Tmax,
    )
