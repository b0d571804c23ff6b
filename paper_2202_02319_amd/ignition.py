"""Minimum ignition energy by a bracketing search on the batched ensemble
path: the paper's ensemble workflow over the deposited laser energy (Application examples › Ignition of a diffusion flame › Ensemble and data analysis,
ensemble and data analysis): for each laser duration, an interval [a, b] is
tightened such that energy a does not ignite and b does.

The paper runs one bisection per duration as separate simulations.  Here
each round is ONE batched ensemble, with one launch per kernel over all
members and the steps captured in a HIP graph, that holds several energies
for every search at once (a k-section rather than a bisection):

- the first search iteration runs `members` energies spaced evenly over
  [E_lo, E_hi], ends included, which also checks that the bracket holds the
  transition;
- later iterations run `members` interior energies of the current bracket,
  so a bracket shrinks by (members - 1) in the first iteration and by
  (members + 1) in each one after it (one interior energy per iteration
  would be the paper's bisection).

A member ignites when its peak temperature over the run exceeds T_ign
(tracked on the device by the library's per-member maximum kernel every
`chunk` steps).  Every member of a search advances with the same fixed
time step, so that after a given number of steps all members have reached
the same time and their peaks compare at equal times (a per-member stable
step would let the hotter members fall behind).  All arithmetic runs in the
HIP library; this module chooses energies and reads back one peak per
member.
"""
from __future__ import annotations

import copy
from dataclasses import dataclass, field

import numpy as np
import torch

from . import htr


def narrow(energies, ignited):
    """The new bracket from one round: the largest energy that did not ignite
    below the smallest that did.  energies ascending; the outcomes must be
    monotone (no ignition, then ignition); raises otherwise or if the
    energies do not contain the transition."""
    e = np.asarray(energies, dtype=float)
    ig = np.asarray(ignited, dtype=bool)
    if e.ndim != 1 or e.shape != ig.shape or e.size < 2:
        raise ValueError("need matching 1-D energies and outcomes, at least two")
    if not np.all(np.diff(e) > 0):
        raise ValueError("energies must be ascending")
    if ig[0]:
        raise ValueError("the lowest energy already ignites: lower E_lo")
    if not ig[-1]:
        raise ValueError("the highest energy does not ignite: raise E_hi")
    k = int(np.argmax(ig))
    if not np.all(ig[k:]):
        raise ValueError(f"ignition is not monotone in the energy: {ig.tolist()}")
    return float(e[k - 1]), float(e[k])


def round_energies(lo, hi, members, first):
    """The energies of one round: `members` points spaced evenly over
    [lo, hi] with the ends in the first round, strictly inside afterwards."""
    if first:
        return np.linspace(lo, hi, members)
    return np.linspace(lo, hi, members + 2)[1:-1]


@dataclass
class SearchResult:
    E_lo: float
    E_hi: float
    dt: float = 0.0
    rounds: list = field(default_factory=list)   # (energies, peak temperatures, ignited) per round


def with_energy(case, E):
    """A copy of the case whose laser deposits energy E (fields shared)."""
    c = copy.copy(case)
    c.laser = copy.copy(case.laser)
    c.laser.E = float(E)
    return c


def initial_stable_dt(ctx, case):
    """The stable step of the case's initial state (the library's CFL and
    diffusive limits)."""
    U = htr.cons_from_case(ctx, case)
    T = htr.to_dev(case.T)
    dt = torch.zeros(1, dtype=torch.float64, device=U.device)
    htr.htr_stable_dt(ctx, U, T, dt)
    return float(dt.cpu()[0])


def peak_temperatures(ctx, cases, nsteps, dt, chunk=5):
    """Advances the cases together as one batched ensemble for nsteps SSP-RK3
    steps, member m with the fixed step dt[m] (a scalar: the same for all),
    and returns each member's peak temperature over the run: the initial
    field, then after every `chunk` steps."""
    b = htr.Batch.from_cases(ctx, cases)
    try:
        U, T = htr.batch_state_from_cases(b, cases)
        t = torch.zeros(b.nmem, dtype=torch.float64, device=U.device)
        dtd = torch.as_tensor(np.broadcast_to(np.asarray(dt, dtype=np.float64), (b.nmem,)).copy(),
                              device=U.device)
        peak = torch.empty(b.nmem, dtype=torch.float64, device=U.device)
        work = b.new_work()
        htr.htr_batch_member_max(b, T, peak, accumulate=False)
        done = 0
        while done < nsteps:
            k = min(chunk, nsteps - done)
            htr.htr_rk3_steps_batched(b, U, T, t, dtd, 0, k, work, None, use_graph=True)
            htr.htr_batch_member_max(b, T, peak, accumulate=True)
            done += k
        htr.htr_batch_check(b)
        return peak.cpu().numpy()
    finally:
        b.close()


def min_ignition_energies(ctx, bases, E_lo, E_hi, nsteps, T_ign, members=8, rounds=3, chunk=5,
                          dt=None, dt_factor=0.5):
    """Brackets of the smallest laser energy that ignites (peak T above T_ign
    within nsteps steps), one search per base case (e.g. one per laser
    duration), all searches of a round in one batched ensemble.

    E_lo, E_hi, dt and T_ign are scalars or one value per base.  dt defaults
    to dt_factor times each base's initial stable step, leaving room for the
    faster sound speed of the heated gas."""
    nb = len(bases)
    if nb == 0:
        raise ValueError("no base cases")
    per = lambda v: np.broadcast_to(np.asarray(v, dtype=float), (nb,)).copy()  # noqa: E731
    lo, hi, T_ign = per(E_lo), per(E_hi), per(T_ign)
    if not np.all((hi > lo) & (lo > 0)):
        raise ValueError("need 0 < E_lo < E_hi")
    if members < 2:
        raise ValueError("need at least 2 members per round (the first round runs both ends)")
    if dt is None:
        dt = [dt_factor * initial_stable_dt(ctx, c) for c in bases]
    dt = per(dt)
    res = [SearchResult(float(lo[i]), float(hi[i]), float(dt[i])) for i in range(nb)]
    for r in range(rounds):
        energies = [round_energies(lo[i], hi[i], members, r == 0) for i in range(nb)]
        cases = [with_energy(bases[i], E) for i in range(nb) for E in energies[i]]
        peaks = peak_temperatures(ctx, cases, nsteps, np.repeat(dt, members), chunk)
        for i in range(nb):
            pk = peaks[i * members:(i + 1) * members]
            ig = pk > T_ign[i]
            res[i].rounds.append((energies[i], pk, ig))
            if r == 0:
                lo[i], hi[i] = narrow(energies[i], ig)
            else:
                lo[i], hi[i] = narrow(np.r_[lo[i], energies[i], hi[i]], np.r_[False, ig, True])
            res[i].E_lo, res[i].E_hi = float(lo[i]), float(hi[i])
    return res


def min_ignition_energy(ctx, base_case, E_lo, E_hi, nsteps, T_ign, **kw):
    """The search of min_ignition_energies for one base case."""
    return min_ignition_energies(ctx, [base_case], E_lo, E_hi, nsteps, T_ign, **kw)[0]
