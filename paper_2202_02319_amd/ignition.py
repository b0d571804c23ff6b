"""Minimum ignition energy by a bracketing search on the batched ensemble
path: the paper's ensemble workflow over the deposited laser energy
(Application examples › Ignition of a diffusion flame; Methods › Diffusion
flame › Ensemble and data analysis): for each laser duration, an interval
[a, b] is tightened such that energy a does not ignite and b does.

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

Ignition is judged as the paper judges it, by the reaction products still
growing after the deposit: here through the chemical heat they release.
The library accumulates each member's time-integrated heat release
J(t) = integral of sum_cells dV HRR dt on the device; a member ignites when
the heat released after the deposit has ended (t_d = t0 + 4 sigma_t),
J(t_end) - J(t_d), is at least `kappa` times the deposited energy E and the
release is still going on over the last `chunk` steps.  Without chemistry
(the inert control) J stays zero and nothing ignites.  The peak temperature
is tracked as well (the paper confirms failures by the global maximum
temperature falling back).  Every member of a search advances with the same
fixed time step, so that all members reach t_d and t_end at the same step.
All arithmetic runs in the HIP library; this module chooses energies and
reads back a few numbers per member.
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
    rounds: list = field(default_factory=list)   # (energies, MemberRuns, ignited) per round


@dataclass
class MemberRuns:
    """Per-member results of one batched run."""
    J_d: np.ndarray        # time-integrated heat release at the deposit end t_d
    J_end: np.ndarray      # ... at the end of the run
    J_last: np.ndarray     # ... `chunk` steps before the end
    peak_T: np.ndarray     # peak temperature over the run (sampled every chunk)
    final_max_T: np.ndarray
    n_d: int               # the step at which J_d was read

    def released(self):
        """Chemical heat released after the deposit, J(t_end) - J(t_d)."""
        return self.J_end - self.J_d


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


def deposit_end_step(laser, dt):
    """The first step count n with n dt >= t0 + 4 sigma_t."""
    return int(np.ceil((laser.t0 + 4.0 * laser.sigma_t) / dt - 1e-9))


def run_members(ctx, cases, n_d, n_after, dt, chunk=5):
    """Advances the cases together as one batched ensemble with the fixed step
    dt[m] (one value for all), n_d steps to the deposit end and n_after more,
    and returns the members' heat release at the deposit end and at the end
    (and `chunk` steps before it) and their temperature peaks."""
    if n_after < chunk or chunk < 1:
        raise ValueError("need n_after >= chunk >= 1")
    b = htr.Batch.from_cases(ctx, cases)
    try:
        U, T = htr.batch_state_from_cases(b, cases)
        dev = U.device
        t = torch.zeros(b.nmem, dtype=torch.float64, device=dev)
        J = torch.zeros(b.nmem, dtype=torch.float64, device=dev)
        dtd = torch.as_tensor(np.broadcast_to(np.asarray(dt, dtype=np.float64), (b.nmem,)).copy(), device=dev)
        peak = torch.empty(b.nmem, dtype=torch.float64, device=dev)
        cur = torch.empty(b.nmem, dtype=torch.float64, device=dev)
        work = b.new_work()
        htr.htr_batch_member_max(b, T, peak, accumulate=False)

        def advance(nsteps):
            done = 0
            while done < nsteps:
                k = min(chunk, nsteps - done)
                htr.htr_rk3_steps_batched(b, U, T, t, dtd, 0, k, work, J, use_graph=True)
                htr.htr_batch_member_max(b, T, peak, accumulate=True)
                done += k
        advance(n_d)
        J_d = J.cpu().numpy().copy()
        advance(n_after - chunk)
        J_last = J.cpu().numpy().copy()
        advance(chunk)
        J_end = J.cpu().numpy().copy()
        htr.htr_batch_member_max(b, T, cur, accumulate=False)
        htr.htr_batch_check(b)
        return MemberRuns(J_d, J_end, J_last, peak.cpu().numpy(), cur.cpu().numpy(), n_d)
    finally:
        b.close()


def ignited(runs, energies, kappa):
    """The ignition criterion: heat released after the deposit >= kappa E and
    still released over the last chunk."""
    E = np.asarray(energies, dtype=float)
    return (runs.released() >= kappa * E) & (runs.J_end - runs.J_last > 0.0)


def min_ignition_energies(ctx, bases, E_lo, E_hi, n_after, kappa=1e-2, members=8, rounds=3, chunk=5,
                          dt=None, dt_factor=0.5):
    """Brackets of the smallest laser energy that ignites, one search per base
    case (e.g. one per laser duration), all searches of a round in one
    batched ensemble.  Each member runs to the end of its deposit and n_after
    steps more.

    E_lo, E_hi and dt are scalars or one value per base.  dt defaults to
    dt_factor times each base's initial stable step, leaving room for the
    faster sound speed of the heated gas."""
    nb = len(bases)
    if nb == 0:
        raise ValueError("no base cases")
    per = lambda v: np.broadcast_to(np.asarray(v, dtype=float), (nb,)).copy()  # noqa: E731
    lo, hi = per(E_lo), per(E_hi)
    if not np.all((hi > lo) & (lo > 0)):
        raise ValueError("need 0 < E_lo < E_hi")
    if members < 2:
        raise ValueError("need at least 2 members per round (the first round runs both ends)")
    if not kappa > 0:
        raise ValueError("need kappa > 0")
    if dt is None:
        dt = [dt_factor * initial_stable_dt(ctx, c) for c in bases]
    dt = per(dt)
    n_d = max(deposit_end_step(bases[i].laser, dt[i]) for i in range(nb))
    res = [SearchResult(float(lo[i]), float(hi[i]), float(dt[i])) for i in range(nb)]
    for r in range(rounds):
        energies = [round_energies(lo[i], hi[i], members, r == 0) for i in range(nb)]
        cases = [with_energy(bases[i], E) for i in range(nb) for E in energies[i]]
        runs = run_members(ctx, cases, n_d, n_after, np.repeat(dt, members), chunk)
        for i in range(nb):
            sl = slice(i * members, (i + 1) * members)
            sub = MemberRuns(runs.J_d[sl], runs.J_end[sl], runs.J_last[sl], runs.peak_T[sl], runs.final_max_T[sl],
                             runs.n_d)
            ig = ignited(sub, energies[i], kappa)
            res[i].rounds.append((energies[i], sub, ig))
            if r == 0:
                lo[i], hi[i] = narrow(energies[i], ig)
            else:
                lo[i], hi[i] = narrow(np.r_[lo[i], energies[i], hi[i]], np.r_[False, ig, True])
            res[i].E_lo, res[i].E_hi = float(lo[i]), float(hi[i])
    return res


def min_ignition_energy(ctx, base_case, E_lo, E_hi, n_after, **kw):
    """The search of min_ignition_energies for one base case."""
    return min_ignition_energies(ctx, [base_case], E_lo, E_hi, n_after, **kw)[0]
