"""Ignition-energy search on the batched path: the bracketing logic on the
host, and on the GPU the search against single-grid runs of the bracket's
ends."""
import numpy as np
import pytest
import torch

import synth
from paper_2202_02319_amd import htr
from paper_2202_02319_amd.ignition import (initial_stable_dt, min_ignition_energies, narrow, round_energies,
                                           with_energy)


def test_narrow_keeps_the_transition():
    e = np.linspace(1.0, 2.0, 6)
    assert narrow(e, [False, False, True, True, True, True]) == (1.2, 1.4)
    assert narrow(e, [False] * 5 + [True]) == (1.8, 2.0)
    for bad in ([True] * 6, [False] * 6, [False, True, False, True, True, True]):
        with pytest.raises(ValueError):
            narrow(e, bad)
    with pytest.raises(ValueError):
        narrow(e[::-1], [False] * 3 + [True] * 3)


@pytest.mark.parametrize("members", [2, 3, 6])
def test_bracket_shrinks_on_a_monotone_response(members):
    """The rounds of the search, with a host-side response in place of the
    ensemble run: the bracket holds the threshold, shrinks by (members - 1)
    in the first round and by (members + 1) after it, and later rounds stay
    strictly inside the bracket."""
    thr = 0.6180339
    lo, hi = 0.1, 2.0
    width = hi - lo
    for r in range(4):
        e = round_energies(lo, hi, members, r == 0)
        assert len(e) == members
        if r == 0:
            lo, hi = narrow(e, e > thr)
            width /= members - 1
        else:
            assert lo < e[0] and e[-1] < hi
            lo, hi = narrow(np.r_[lo, e, hi], np.r_[False, e > thr, True])
            width /= members + 1
        assert lo < thr <= hi
        assert hi - lo == pytest.approx(width, rel=1e-9)


def _base(n=16):
    """One 16^3 member of the mixing-layer ensemble (its mechanism, mixture
    and laser kernel)."""
    return synth.ensemble_c4(nmem=1, sizes=[n]).members[0]


def _single_peak(case, nsteps, dt_step, chunk):
    """Peak T of a single-grid run (same fixed step, same sampling)."""
    ctx = htr.Context.from_case(case)
    U = htr.cons_from_case(ctx, case)
    T = torch.as_tensor(case.T.copy(), device="cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.full((1,), dt_step, dtype=torch.float64, device="cuda")
    work = ctx.new_work()
    peak = float(T.max())
    for k in range(nsteps):
        htr.htr_rk3_step(ctx, U, T, t, dt, 0, case.laser, None, work, None)
        if (k + 1) % chunk == 0 or k + 1 == nsteps:
            peak = max(peak, float(T.max()))
    htr.htr_check(ctx)
    return peak


@pytest.mark.gpu
def test_search_on_the_batched_path_matches_single_runs():
    """Two searches (laser durations sigma_t and 2 sigma_t) in one ensemble
    per round: the brackets shrink as designed, the batched peaks equal
    single-grid runs bit for bit, and the bracket ends run alone fall on
    either side of the threshold."""
    b0 = _base()
    b1 = with_energy(b0, b0.laser.E)
    b1.laser.sigma_t = 2.0 * b0.laser.sigma_t
    bases = [b0, b1]
    ctx = htr.Context.from_case(b0)
    E0 = b0.laser.E
    nsteps, chunk, members = 40, 5, 4
    dt = 0.5 * initial_stable_dt(ctx, b0)
    # per search, a threshold halfway between the peaks of the lowest and highest energies
    T_ign = []
    for b in bases:
        p_lo = _single_peak(with_energy(b, 0.25 * E0), nsteps, dt, chunk)
        p_hi = _single_peak(with_energy(b, 2.0 * E0), nsteps, dt, chunk)
        print(f"sigma_t {b.laser.sigma_t:.3e}: peak T {p_lo:.3f} K at 0.25 E0, {p_hi:.3f} K at 2 E0", flush=True)
        assert p_hi > p_lo + 1.0
        T_ign.append(0.5 * (p_lo + p_hi))
    res = min_ignition_energies(ctx, bases, 0.25 * E0, 2.0 * E0, nsteps, T_ign, members=members, rounds=2,
                                chunk=chunk, dt=dt)
    for i, (b, r) in enumerate(zip(bases, res)):
        assert r.E_hi - r.E_lo == pytest.approx(1.75 * E0 / ((members - 1) * (members + 1)), rel=1e-9)
        for energies, peaks, _ in r.rounds:
            assert np.all(np.diff(peaks) > 0)
        # batched peaks of the last round equal single-grid runs of the same members
        energies, peaks, _ = r.rounds[-1]
        for m in (0, members - 1):
            assert peaks[m] == _single_peak(with_energy(b, energies[m]), nsteps, dt, chunk)
        assert _single_peak(with_energy(b, r.E_lo), nsteps, dt, chunk) <= T_ign[i]
        assert _single_peak(with_energy(b, r.E_hi), nsteps, dt, chunk) > T_ign[i]
