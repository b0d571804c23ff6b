"""Multi-fidelity co-processing: a high-fidelity (HF) simulation and an
ensemble of low-fidelity (LF) members advanced at the same time on one GPU.

The paper runs its bi-fidelity ensembles with the HF sample on the GPUs and
the LF samples on the CPUs of the same nodes, concurrently, so that the
total time stays close to the HF time alone whatever the number of LF
samples (Results › Ensemble simulation; Application examples › Ignition of
a diffusion flame).  Here both fidelities run in the HIP library on the same
MI355X, on two HIP streams: the HF grid's steps on one, the LF ensemble's
captured graph on the other, so that the LF kernels fill what the HF
launches leave idle (launch gaps, tails of waves, the small per-member
kernels).  No CPU solver is involved: every step of both fidelities runs in
the library's kernels; this module orders the launches and times them.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import torch

from . import htr


@dataclass
class CoRun:
    hf_ms: float          # HF steps alone
    lf_ms: float          # LF steps alone
    both_ms: float        # both fidelities at once, on two streams
    hf_steps: int
    lf_steps: int

    def overlap(self):
        """Fraction of the shorter run hidden under the longer one: 1 when
        the concurrent time equals the longer run alone, 0 when it equals the
        sum of both."""
        lo, hi = min(self.hf_ms, self.lf_ms), max(self.hf_ms, self.lf_ms)
        return (self.hf_ms + self.lf_ms - self.both_ms) / lo if lo > 0 else 0.0


class Fidelities:
    """One HF single-grid problem and one LF ensemble with their states and
    work memory, each with its own stream (default priority)."""

    def __init__(self, hf_case, lf_cases, lf_dlnA=None, device="cuda"):
        self.hf_case = hf_case
        self.hf = htr.Context.from_case(hf_case)
        self.lf_ctx = htr.Context(lf_cases[0].mech, lf_cases[0].grid)
        self.lf = htr.Batch.from_cases(self.lf_ctx, lf_cases, lf_dlnA)
        self.hf_U0 = htr.cons_from_case(self.hf, hf_case, device)
        self.hf_T0 = htr.to_dev(hf_case.T, device)
        self.lf_U0, self.lf_T0 = htr.batch_state_from_cases(self.lf, lf_cases, device)
        self.hf_work = self.hf.new_work(device)
        self.lf_work = self.lf.new_work(device)
        self.s_hf = torch.cuda.Stream(device=device)
        self.s_lf = torch.cuda.Stream(device=device)
        self.laser = hf_case.laser if hf_case.laser.on else None
        self.reset()

    def reset(self):
        """Both fidelities back to their initial states (time, dt, J zeroed)."""
        z = lambda n: torch.zeros(n, dtype=torch.float64, device=self.hf_U0.device)  # noqa: E731
        self.hf_U, self.hf_T = self.hf_U0.clone(), self.hf_T0.clone()
        self.lf_U, self.lf_T = self.lf_U0.clone(), self.lf_T0.clone()
        self.hf_t, self.hf_dt, self.hf_J = z(1), z(1), z(1)
        self.lf_t, self.lf_dt, self.lf_J = z(self.lf.nmem), z(self.lf.nmem), z(self.lf.nmem)
        torch.cuda.synchronize()

    def hf_steps(self, n):
        for _ in range(n):
            htr.htr_rk3_step(self.hf, self.hf_U, self.hf_T, self.hf_t, self.hf_dt, 1, self.laser, None, self.hf_work,
                             self.hf_J, stream=self.s_hf)

    def lf_steps(self, n):
        htr.htr_rk3_steps_batched(self.lf, self.lf_U, self.lf_T, self.lf_t, self.lf_dt, 1, n, self.lf_work,
                                  self.lf_J, use_graph=True, stream=self.s_lf)

    def check(self):
        htr.htr_check(self.hf, self.s_hf)
        htr.htr_batch_check(self.lf, self.s_lf)


def co_process(fid: Fidelities, hf_steps, lf_steps, warmup=True):
    """Times the HF steps alone, the LF steps alone and both at once (each
    from the initial states), wall time between device synchronisations."""
    def timed(run_hf, run_lf):
        fid.reset()
        t0 = time.perf_counter()
        if run_hf:
            fid.hf_steps(hf_steps)
        if run_lf:
            fid.lf_steps(lf_steps)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        fid.check()
        return ms
    if warmup:                 # graph capture and first launches outside the timing
        timed(True, True)
    hf = timed(True, False)
    lf = timed(False, True)
    both = timed(True, True)
    return CoRun(hf, lf, both, hf_steps, lf_steps)
