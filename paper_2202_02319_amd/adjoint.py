"""Time-integrated heat release and its gradient through the discrete
adjoint, behind a torch.autograd.Function with step checkpointing.

J(theta) = sum_steps dt sum_k b_k sum_cells dV HRR(U^(k), t_k) for a fixed
number of SSP-RK3 steps with a frozen step dt, theta = (E, centre x, y, z,
ln A offsets of every reaction).  The forward pass keeps the state every
`checkpoint_every` steps, and it takes the last segment's steps with their
tapes and keeps them; the backward pass re-runs every other segment keeping
its stage states and forward tapes, and walks each segment in reverse with
htr_rk3_step_adjoint.  All arithmetic runs in the HIP library; torch holds
the buffers.
"""
from __future__ import annotations

import copy

import torch

from . import htr


class HeatReleaseProblem:
    """A fixed problem: context, initial state, frozen dt, step count."""

    def __init__(self, ctx, U0, T0, laser, dt, nsteps, checkpoint_every=10, t0=0.0):
        self.ctx, self.U0, self.T0 = ctx, U0.contiguous(), T0.contiguous()
        self.laser = copy.copy(laser)
        self.dt, self.nsteps, self.K, self.t0 = float(dt), int(nsteps), int(checkpoint_every), float(t0)
        self.work = ctx.new_work()
        self.adj_work = htr.new_adjoint_work(ctx)
        self.nth = 4 + ctx.nr
        # one segment's re-run: per step its start state, stage states and forward tape
        self.seg_states = [torch.empty_like(self.U0) for _ in range(self.K)]
        self.seg_stages = [torch.empty_like(self.work) for _ in range(self.K)]
        self.seg_tapes = [htr.new_tape(ctx) for _ in range(self.K)]

    def _laser_for(self, theta):
        L = copy.copy(self.laser)
        th = theta.detach().cpu().tolist()
        L.E = th[0]
        L.center = (th[1], th[2], th[3])
        return L

    def _step(self, U, T, t, L, dlnA, J, work=None, tape=None):
        t_dev = torch.full((1,), t, dtype=torch.float64, device=U.device)
        dt_dev = torch.full((1,), self.dt, dtype=torch.float64, device=U.device)
        if tape is None:
            htr.htr_rk3_step(self.ctx, U, T, t_dev, dt_dev, 0, L, dlnA, self.work, J)
        else:
            htr.htr_rk3_step_taped(self.ctx, U, T, t_dev, dt_dev, 0, L, dlnA, work, J, tape)

    def forward(self, theta, keep_last=False):
        """J and the checkpoints [(step, U, T)].  keep_last: the last
        segment's steps are taken with their tapes, kept for the backward
        pass, which then does not re-run that segment."""
        L = self._laser_for(theta)
        dlnA = theta[4:].detach().contiguous()
        U, T = self.U0.clone(), self.T0.clone()
        J = torch.zeros(1, dtype=torch.float64, device=U.device)
        ckpts = []
        last0 = ((self.nsteps - 1) // self.K) * self.K if self.nsteps > 0 else 0
        self._kept = None
        for n in range(self.nsteps):
            if n % self.K == 0:
                ckpts.append((n, U.clone(), T.clone()))
            if keep_last and n >= last0:
                i = n - last0
                self.seg_states[i].copy_(U)
                self._step(U, T, self.t0 + n * self.dt, L, dlnA, J, self.seg_stages[i], self.seg_tapes[i])
            else:
                self._step(U, T, self.t0 + n * self.dt, L, dlnA, J)
        htr.htr_check(self.ctx)
        if keep_last and self.nsteps > 0:
            self._kept = (ckpts, last0, T.clone())
        return J, ckpts

    def switch_flips(self, theta_a, theta_b):
        """Runs the forward at two parameter points side by side, each step
        taped, and counts the discrete switches that differ between them:
        (J_a, J_b, sensor flags that differ, per-face TENO cut-off patterns
        that differ),
        over every stage of every step.  Where both counts are zero, the two
        runs took the same branch everywhere, so the frozen-switch adjoint is
        the derivative of the piecewise-smooth J between them."""
        runs = []
        for th in (theta_a, theta_b):
            runs.append(dict(L=self._laser_for(th), dlnA=th[4:].detach().contiguous(), U=self.U0.clone(),
                             T=self.T0.clone(), J=torch.zeros(1, dtype=torch.float64, device=self.U0.device),
                             work=torch.empty_like(self.work), tape=htr.new_tape(self.ctx)))
        nflag = nteno = 0
        for n in range(self.nsteps):
            for r in runs:
                r["tape"].zero_()
                self._step(r["U"], r["T"], self.t0 + n * self.dt, r["L"], r["dlnA"], r["J"], r["work"], r["tape"])
            fa, ta = htr.tape_switches(self.ctx, runs[0]["tape"])
            fb, tb = htr.tape_switches(self.ctx, runs[1]["tape"])
            nflag += int((fa != fb).sum())
            nteno += int((ta != tb).sum())
        htr.htr_check(self.ctx)
        return float(runs[0]["J"].item()), float(runs[1]["J"].item()), nflag, nteno

    def backward(self, theta, ckpts, Jbar=1.0):
        """(dJ/dtheta, dJ/dU0) by the discrete adjoint."""
        L = self._laser_for(theta)
        dlnA = theta[4:].detach().contiguous()
        Ubar = torch.zeros_like(self.U0)
        pbar = torch.zeros(self.nth, dtype=torch.float64, device=self.U0.device)
        J = torch.zeros(1, dtype=torch.float64, device=self.U0.device)
        kept = self._kept if (getattr(self, "_kept", None) and self._kept[0] is ckpts) else None
        for (n0, Uc, Tc) in reversed(ckpts):
            n1 = min(n0 + self.K, self.nsteps)
            if kept is not None and n0 == kept[1]:
                # the forward pass kept this segment's states and tapes
                T = kept[2].clone()
            else:
                U, T = Uc.clone(), Tc.clone()
                # re-run the segment, keeping each step's start state, stage
                # states and tape (per-cell fields, T and sensor flags per stage)
                for i, n in enumerate(range(n0, n1)):
                    self.seg_states[i].copy_(U)
                    self._step(U, T, self.t0 + n * self.dt, L, dlnA, J, self.seg_stages[i], self.seg_tapes[i])
            for i in reversed(range(n1 - n0)):
                n = n0 + i
                htr.htr_rk3_step_adjoint(self.ctx, self.seg_states[i], self.seg_stages[i], T, self.t0 + n * self.dt,
                                         self.dt, L, dlnA, Jbar, Ubar, pbar, self.adj_work, self.seg_tapes[i])
        htr.htr_check(self.ctx)
        return pbar, Ubar


class HeatReleaseObjective(torch.autograd.Function):
    """J = HeatReleaseObjective.apply(theta, problem); J.backward() fills
    theta.grad with dJ/dtheta from the discrete adjoint."""

    @staticmethod
    def forward(ctx, theta, problem):
        J, ckpts = problem.forward(theta, keep_last=True)
        ctx.problem = problem
        ctx.ckpts = ckpts
        ctx.save_for_backward(theta)
        return J.reshape(())

    @staticmethod
    def backward(ctx, gJ):
        (theta,) = ctx.saved_tensors
        pbar, _ = ctx.problem.backward(theta, ctx.ckpts, Jbar=float(gJ))
        return pbar.to(theta.dtype), None
