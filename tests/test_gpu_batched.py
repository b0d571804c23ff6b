"""Batched ensemble (uneven member grids, per-member laser energy, kernel
centre and ln A): one launch per kernel over all members must reproduce each
member's single-grid run bit for bit (same kernels, same operation order),
the captured HIP graph must reproduce eager stepping on every replay, and a
member must match the oracle."""
import numpy as np
import pytest
import torch

import synth
from conftest import normwise_state
from gpu_util import dev, host
from oracle import Oracle
from paper_2202_02319_amd import htr

pytestmark = pytest.mark.gpu

SIZES = [16, 24, 12, 20, 16]


@pytest.fixture(scope="module")
def ens():
    return synth.ensemble_c4(nmem=len(SIZES), sizes=SIZES)


def _ctx(e):
    return htr.Context(e.mech, e.members[0].grid)


def _single_steps(e, m, nsteps, dlnA=True):
    c = e.members[m]
    g = htr.Context(e.mech, c.grid)
    U = htr.cons_from_case(g, c)
    T = dev(c.T)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = g.new_work()
    dl = dev(e.dlnA[m]) if dlnA else None
    for _ in range(nsteps):
        htr.htr_rk3_step(g, U, T, t, dt, 1, c.laser, dl, work, J)
    htr.htr_check(g)
    return host(U), host(T), float(host(t)[0]), float(host(J)[0])


def _batch_setup(e, dlnA=True):
    ctx = _ctx(e)
    b = htr.Batch.from_cases(ctx, e.members, e.dlnA if dlnA else None)
    U, T = htr.batch_state_from_cases(b, e.members)
    z = lambda: torch.zeros(b.nmem, dtype=torch.float64, device="cuda")  # noqa: E731
    return ctx, b, U, T, z(), z(), z(), b.new_work()


def test_batched_steps_equal_single_runs(ens):
    ctx, b, U, T, t, dt, J, work = _batch_setup(ens)
    htr.htr_rk3_steps_batched(b, U, T, t, dt, 1, 3, work, J, use_graph=False)
    htr.htr_batch_check(b)
    Uh, Th, th, Jh = host(U), host(T), host(t), host(J)
    for m in range(b.nmem):
        Us, Ts, ts, Js = _single_steps(ens, m, 3)
        Ub = b.unpack(Uh, ctx.nv, m)
        assert np.array_equal(Ub, Us), (m, np.abs(Ub - Us).max())
        assert np.array_equal(b.unpack(Th, 1, m)[0], Ts)
        assert th[m] == ts and Jh[m] == Js


def test_batched_rhs_equal_single(ens):
    ctx, b, U, T, t, dt, J, work = _batch_setup(ens, dlnA=False)
    t.fill_(2e-8)
    out = torch.empty_like(U)
    htr.htr_rhs_batched(b, U, T, t, out)
    htr.htr_batch_check(b)
    oh = host(out)
    for m, c in enumerate(ens.members):
        g = htr.Context(ens.mech, c.grid)
        Um = htr.cons_from_case(g, c)
        om = torch.empty_like(Um)
        htr.htr_rhs(g, Um, dev(c.T), 2e-8, c.laser, om)
        htr.htr_check(g)
        assert np.array_equal(b.unpack(oh, ctx.nv, m), host(om))


def test_graph_replays_match_eager(ens):
    ctx, b, U, T, t, dt, J, work = _batch_setup(ens)
    U0, T0 = U.clone(), T.clone()
    htr.htr_rk3_steps_batched(b, U, T, t, dt, 1, 2, work, J, use_graph=False)
    htr.htr_batch_check(b)
    ref = (host(U), host(T), host(t), host(J))
    for rep in range(3):
        U.copy_(U0)
        T.copy_(T0)
        t.zero_()
        J.zero_()
        torch.cuda.synchronize()
        htr.htr_rk3_steps_batched(b, U, T, t, dt, 1, 2, work, J, use_graph=True)
        htr.htr_batch_check(b)
        got = (host(U), host(T), host(t), host(J))
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), rep
        _ = torch.randn(1000, device="cuda").sum().item()      # eager work between replays


def test_member_against_oracle(ens):
    ctx, b, U, T, t, dt, J, work = _batch_setup(ens)
    htr.htr_rk3_steps_batched(b, U, T, t, dt, 1, 2, work, J, use_graph=False)
    htr.htr_batch_check(b)
    m = 2
    c = ens.members[m]
    o = Oracle(c)
    Uo = o.prim_to_cons()
    To = c.T.copy()
    lnA = ens.mech.lnA + ens.dlnA[m]
    tt, Jo = 0.0, 0.0
    for _ in range(2):
        dto = o.stable_dt(Uo, To)
        Jo = o.rk3_step(Uo, To, tt, dto, lnA=lnA, J=Jo)
        tt += dto
    Ub = b.unpack(host(U), ctx.nv, m)
    rho_c = float(Uo[:o.ns].sum(axis=0).max() * o.cells(Uo, To.copy())[2].max())
    assert normwise_state(Ub, Uo, o.ns, rho_c).max() <= 1e-9
    assert float(host(J)[m]) == pytest.approx(Jo, rel=1e-9)


def test_member_max_per_member(ens):
    """The per-member maximum equals each member's slice maximum (exact: a
    maximum does not round), and accumulate keeps the larger of the two."""
    ctx, b, U, T, t, dt, J, work = _batch_setup(ens, dlnA=False)
    g = torch.Generator(device="cpu").manual_seed(7)
    f = torch.randn(b.N, generator=g, dtype=torch.float64).cuda()
    out = torch.empty(b.nmem, dtype=torch.float64, device="cuda")
    htr.htr_batch_member_max(b, f, out)
    ref = [float(f[b.offsets[m]:b.offsets[m + 1]].max()) for m in range(b.nmem)]
    assert host(out).tolist() == ref
    f2 = f - 0.5
    f2[b.offsets[2]:b.offsets[3]] += 10.0
    htr.htr_batch_member_max(b, f2, out, accumulate=True)
    ref2 = [max(ref[m], float(f2[b.offsets[m]:b.offsets[m + 1]].max())) for m in range(b.nmem)]
    assert host(out).tolist() == ref2
    htr.htr_batch_check(b)


def test_full_size_ensemble():
    """The ensemble workload at its full size (64 members, N^3 with N in
    {32, ..., 96}, 22M cells), in the benchmark's launch configuration
    (autotuned tiles per size class, graph replay):
    - one batched RHS against the oracle on windows (5-cell halo) of three
      members, one of them around its laser kernel, with each member's own
      ln A offsets;
    - three batched steps: the smallest member against the oracle's steps,
      the largest against its own single-grid run, bit for bit."""
    import dataclasses
    from conftest import flux_floor, rhs_close
    from gpu_util import sub_window
    e = synth.ensemble_c4()
    ctx = htr.Context(e.mech, e.members[0].grid)
    b = htr.Batch.from_cases(ctx, e.members, e.dlnA)
    U, T = htr.batch_state_from_cases(b, e.members)
    work = b.new_work()
    shapes, grid = htr.htr_batch_autotune(b, U, T.clone(), work)
    t_eval = e.members[0].laser.t0
    tt = torch.full((b.nmem,), t_eval, dtype=torch.float64, device="cuda")
    out = torch.empty_like(U)
    htr.htr_rhs_batched(b, U, T.clone(), tt, out)
    htr.htr_batch_check(b)
    Uh, got = host(U), host(out)
    sizes = [c.grid.n[0] for c in e.members]
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes)), 17]
    rng = np.random.default_rng(4)
    for k, m in enumerate(picks):
        c = e.members[m]
        mech_m = dataclasses.replace(e.mech, lnA=e.mech.lnA + e.dlnA[m])
        cm = synth.Case(c.name, mech_m, c.grid, c.Y, c.T, c.p, c.vel, laser=c.laser)
        n = c.grid.n
        if k == 0:
            lo = [int(np.argmin(np.abs(c.grid.xnode[a] - c.laser.center[a]))) - 4 for a in range(3)]
        else:
            lo = [int(rng.integers(0, n[a])) for a in range(3)]
        sub, flat, inner = sub_window(cm, lo, (8, 8, 8), 5)
        o = Oracle(sub)
        Um = b.unpack(Uh, ctx.nv, m)[:, flat]
        ref = o.rhs(Um, sub.T.copy(), t=t_eval)[:, inner]
        p = o.cells(Um, sub.T.copy())[1]
        ok, ratio = rhs_close(b.unpack(got, ctx.nv, m)[:, flat][:, inner], ref,
                              flux_floor(Um, p, float(c.grid.xin[0][0]), o.ns), rel=1e-12)
        assert ok, (m, ratio)
    # three steps in the benchmark's configuration
    z = lambda: torch.zeros(b.nmem, dtype=torch.float64, device="cuda")  # noqa: E731
    t, dt, J = z(), z(), z()
    U2, T2 = U.clone(), T.clone()
    htr.htr_rk3_steps_batched(b, U2, T2, t, dt, 1, 3, work, J, use_graph=True)
    htr.htr_batch_check(b)
    U2h = host(U2)
    ms, ml = picks[0], picks[1]
    c = e.members[ms]
    o = Oracle(c)
    Uo, To, to, Jo = o.prim_to_cons(), c.T.copy(), 0.0, 0.0
    for _ in range(3):
        dto = o.stable_dt(Uo, To)
        Jo = o.rk3_step(Uo, To, to, dto, lnA=e.mech.lnA + e.dlnA[ms], J=Jo)
        to += dto
    rho_c = float(Uo[:o.ns].sum(axis=0).max() * o.cells(Uo, To.copy())[2].max())
    assert normwise_state(b.unpack(U2h, ctx.nv, ms), Uo, o.ns, rho_c).max() <= 1e-9
    assert float(host(J)[ms]) == pytest.approx(Jo, rel=1e-9)
    c = e.members[ml]
    g = htr.Context(e.mech, c.grid)
    htr.htr_set_tiling(g, shapes[ml], 0)
    Ug, Tg = htr.cons_from_case(g, c), dev(c.T)
    z1 = lambda: torch.zeros(1, dtype=torch.float64, device="cuda")  # noqa: E731
    tg, dtg, Jg, wg = z1(), z1(), z1(), g.new_work()
    for _ in range(3):
        htr.htr_rk3_step(g, Ug, Tg, tg, dtg, 1, c.laser, dev(e.dlnA[ml]), wg, Jg)
    htr.htr_check(g)
    assert np.array_equal(host(Ug), b.unpack(U2h, ctx.nv, ml))
    assert float(host(Jg)[0]) == float(host(J)[ml])


def test_graph_replay_follows_scheme_changes(ens):
    """The captured graph bakes the scheme into its kernel arguments: after
    htr_set_flags the next replay must run the new scheme, bit for bit as
    eager stepping does (a stale graph would keep the old one)."""
    ctx, b, U, T, t, dt, J, work = _batch_setup(ens)
    U0, T0 = U.clone(), T.clone()
    results = {}
    for flags in (0, synth.FORCE_TENO, synth.FORCE_CENTRAL | synth.CHEM_OFF, 0):
        ctx.set_flags(flags)
        runs = []
        for graph in (True, False):
            U.copy_(U0)
            T.copy_(T0)
            t.zero_()
            dt.zero_()
            J.zero_()
            htr.htr_rk3_steps_batched(b, U, T, t, dt, 1, 2, work, J, use_graph=graph)
            htr.htr_batch_check(b)
            runs.append((host(U), host(J)))
        assert np.array_equal(runs[0][0], runs[1][0]), flags
        assert np.array_equal(runs[0][1], runs[1][1]), flags
        results.setdefault(flags, []).append(runs[0][0])
    # the schemes really differ, and going back to a scheme reproduces it
    assert not np.array_equal(results[0][0], results[synth.FORCE_TENO][0])
    assert not np.array_equal(results[0][0], results[synth.FORCE_CENTRAL | synth.CHEM_OFF][0])
    assert np.array_equal(results[0][0], results[0][1])


def test_multifidelity_co_processing_matches_separate_runs():
    """An HF grid (the 64^3 mixing layer) and an LF ensemble (16 members of
    16^3) advanced at once on two streams end bit for bit where each run
    alone ends."""
    from paper_2202_02319_amd.multifidelity import Fidelities, co_process
    hf_case = synth.case_c5()
    e = synth.ensemble_c4(nmem=16, sizes=[16] * 16)
    fid = Fidelities(hf_case, e.members, e.dlnA)
    fid.reset()
    fid.hf_steps(3)
    torch.cuda.synchronize()
    hf_alone = fid.hf_U.clone()
    fid.reset()
    fid.lf_steps(6)
    torch.cuda.synchronize()
    lf_alone = fid.lf_U.clone()
    fid.reset()
    fid.hf_steps(3)
    fid.lf_steps(6)
    torch.cuda.synchronize()
    fid.check()
    assert torch.equal(fid.hf_U, hf_alone)
    assert torch.equal(fid.lf_U, lf_alone)
    run = co_process(fid, 3, 6)
    print(f"HF {run.hf_ms:.2f} ms, LF {run.lf_ms:.2f} ms, both {run.both_ms:.2f} ms, overlap {run.overlap():.2f}")
    assert run.both_ms > 0
