"""The step that allocates nothing (htr_rk3_step_noalloc, scratch in a fixed
device array) against the step with caller work memory (htr_rk3_step) on the
same inputs: two calls in a row on the same GPU, the second on a smaller
grid, each compared bit for bit (same kernels) and with the oracle's steps
at the after-steps bar; an oversized grid is refused before device work."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from conftest import normwise
from gpu_util import both, dev, host
from paper_2202_02319_amd import _lib, htr

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-9


def _case(n, seed):
    # the 5-species, 4-reaction mechanism of the 1-D reacting workload,
    # whose seed keeps explicit RK3 stable at these temperatures
    c = synth.small_case(n=n, seed=seed, mech=synth.case_c1().mech)
    c.laser.t0 = 2e-8
    return c


def _steps(g, case, U0, nsteps, noalloc):
    U = dev(U0)
    T = dev(case.T)
    z = lambda: torch.zeros(1, dtype=torch.float64, device="cuda")  # noqa: E731
    t, dt, J = z(), z(), z()
    work = None if noalloc else g.new_work()
    for _ in range(nsteps):
        if noalloc:
            htr.htr_rk3_step_noalloc(g, U, T, t, dt, 1, case.laser, None, J)
        else:
            htr.htr_rk3_step(g, U, T, t, dt, 1, case.laser, None, work, J)
    htr.htr_check(g)
    return host(U), host(T), float(host(t)[0]), float(host(J)[0])


def _oracle_steps(o, case, U0, nsteps):
    U = U0.copy()
    T = case.T.copy()
    t, J = 0.0, 0.0
    for _ in range(nsteps):
        dt = o.stable_dt(U, T)
        J = o.rk3_step(U, T, t, dt, J=J)
        t += dt
    return U, J


@pytest.mark.parametrize("n,seed", [((21, 13, 9), 41), ((9, 7, 5), 42), ((37, 1, 1), 46)])
def test_noalloc_step_matches_step_with_work(n, seed):
    case = _case(n, seed)
    o, g = both(case)
    U0 = o.prim_to_cons()
    a = _steps(g, case, U0, 3, noalloc=False)
    b = _steps(g, case, U0, 3, noalloc=True)
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    Uo, Jo = _oracle_steps(o, case, U0, 3)
    err = normwise(b[0], Uo)
    assert err.max() <= STEP_TOL, err
    assert b[3] == pytest.approx(Jo, rel=STEP_TOL)


def test_noalloc_two_calls_in_a_row_second_smaller():
    # the second call reuses the array that still holds the first call's
    # (larger) contents
    big = _case((21, 13, 9), 43)
    small = _case((9, 7, 5), 44)
    runs = []
    for case in (big, small):
        o, g = both(case)
        U0 = o.prim_to_cons()
        runs.append((g, case, U0))
    got = [_steps(g, case, U0, 1, noalloc=True) for g, case, U0 in runs]
    ref = [_steps(g, case, U0, 1, noalloc=False) for g, case, U0 in runs]
    for x, y in zip(got, ref):
        for p, q in zip(x, y):
            assert np.array_equal(np.asarray(p), np.asarray(q))


def test_noalloc_refuses_oversized_grid():
    case = synth.small_case(n=(64, 48, 40), ns=9, nr=20, seed=45)   # 122,880 cells > the array
    g = htr.Context.from_case(case)
    U = torch.zeros((13, g.N), dtype=torch.float64, device="cuda")
    T = torch.full((g.N,), 1000.0, dtype=torch.float64, device="cuda")
    z = torch.zeros(2, dtype=torch.float64, device="cuda")
    L = g.lib
    st = L.htr_rk3_step_noalloc(g.h, C.c_void_p(U.data_ptr()), C.c_void_p(T.data_ptr()),
                                C.c_void_p(z.data_ptr()), C.c_void_p(z.data_ptr() + 8), 1, None, None, None, None)
    assert st == _lib.HTR_EINVAL
    assert b"HTR_NOALLOC_MAX_BYTES" in L.htr_last_error()
    assert float(T[0].item()) == 1000.0
