"""The seeded workloads: shapes and sizes, and the explicit-stability screen
of their chemistry (the fastest pseudo-first-order destruction rate at the
workload's peak temperature times the initial stable step stays below one)."""
import numpy as np
import pytest

import synth
from oracle import Oracle


def _sub_block(case, m=16):
    n = case.grid.n
    sl = [min(m, v) for v in n]
    g = synth.uniform_grid(tuple(sl), case.grid.spacing())

    def cut(a):
        a = a.reshape(a.shape[:-1] + (n[2], n[1], n[0]))
        return a[..., :sl[2], :sl[1], :sl[0]].reshape(a.shape[:-3] + (-1,)).copy()
    return synth.Case(case.name, case.mech, g, cut(case.Y), cut(case.T), cut(case.p), cut(case.vel),
                      flags=case.flags)


def _stiffness(case, Tmax, dlnA=0.0):
    sb = _sub_block(case)
    o = Oracle(sb)
    dt = o.stable_dt(o.prim_to_cons(), sb.T.copy())
    mech = case.mech if not dlnA else synth.Mechanism(**{**case.mech.__dict__, "lnA": case.mech.lnA + dlnA})
    lam = 0.0
    for q in (0, sb.grid.N // 2, sb.grid.N - 1):
        hot = synth.Case("hot", mech, synth.uniform_grid((1, 1, 1), 1e-4), sb.Y[:, [q]].copy(), np.array([Tmax]),
                         np.array([101325.0]), np.zeros((3, 1)))
        oh = Oracle(hot)
        lam = max(lam, oh.destruction_rate(oh.prim_to_cons(), np.array([Tmax])).max())
    return lam * dt


@pytest.mark.parametrize("name,make,Tmax,dlnA", [
    ("C1", lambda: synth.case_c1(), 1500.0, 0.0),
    ("C2", lambda: synth.case_c2(n=32), 1200.0, 0.0),
    ("C3", lambda: synth.case_c3(n=(32, 32, 32)), 2000.0, 0.0),
    ("C4", lambda: synth.case_c3(n=(32, 32, 32)), 2000.0, 0.5),
    ("ignition", lambda: synth.case_c3(n=(32, 32, 32), ns=5, nr=4, mech_seed=synth.cases.IGNITION_MECH_SEED),
     2500.0, 0.0),
])
def test_chemistry_explicitly_stable(name, make, Tmax, dlnA):
    case = make()
    if name == "C2":     # same spacing as the 128^3 box
        full = synth.case_c2()
        case = _sub_block(full)
    assert _stiffness(case, Tmax, dlnA) < 1.0


def test_config_shapes():
    c1 = synth.case_c1()
    assert c1.grid.n == (256, 1, 1) and c1.mech.ns == 5 and c1.mech.nr == 4 and c1.steps == 200
    c2 = synth.case_c2(n=16)
    assert c2.mech.ns == 9 and c2.mech.nr == 20
    e = synth.ensemble_c4(nmem=6, sizes=[32, 40, 48, 32, 96, 56])
    assert [m.grid.n[0] for m in e.members] == [32, 40, 48, 32, 96, 56]
    assert e.dlnA.shape == (6, 20) and np.all(np.abs(e.dlnA) <= 0.5)
    E = [m.laser.E for m in e.members]
    assert max(E) / min(E) <= 1.3 / 0.7 + 1e-12
    full = synth.ensemble_c4()
    sizes = np.array([m.grid.n[0] for m in full.members])
    assert len(sizes) == 64 and set(sizes) <= set(range(32, 97, 8))


def test_mechanisms_are_element_balanced():
    for seed in range(5):
        m = synth.make_mechanism(9, 20, seed)
        dnu = m.nu_r - m.nu_f
        assert np.all(dnu @ m.elem.T == 0)
        assert np.all(m.nu_f.sum(axis=1) >= 1) and np.all(m.nu_f.sum(axis=1) <= 2)
        assert np.all(m.nu_r.sum(axis=1) >= 1) and np.all(m.nu_r.sum(axis=1) <= 2)
