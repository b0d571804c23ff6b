"""The oracle's pins catch plausible mistakes: each case below plants one
mistake in a copy of the oracle source (on the CPU), builds it, and checks
that the pins meant to see it fail on that build while the real oracle
passes them.  Planted: the species enthalpy transport of the heat flux
dropped or mis-signed, the viscous work formed with a node instead of the
face velocity, the viscous stress without its transposed-gradient term, the
correction flux of the species diffusion dropped (paper: Methods › Solver,
eqs. (3), (5), (6))."""
import numpy as np
import pytest

import oracle.oracle as oo
import synth
from test_oracle_bruteforce_full import check_whole_rhs
from test_oracle_energy import check_enthalpy_diffusion, check_viscous_heating


def _brute(flags=synth.FORCE_CENTRAL):
    return lambda: check_whole_rhs((3, 4, 5), ns=3, nr=2, seed=29, flags=flags)


def _species_fluxes_sum_to_zero():
    case = synth.small_case(n=(6, 5, 4), ns=4, nr=2, seed=9, flags=synth.CHEM_OFF | synth.FORCE_CENTRAL,
                            laser=False)
    case.vel[:] = 0.0
    o = oo.Oracle(case)
    U = o.prim_to_cons()
    d = o.rhs(U, case.T.copy())
    ns = case.mech.ns
    assert np.max(np.abs(d[:ns].sum(axis=0))) <= 1e-12 * np.max(np.abs(d[:ns]))


MUTANTS = {
    "enthalpy_transport_dropped": (
        [("    qn += Js[s] * hf[s];\n", "    qn += 0.0 * Js[s] * hf[s];\n")],
        [check_enthalpy_diffusion, _brute()]),
    "enthalpy_transport_sign": (
        [("    qn += Js[s] * hf[s];\n", "    qn -= Js[s] * hf[s];\n")],
        [check_enthalpy_diffusion, _brute()]),
    "viscous_work_node_velocity": (
        [("    work += tau[m] * 0.5 * (A.u[m] + B.u[m]);\n", "    work += tau[m] * A.u[m];\n")],
        [check_viscous_heating, _brute()]),
    "stress_without_transpose": (
        [("    tau[m] = mu * (grad[d][m] + grad[m][d]);\n", "    tau[m] = mu * (grad[d][m] + grad[d][m]);\n")],
        [check_viscous_heating, _brute()]),
    "correction_flux_dropped": (
        [("    Js[s] += Yf[s] * corr;\n", "    Js[s] += 0.0 * Yf[s] * corr;\n")],
        [_species_fluxes_sum_to_zero, _brute()]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    repl, checks = MUTANTS[name]
    for chk in checks:          # the real oracle passes every one of them
        chk()
    lib = oo.build_variant(repl, str(tmp_path), name=f"liboracle_{name}.so")
    with oo.use_library(lib):
        for chk in checks:
            with pytest.raises(AssertionError):
                chk()
