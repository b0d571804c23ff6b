"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  Draws numbers only; evaluates none of the method's formulas."""
from .mechanism import Mechanism, make_mechanism, single_species  # noqa: F401
from .cases import (  # noqa: F401
    Case, Ensemble, Grid, Laser, CHEM_OFF, VISC_OFF, FORCE_CENTRAL, FORCE_TENO, WENO3Z,
    BC_PERIODIC, BC_WALL, BC_INFLOW, BC_OUTFLOW,
    uniform_grid, stretched_grid, CurvGrid, as_curvilinear, affine_grid, rotation, skewed_grid, wavy_grid,
    vortex_case_curv, tgv2d_case, case_c1, case_c2, case_c3, case_c5, ensemble_c4, ignition_base,
    sod_case, vortex_case, vortex_exact, small_case, mixing_layer,
)
