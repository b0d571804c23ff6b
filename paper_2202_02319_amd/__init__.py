"""MI355X (gfx950) HIP implementation of the explicit reacting-flow RHS of
arXiv 2202.02319 (TENO6/central convective fluxes, mixture-averaged
diffusion, Arrhenius chemistry, laser source, SSP-RK3), exposed through the
C interface in include/htr.h and the thin binding in `htr`."""
