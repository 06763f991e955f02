"""FP64 CPU oracle of the FE-LBM step.  Test infrastructure only: the
product path never imports it."""
from .felbm_oracle import (  # noqa: F401
    CS2, E, OPPOSITE, Q, W, Geometry, Matrices, Oracle, Params, SolverError, chemical_potential, collide,
    contact_angle, density, element_forces, element_gradient, equilibria, gamma, laplacian_C, laplacian_mu,
    moments, pcg, relaxation_time, rhs, wall_flux, wall_operator,
)
