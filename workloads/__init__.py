"""Seeded synthetic inputs (meshes, initial fields, wetting fields) shared by
the CPU oracle, the tests and the benchmark.  Geometry and input recipes only:
no lattice Boltzmann or finite element arithmetic lives here."""
from .mesh import Mesh, channel_mesh, graded_rows, split_grid_mesh, uniform_rows, unwrap_tri_xy  # noqa: F401
from .configs import (Physics, Workload, capillary_channel, config, droplet_field, fourier_field, free_droplet,  # noqa: F401
                      make_physics, wetting_drop, wetting_from_angles)
