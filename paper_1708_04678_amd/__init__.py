"""MI355X (gfx950) finite element lattice Boltzmann step for contact-line
dynamics (arXiv:1708.04678): HIP kernels behind a C ABI (include/felbm.h),
with a ctypes binding."""
from .felbm import (FIELDS, FP32, FP64, Context, Context3D, FelbmError, library_path, load_library,  # noqa: F401
                    validate_mesh)
