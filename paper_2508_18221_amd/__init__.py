"""MI355X (gfx950) coupled BSSN + Valencia GRMHD spectral RK stage.

The product is libgrmhd.so (HIP kernels + C-ABI, include/grmhd.h); this
package holds its sources (csrc/), the build step and a thin ctypes binding."""

from ._lib import load, GrmhdError, NFIELDS  # noqa: F401
from .solver import Solver, Server, step_batch, make_grid, make_phys  # noqa: F401
