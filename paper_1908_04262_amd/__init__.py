"""mifoam: free-surface lattice Boltzmann foaming sweep on MI355X (gfx950).

The compute path is the HIP library libmifoam.so (C ABI in include/mifoam.h); this
package holds its sources (csrc/), its build script and a ctypes binding.
"""
from .mifoam import (  # noqa: F401
    EXPORTS, SWEEP_VARIANTS, Batch, CurvatureNet, MifoamError, Sim, generate_stencils, load_library, make_params,
    poisson_nuclei)
