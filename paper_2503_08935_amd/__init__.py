"""MI355X (gfx950) preconditioned Bi-CGSTAB for the 3D Poisson equation.

After Pennati et al., "A Parallel and Highly-Portable HPC Poisson Solver:
Preconditioned Bi-CGSTAB with alpaka" (arXiv 2503.08935). The solver lives in
the HIP library libpoisson.so behind the C ABI of include/poisson.h; this
package is its Python binding plus the seeded input generators.
"""
from ._binding import (ERR_ARG, ERR_BREAKDOWN, ERR_DEVICE, ERR_INTERNAL, ERR_NOMEM,  # noqa: F401
                       ERR_NONFINITE, ERR_UNSUPPORTED, EXPORTS, FP64, KERNEL_CHEB_PAIR, KERNEL_CHEB_STEP,
                       KERNEL_CHEB_TRIPLE, NOALLOC_SCRATCH_BYTES,
                       KERNEL_STENCIL_DOT, KERNEL_UPDATE_XR, MIXED, NOT_CONVERGED, OK, PC_BLOCK_JACOBI,
                       PC_CHEBYSHEV, PC_JACOBI, PC_NONE, PENDING, PoissonError, Server, Solver,
                       fill_uniform, footprint, lib, strerror)
