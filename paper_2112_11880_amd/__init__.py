"""MI355X-native complex Krylov path for finite-element Helmholtz systems.

The computation lives in libhk.so (hand-written HIP for gfx950, C ABI in
include/hk.h); this package is its Python binding.
"""
from .hk import (  # noqa: F401
    CSR, HKError, load, zdotc, zdotu, dznrm2, zaxpy, zscal, zaxmy, zcopy, zconj,
    krylov_solve, krylov_solve_mixed, sweep_solve, blockdiag_solve,
    SWEEP_SHAPES, BLOCKDIAG_SHAPES, HK_MIXED_LITERAL_INNER,
    HK_OK, HK_EINVAL, HK_NOT_CONVERGED, HK_BREAKDOWN, HK_NONFINITE, BD_NAMES,
)
from .adjoint import HelmholtzProblem, HelmholtzSolve, helmholtz_solve, assemble, elem_sens  # noqa: F401,E402
