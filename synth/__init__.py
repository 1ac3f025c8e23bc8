"""Seeded synthetic inputs for the complex Helmholtz Krylov path.

This package generates inputs only: P1 tetrahedral meshes of a box, element
stiffness/mass assembly into CSR, symmetric Dirichlet elimination, sound-speed
blocks and right-hand sides, all from fixed seeds.  It contains none of the
solver path's arithmetic (sparse products, reductions, Krylov recurrences).
Both the CPU oracle and the HIP path consume what it produces; neither is
imported here.
"""
from .helmholtz import (  # noqa: F401
    OFFSETS, Mesh, make_mesh, assemble, FEProblem, build_problem, complex_rhs,
    helmholtz_values, block_mass_lists, tets_by_block,
)
from . import configs  # noqa: F401
