"""Plain CPU FP64 oracle for the Jacobian-free Newton-Krylov path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library
and its Python binding) may import, call or execute anything in this
package; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
GPU path; both consume the same seeded inputs from ``meshgen``.

Every function follows a passage of Cardiff, Armfield, Tukovic &
Batistic, "A Jacobian-free Newton-Krylov method for cell-centred finite
volume solid mechanics" (arXiv 2502.17217), cited by section and
equation label.  The implementation is written for readability: numpy
vector operations over faces/cells, no blocking or fusion, and every
arithmetic routine accepts complex128 displacements so that exact
directional derivatives can be taken by the complex step.

Modules
  geometry  face area vectors, centroids, cell volumes/centroids
  fv        least-squares gradient, mechanical laws, face fluxes,
            Rhie-Chow term, residual
  jacobian  finite-difference and complex-step J.v, brute-force J,
            compact-stencil approximate Jacobian
  krylov    restarted (flexible) GMRES with classical Gram-Schmidt and
            re-orthogonalisation, right preconditioning
  newton    Newton-Raphson with equal load increments
"""

from .geometry import mesh_geometry
from .fv import residual, gradient, material_constants, prepare
from .jacobian import (jv_fd, jv_complex_step, eps_walker_pernice, brute_force_jacobian,
                       approximate_jacobian, approximate_jacobian_scalar)
from .krylov import gmres
from .newton import newton_solve, dynamic_solve

__all__ = ["mesh_geometry", "residual", "gradient", "material_constants", "prepare",
           "jv_fd", "jv_complex_step", "eps_walker_pernice", "brute_force_jacobian",
           "approximate_jacobian", "approximate_jacobian_scalar", "gmres", "newton_solve",
           "dynamic_solve"]
