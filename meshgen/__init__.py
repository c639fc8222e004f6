"""Seeded synthetic inputs shared by the oracle and the GPU library.

This package only produces *inputs*: point coordinates, face/cell
connectivity, boundary patches with their prescribed values, material
parameters and solver settings.  It contains none of the method's
arithmetic (no face areas, centroids, gradients, stresses or residuals);
those are computed independently by ``oracle/`` and by the HIP library.

Mesh dictionary layout (OpenFOAM-style polyhedral description, used by
both sides):

``dim``          2 (plane strain, unit depth) or 3
``points``       float64 [n_points, dim]
``face_ptr``     int64   [n_faces + 1]   CSR offsets into ``face_pts``
``face_pts``     int32   [...]           polygon vertices (2-D: the two
                 edge end points), ordered so that the right-hand normal
                 points out of the owner cell
``owner``        int32   [n_faces]
``neighbour``    int32   [n_internal]    internal faces come first
``n_cells``      int
``patches``      list of dicts, boundary faces grouped contiguously:
                 ``name``, ``start`` (first face index), ``size``,
                 ``type`` in {"displacement", "traction", "pressure", "symmetry"},
                 ``value`` (3 floats: displacement, traction vector, or
                 pressure in value[0]), optional ``per_face`` [size, dim]
"""

from .structured import (box_mesh_2d, box_mesh_3d, annulus_mesh_2d,
                         set_patch, mesh_summary, renumber_cells, mirrored_box_pair)
from .configs import (config_c1, config_c2, config_c3, config_c4,
                      config_c5_stream, Material, cantilever_mesh)

__all__ = [
    "box_mesh_2d", "box_mesh_3d", "annulus_mesh_2d", "set_patch",
    "mesh_summary", "renumber_cells", "config_c1", "config_c2",
    "config_c3", "config_c4", "config_c5_stream", "Material",
    "cantilever_mesh", "mirrored_box_pair",
]
