"""Seeded synthetic inputs shared by the GPU path's tests and by the oracle.

This package holds geometry generators (meshes of curved 6-node or flat 3-node triangles),
seeded random vectors and seeded request streams (sizes, shapes, draws)
only.  It contains none of the boundary element
method's arithmetic: no shape-function evaluation, no quadrature, no Green's
function, no tree.  Both sides of every parity test take their meshes and
input vectors from here and compute everything else on their own.
"""

from .meshes import (  # noqa: F401
    Mesh,
    icosphere,
    geodesic_sphere,
    cube,
    ellipsoid,
    linear,
    workload,
    WORKLOADS,
)
from .vectors import random_vector, random_directions  # noqa: F401
from .requests import request_stream, mesh_of  # noqa: F401
