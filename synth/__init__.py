"""Seeded synthetic inputs: closed triangle meshes and plane-wave excitations.

This package holds only input generation (geometry, random directions and
polarisations, random start vectors).  It contains none of the solver's
arithmetic and is shared by the tests, the benchmark, the oracle checks and
the GPU path alike.
"""

from .meshes import icosphere, graded_sphere, torus, cube, ellipsoid, mesh_summary  # noqa: F401
from .waves import plane_waves, default_plane_wave, complex_start  # noqa: F401
