"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only builds geometry (vertex and triangle arrays with region
labels), incidence-angle lists and seeded random vectors.  It holds none of the
method's arithmetic: no basis functions, Green's functions, quadrature or
solver steps.  Both the plain CPU oracle and the HIP library consume its
outputs as plain arrays.
"""

from .meshes import (  # noqa: F401
    Body,
    icosphere,
    sphere_body,
    coated_sphere_body,
    ellipsoid_batch,
    stacked_cylinder_body,
)
from .excitation import (  # noqa: F401
    theta_sweep,
    random_complex_vector,
)
