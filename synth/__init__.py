"""Seeded synthetic problem generators.

This module builds the *inputs* of a 3D SIMP compliance problem on a
structured hexahedral grid: grid sizes, material constants, the per-element
passive mask, the list of fixed degrees of freedom and the nodal load vector,
plus seeded random vectors used as operator inputs in tests.  It contains none
of the method's arithmetic (no stiffness, no filter, no solve, no update) and is
the only module shared by the CPU oracle and the HIP path.

Conventions (the paper leaves numbering open; these are fixed here):

* element ``e = i + nelx*(j + nely*k)`` for ``0 <= i < nelx`` etc.
* node    ``n = i + (nelx+1)*(j + (nely+1)*k)``
* degree of freedom ``dof = 3*n + c``, ``c`` in {0: x, 1: y, 2: z}
* axis y points up; "bottom" means ``j = 0``; the clamped face is ``i = 0``.
* mask codes: 0 design element, 1 passive void (density fixed 0),
  2 passive solid (density fixed 1).
"""

from .problems import (  # noqa: F401
    Problem,
    cantilever,
    config_small,
    config_obstacle,
    config_large,
    config_paper_benchmark,
    random_problem,
    batch_problems,
    random_vector,
    random_density,
)
from .meshes import box_mesh, sphere_mesh, random_voxels  # noqa: F401,E402
