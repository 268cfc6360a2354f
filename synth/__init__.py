"""Seeded synthetic inputs shared by the CPU oracle and the GPU tests/bench.

This module defines *problems* (mesh size, split rule, material and SIMP
parameters, Dirichlet masks, nodal load vectors) and *fields* (density and
vector samples).  It holds none of the method's arithmetic: no stiffness,
no solve, no sensitivity, no filter and no optimality-criteria step.

Layout convention (shared interface, stated once here):

* nodes of a structured grid with ``nel = (nx, ny[, nz])`` unit cells are
  numbered x-fastest: ``n = j*(nx+1) + i`` in 2D and
  ``n = (k*(ny+1) + j)*(nx+1) + i`` in 3D;
* nodal vectors are structure-of-arrays ``v[r][c][n]`` (load case r,
  component c, node n), contiguous in n;
* the Dirichlet mask is ``fixed[c][n]`` (uint8, nonzero = fixed);
* the density is one value per simplex cell, ``e = 2*(j*nx+i) + t`` in 2D
  and ``e = 6*((k*ny + j)*nx + i) + t`` in 3D.
"""

from .problems import (  # noqa: F401
    Problem,
    cantilever2d,
    cantilever2d_hole,
    propped_cantilever2d,
    mbb2d,
    cantilever3d,
    bar2d,
    bar3d,
    batch2d,
    learned3d,
    n_nodes,
    n_cells,
    node_id,
)
from .fields import rho_uniform, rho_random, rho_smooth, vec_random  # noqa: F401
from .umesh import UProblem, jittered_cantilever, from_structured  # noqa: F401
