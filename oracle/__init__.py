"""CPU oracle for the SIMP iteration (test infrastructure, not product code).

A plain, slow, FP64 NumPy/SciPy implementation of every step of one SIMP
iteration of arXiv 2012.08208 ("A 55-line code for large-scale parallel
topology optimization in 2D and 3D"):

* ``mesh``  -- structured P1 simplex meshes built from explicit coordinates
  (Section 3.1 and Section 4.3.1; three-dimensional boxes, Section 5.1);
* ``fem``   -- element stiffness from coordinates, SIMP interpolation,
  assembly, Dirichlet elimination, direct solve, compliance and its
  sensitivity (Section 2, eq. str_energy, eq. simp; Section 3.1, eq.
  fe_form; Section 3.2, sensitivity of f);
* ``filt``  -- the distance-weighted sensitivity filter (Section 3.2.2,
  eq. filter and eq. filter_cond; Section 4.5, eq. filter_mat);
* ``oc``    -- the optimality-criteria update with bisection on the
  Lagrange multiplier (Section 3.2, eq. kkt and eq. update; Section 3.2.1);
* ``simp``  -- the iteration loop (Section 4.3-4.5 and the Appendix code);
* ``umesh`` -- the same loop on an arbitrary simplex mesh (Section 6.1),
  with the midpoint filter of Section 3.2.2 and Section 6.2;
* ``net``   -- the convolutional preconditioner network of this library
  (not in the paper): forward, backward, loss and Adam, in FP64 with
  optional BF16 rounding at the points where the kernels store.

Only ``tests/``, the entry module's ``smoke()`` and the CPU-baseline leg of
the benchmark may import this package.  It shares no code with the HIP
path and imports nothing from it.
"""

from . import mesh, fem, filt, oc, simp, umesh, net  # noqa: F401
