"""CPU FP64 oracle for the 3D SIMP compliance loop -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct NumPy/SciPy implementation of
what one SIMP iteration computes (PyTopo3D, arXiv 2504.05604):

* ``ke``     -- the 8-node hexahedron stiffness matrix (Finite Element Analysis
               section), by 2x2x2 Gauss quadrature of B^T D B;
* ``fem``    -- global assembly COO -> CSR, Dirichlet elimination, direct solve,
               compliance and element energies (Finite Element Analysis and
               Optimality Criteria sections);
* ``filt``   -- the cone-weight filter matrix H and its forward/adjoint/sensitivity
               applications (Sensitivity Filtering section);
* ``oc``     -- the OC update with move limits and the volume multiplier found
               exactly (breakpoint search) and by bisection (Optimality Criteria
               section);
* ``simp``   -- one SIMP iteration and a trajectory in the order of the Workflow
               section;
* ``mg``     -- the multigrid building blocks (trilinear transfer, rediscretised
               coarse operators, damped-Jacobi / Chebyshev smoothing, V-cycle) that
               the accelerated solver uses as a preconditioner; these are not in
               the paper, they are the accelerated path's own method, written
               here in plain form so its pieces can be checked.

It shares no code with the HIP library and imports nothing from it.  Only the
test-suite, the package smoke check and the benchmark's CPU-baseline leg may
import it; the product path never calls it.
"""
