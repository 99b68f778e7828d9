"""Plain FP64 CPU oracle for the surface-source subproblem.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product path (the HIP library
and its Python binding) never calls it, and it shares no code with that path:
the only common module is ``inputs`` (seeded problem descriptions, models and
wavelets), which holds none of the method's arithmetic.

Modules, each citing the passage of W. W. Symes, "Efficient Computation of
Extended Surface Sources" (arXiv 2203.16573) that it follows:

* ``fd``     staggered first-derivative operators (Numerical Examples:
             staggered scheme of order 2 in time, 2k in space);
* ``grid``   padded grid, PML profiles, line sampling (same passage);
* ``prop``   forward time stepping and its exact transpose (Operators
             section; Appendix A), with constant density or a density
             array (the operators carry both kappa and rho);
* ``cengine`` the same time stepping as plain C loops (``cprop.c``,
             constant density), bitwise equal to ``prop``, for the
             full-length runs of the large grids;
* ``ops``    F, F^T, the penalty A, the thin-slab preconditioner, the normal
             operator and Algorithm 1, the weighted normal equations with
             their data- and model-space weights, V, the time-reversal
             inverse, Lambda~ and the misfit gradient in kappa
             (Introduction; Time Reversal; Unitarity;
             Accelerated Iterative Inversion; Computing and Symmetrizing
             Lambda);
* ``greens`` the closed-form 2D point-source response used as a pin;
* ``prop3``  the 3D time stepping (planes of sources and receivers,
             constant density) and its exact transpose (Operators section;
             the 3D generalisation among the closing remarks), pinned by
             exact reduction to ``prop`` on y-invariant problems, the dot
             test, energy conservation and the closed-form 3D point-source
             response;
* ``ops3``   the 3D subproblem: F, F^T, the penalty with the lateral
             distance on the source plane, the thin-slab W^-1 and M^-1,
             N and Algorithm 1 (``ops.pcg``), pinned by exact reduction of
             W^-1 to the 2D one on y-invariant input, its symmetry, a dense
             solve and the Krylov minimisation property of the iterates.

Every function is pinned by the CPU tests against facts that do not come
from this code: the dot-product adjoint test, brute-force dense transposes,
discrete energy conservation, reciprocity, the closed-form Green's function at
second-order convergence, the 1D plane-wave amplitudes (including the
energy transmission coefficient that the weighted composition and the
time-reversal inverse reduce to, and the exact 1D form of the sv relation),
polynomial exactness of the stencils, dense normal-equation solves, the
gradient of the weighted objective, central differences of the misfit in
kappa and Krylov-subspace optimality; with variable density, the dot test,
energy conservation and the reflection and transmission coefficients of a
density-only impedance jump at second order.  The C engine is pinned by
equality with ``prop`` on every operator and by its own dot test.
"""
from . import fd, grid, prop, ops, greens, prop3, ops3  # noqa: F401
from .ops import (Model, pcg, pcg_solve, precond, penalty, dscale, normal,  # noqa: F401
                  normal_w, pcg_solve_w, misfit_gradient, normal_v, pcg_solve_v)
