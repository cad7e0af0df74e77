"""CPU FP64 oracle for matrix-free weighted quadrature (MF-WQ) and the Fast
Diagonalization preconditioner.  TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never calls it, and it imports nothing from the product: the two
share no kernels, headers, helpers, tables or constants.  The only shared module
is ``synth`` (seeded input definitions, no arithmetic of the method).

Plain, slow and written to be checked against the paper by eye:

* ``bspline``  Cox-de Boor B-splines and 1D Galerkin integrals (Section 2.1).
* ``wq``       quadrature points and weighted-quadrature weights
               (Section 2.2, eqs. exactness1d, weights-support, exactness_K).
* ``geometry`` spline map, Jacobian and the coefficient tensor C (eq. C).
* ``operator`` explicit sparse assembly of the WQ stiffness matrix
               (sum over alpha, beta of W D B, Section 3.2), the WQ mass
               matrix of the reaction term (eq. WDB) and plain matrix-free
               applies (Algorithms 1 and 2, eq. sum-factorization).
* ``fd``       Fast Diagonalization preconditioner (Section 4, by citation).
* ``krylov``   right-preconditioned BiCGStab (Section 4).
* ``adjoint``  gradients of J(u) = 1/2 |u - u_obs|^2 with respect to K and
               the reaction coefficient alpha at the quadrature points and to f.
* ``errors``   H1 / L2 errors against a manufactured solution.

Every function documents the passage it follows.  Readings of places where the
paper is silent or ambiguous are named R1..R10 in the docstrings; the same
readings are implemented (independently) by the library.  Every function is
pinned by tests/test_oracle_pins.py and tests/test_oracle_adjoint.py against
facts the paper or the mathematics fixes, or against a rebuild from the
definitions with independent library routines; none is "parity unpinned".
"""
