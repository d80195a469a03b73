"""Plain, slow CPU oracle for the TSL sign function and its gauge-link derivative.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (no kernels, headers, tables or helpers); the only common code is
the seeded input generator package ``synthetic``, which holds none of the
method's arithmetic.

Everything is float64 / complex128.  Modules:

* ``wilson``  -- Wilson-Dirac operator D_w(mu), H = g5 D_w (App. A, eq. WD_op/WD_G):
  a gather stencil (torch, differentiable in the links), an independent dense
  builder for tiny lattices and the free-field closed form;
* ``sign``    -- exact matrix sign (Schur, eigen-decomposition, Newton; Sec. 2,
  eq. spectral_form) and its Frechet derivative through Theorem 1;
* ``tsl``     -- plain two-sided Lanczos approximation of sgn(A)x (Sec. 2, the
  Krylov spaces of A and A^dagger started from the same x);
* ``grad``    -- derivative of S_k = Re<eta|TSL_k(H(U), psi)> with respect to all
  links by torch autograd, finite differences, the exact (Daleckii-Krein)
  gradient on tiny lattices and the U(1) Ward identity (Sec. 4.3);
* ``deflation`` -- deflated sign function with known eigenpairs (Sec. 3, App. E);
* ``constfield`` -- exact eigenpairs and sign of H on a gauge-rotated constant
  field (one 12 x 12 matrix per momentum), the deflation inputs at 16^4;
* ``tuning`` -- the tuning run that picks the Krylov sizes and its cross-check
  (Sec. 4.1).

Parity status of each function is stated in its docstring; every function is
pinned by ``tests/test_oracle_*.py`` against closed forms, identities or brute
force unless it says "parity unpinned".
"""
