"""CPU oracle for the HPS Helmholtz hot path (TEST INFRASTRUCTURE ONLY).

This package is the plain, slow, obviously-correct FP64 reference that the GPU
library is checked against.  It is test infrastructure: only the test suite,
the smoke entry point and the CPU-baseline leg of the benchmark may import it.
The product path (the C-ABI library and its Python binding) never imports,
links or executes anything in here, and this package never imports the
product path.

What it computes (paper sections cited per function):

* the forward scattering problem of Section 1 / Section 2: the total field
  solves Delta u + k^2 (1 - q) u = 0 inside the square Omega, coupled to the
  radiating exterior through Green's formula (Remark in Section 2), with plane
  wave incidence and the scattered field sampled on the circle of radius R;
* the Frechet derivative (Theorem 1) and its adjoint (Theorem 2, discrete
  transpose), the band-limited sine model (eq. sineseries, Section 3.2) and
  one Gauss-Newton step on the normal equations (eq. normaleq, Section 3.3).

The discrete system is assembled in full as one sparse matrix and solved by
SuperLU; the fast hierarchical solver reproduces that same system, so the two
must agree to rounding.  Pins (closed forms, invariants, brute force) live in
tests/test_oracle_*.py.  Parity status per function is listed in the module
docstrings.
"""
