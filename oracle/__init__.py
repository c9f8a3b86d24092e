"""Plain FP64 CPU oracle for the fluctuating boundary integral method (FBIM).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package; only the test-suite, the smoke
check of the entry script and the CPU-baseline leg of the benchmark use it.
It shares no code with the HIP library: kernels, quadrature rules, special
functions, parameter rules and solvers are all written here independently,
in slow, obviously-correct form, from Bao, Rachh, Keaveny, Greengard and
Donev, "A fluctuating boundary integral method for Brownian suspensions"
(J. Comput. Phys. preprint, arXiv:1709.01480).

Modules
  special  exponential integral E1 (textbook series / continued fraction)
  alpert   Alpert hybrid Gauss-trapezoid rules for log singularities,
           derived from the moment system; Lagrange interpolation weights
  fbim     geometry, Ewald-split Stokeslet kernels, dense single-layer
           matrix, saddle-point mobility, Brownian velocity, EM-RFD step
  direct   O(N^2) real-space and direct k-space sums in plain C (OpenMP)
           for sizes where dense numpy assembly is too large

Functions whose result is pinned only by consistency (no closed form or
printed value) say "parity unpinned" in their docstring.
"""
