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
           for sizes where dense numpy assembly is too large; the cell-list
           real-space sum and the Gaussian gridding of the fast path
  matfree  the Brownian step without assembling M (GMRES, Lanczos)
  fastpath the FP64 CPU fast path of the matvec (cell list, shared Alpert
           block, spectral Ewald) that the GPU is timed beside
  precond  the block-diagonal preconditioner and a plain GMRES
  philox   Philox4x32-10 and Box-Muller, the library's noise generator
  mlp      the learned correction's network, forward and backward

Functions whose result is pinned only by consistency (no closed form or
printed value) say "parity unpinned" in their docstring.
"""
