"""Plain, slow, FP64 CPU oracle for the contour-integral Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  This package is the correctness reference that the
HIP path is checked against.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product library never does,
and the two share no code (only the seeded input generators in `workloads`).

Everything here is NumPy/SciPy in float64 / complex128 and follows the paper
(Liu, Xi, Saad, de Hoop, "Solving the 3D high-frequency Helmholtz equation
using contour integration and polynomial preconditioning") step by step:

  operator   -- the test matrix A = S - M - iD of Sec. 7.1 (eq. stiff-mass),
                7-point stencil and an explicitly assembled sparse copy;
                the spectrum rectangle of Lemma 3.1.
  contour    -- quadrature poles and weights of Sec. 6.1-6.2 (eq. ellipse,
                eq. quad-points, eq. quad-radius) and the rational filter.
  polynomial -- exponential-Taylor residual polynomial (eq. exp-taylor), the
                convergence-rate objective (eq. fix-pt-conv) and the delta
                search of Sec. 4.2; Thm 4.1's closed form for q = 1.
  fixed_point-- the polynomial fixed-point iteration, eq. fix-pt-exp.
  fci        -- Algorithm 1 (FCI).
  krylov     -- flexible GMRES (the Krylov wrapper of Sec. 2) with classical
                Gram-Schmidt applied twice and Givens rotations; plain GMRES.
  spectral   -- the Fourier-spectral operator of Sec. 7.1 (eq. eig-Laplacian-spectral).
  laplacian  -- the regularised sine-transform inverse of the discrete Laplacian,
                the inner preconditioner of Alg. 1 step 4 (Sec. 6.3).
  case_two   -- the double-size formulation of eq. mat-2x2 (B = iC - I), its
                spectrum box from Thm 3.2 and the remark after it, and FGMRES
                with FCI on it.
  conv       -- direct-loop 3D convolution forward/backward for the learned
                preconditioner extension (not part of the paper).

Parity status of each function is stated in its module header.
"""
from . import operator, contour, polynomial, fixed_point, fci, krylov, conv, case_two, laplacian, spectral  # noqa: F401
