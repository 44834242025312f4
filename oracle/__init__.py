"""CPU oracle for the multiple-precision SpMV / BiCG / GPBiCG path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline leg
of the benchmark, never by the product path.  Plain Python integers and fractions, exact
arithmetic followed by one round-to-nearest-even per operation.  It shares no code with the GPU
library, its binding or the input generators.

Parity status of each function (what pins it, see tests/test_oracle_*.py):
  mpnum.round_scaled / round_fraction / mul / add / sub / div / sqrt : pinned (brute force at
      small p, mpmath at p bits, closed-form ties, carries and cancellations)
  spmv.spmv_exact / spmv_seq / transpose / grad_vals : pinned (Fraction sums, invariants, the
      rounding-error bound for sequential summation)
  blas.dot / axpy / xpby : pinned (Fraction definitions)
  krylov.bicg / gpbicg : pinned (recursive vs true residual, BiCG = CG on symmetric matrices,
      small systems against exact Gaussian elimination, forced breakdowns)
  krylov.cgs / bicgstab : pinned (small systems against exact Gaussian elimination, recursive
      vs true residual, BiCG's Lanczos coefficients, BiCGSTAB's r orthogonal to t, breakdowns)
  dense.gemv : pinned (Fraction sums, the sparse product of the same matrix without its zeros,
      integer rows summed exactly, the sequential-summation bound)
  ilu.ilu0 / lower_solve / upper_solve / apply, krylov.bicgstab_precond : pinned (L U = A on A's
      pattern, complete LU on tridiagonal matrices, rounded exact rows in EXACT mode, solve
      residual bounds, the identity preconditioner giving plain BiCGSTAB bit for bit, Gauss
      solutions of small systems)
"""
from . import blas, codec, dense, ilu, krylov, mpnum, spmv  # noqa: F401
