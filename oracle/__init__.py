"""CPU FP64 oracle for the tau-preconditioned GMRES solver of the Riesz
fractional nonlinear Schroedinger linear systems.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import or call this package.  The product
(the HIP library and its Python binding) never imports it and shares no code
with it: this is a plain, slow, obviously-correct restatement of the paper's
definitions (dense per-axis Toeplitz and sine-transform matrices, the
preconditioner inverse written out in its eigenbasis, a textbook GMRES loop),
written to check the GPU path against.

Modules
-------
fcd       coefficients c_k (Sec. 2.1), the Toeplitz matrix T_1 (Sec. 2.1),
          the Hankel correction and tau-matrix (Sec. 4), the sine transform S
          and the tau eigenvalues.
system    d-level operators: T_d as a Kronecker sum (Sec. 2.2), the diagonal
          D, the system matrix A = D - T_d + iI, the scheme right-hand side,
          the complex form of the sine-transform TBAN preconditioner (Sec. 4),
          and dense builders of the real 2x2 block forms of Sec. 3 and 4.
gmres     right-preconditioned restarted GMRES with classical Gram-Schmidt
          applied twice and complex Givens rotations (Sec. 5 protocol).
stepping  the three-level linearly implicit schemes of Sec. 2 as repeated
          solves, the two-level starter and the discrete mass.
solver    OracleSolver: the same call sequence as the C ABI
          (assemble, precond_setup, solve, step, first_step).
adjoint   reverse mode of the stepper: adjoint solves and the gradient of a
          real loss of the final state with respect to u^0 and a potential V.

Parity status: every function is pinned by at least one CPU test in
tests/test_oracle_*.py against something other than itself (closed forms,
dense LU, library routines, brute force, paper bounds, the paper's printed
mass-error table).  None is "parity unpinned".
"""

from . import fcd, system, gmres, stepping, solver, adjoint  # noqa: F401
from .solver import OracleSolver  # noqa: F401
