"""Time stepping of the Riesz fractional NLS by repeated linear solves.

Test infrastructure only (see the package docstring).

* Three-level step (Sec. 2.1 LICD scheme, Sec. 2.2 TLID scheme): with
  D = rho dt |u^n|^2, solve (D - T_d + i I) u^{n+1} = (i I + T_d - D) u^{n-1}.
* Starter u^0 -> u^1: the paper only cites a second-order scheme for it.  The
  reading used here is one Crank-Nicolson step with the nonlinearity frozen at
  u^0, which is the same linear system with dt replaced by dt/2:
  (D' - T' + i I) u^1 = (i I + T' - D') u^0, T' = T_d/2, D' = rho (dt/2) |u^0|^2.
* Discrete mass Q^n = h^d (||u^{n+1}||^2 + ||u^n||^2) / 2.  With
  B = D - T_d real symmetric, u^{n+1} = -(B + iI)^{-1}(B - iI) u^{n-1} is a
  unitary (Cayley) map, so ||u^{n+1}|| = ||u^{n-1}|| and Q^n is conserved up
  to the solver tolerance (cf. the mass-error table of Sec. 5.1).
"""
from __future__ import annotations

import numpy as np

from . import system
from .gmres import pgmres


def solve_system(alpha, n, mu_, D, b, *, omega=1.0, **kw):
    A = lambda x: system.apply_A(alpha, n, mu_, D, x)  # noqa: E731
    P = lambda r: system.apply_precond_inverse(alpha, n, mu_, D, r, omega)  # noqa: E731
    return pgmres(A, P, b, **kw)


def step(alpha, rho, n, mu_, tau, u_prev, u_cur, V=None, **kw):
    D = system.diagonal_D(rho, tau, u_cur, V)
    b = system.scheme_rhs(alpha, n, mu_, D, u_prev)
    return solve_system(alpha, n, mu_, D, b, **kw)


def first_step(alpha, rho, n, mu_, tau, u0, V=None, **kw):
    return step(alpha, rho, n, 0.5 * mu_, 0.5 * tau, u0, u0, V, **kw)


def mass(h: float, u_next: np.ndarray, u_cur: np.ndarray) -> float:
    d = u_cur.ndim
    return h ** d * 0.5 * (float(np.vdot(u_next, u_next).real) + float(np.vdot(u_cur, u_cur).real))
