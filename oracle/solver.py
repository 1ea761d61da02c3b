"""OracleSolver: the C ABI's call sequence on the CPU oracle.

Test infrastructure only (see the package docstring).

assemble(alpha, rho, d, n, h, tau) -> precond_setup(u_cur[, V], omega) ->
solve(b) -> x, and step(u_prev, u_cur) -> u_next / first_step(u0) -> u1.
"""
from __future__ import annotations

import numpy as np

from . import fcd, system, stepping
from .gmres import pgmres


class OracleSolver:
    def __init__(self, alpha: float, rho: float, d: int, n: int, h: float, tau: float):
        self.alpha, self.rho, self.d, self.n, self.h, self.tau = alpha, rho, d, n, h, tau
        self.mu = fcd.mu(alpha, h, tau)
        self.D = None
        self.omega = 1.0

    # a2
    def precond_setup(self, u_cur: np.ndarray, V: np.ndarray | None = None, omega: float = 1.0):
        self.D = system.diagonal_D(self.rho, self.tau, u_cur, V)
        self.omega = omega
        return self.D

    # a3, a4
    def apply_A(self, x):
        return system.apply_A(self.alpha, self.n, self.mu, self.D, x)

    def apply_Pinv(self, r):
        return system.apply_precond_inverse(self.alpha, self.n, self.mu, self.D, r, self.omega)

    def rhs(self, u_prev):
        return system.scheme_rhs(self.alpha, self.n, self.mu, self.D, u_prev)

    # a5-a7
    def solve(self, b: np.ndarray, *, tol=1e-10, restart=30, maxit=2000, fixed_iters=0):
        return pgmres(self.apply_A, self.apply_Pinv, b, tol=tol, restart=restart,
                      maxit=maxit, fixed_iters=fixed_iters)

    # a9
    def step(self, u_prev, u_cur, V=None, **kw):
        self.precond_setup(u_cur, V)
        return self.solve(self.rhs(u_prev), **kw)

    def first_step(self, u0, V=None, **kw):
        return stepping.first_step(self.alpha, self.rho, self.n, self.mu, self.tau, u0, V, **kw)
