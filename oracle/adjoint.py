"""Reverse mode of the time stepper: adjoint solves and the gradient of a
real loss of the final state with respect to u^0 and a real potential V.

Test infrastructure only (see the package docstring).

Gradients of a real L with respect to a complex z follow the convention
g_z = dL/dRe z + i dL/dIm z, so that dL = Re(g_z^H dz).

One three-level step (Sec. 2.1, 2.2) computes x = A^{-1} b with
A = D - T_d + iI, b = B u_prev, B = iI + T_d - D and D = dt (rho |u_cur|^2 + V).
From dx = A^{-1}(db - dA x), with lam = A^{-H} g_x:
    dL = Re(lam^H db) - Re(lam^H dD x),
so g_b = lam, and through b = B u_prev (dB = -dD):
    g_u_prev += B^H lam = (-iI + T_d - D) lam,
    g_D       = -Re(conj(lam) x) - Re(conj(lam) u_prev),
and through D = dt (rho |u_cur|^2 + V) (d|u|^2 = 2 Re(conj(u) du)):
    g_u_cur += 2 dt rho g_D u_cur,    g_V += dt g_D.
A is complex symmetric (T_d real symmetric, D real diagonal), so
A^H = conj(A) and lam = conj(A^{-1} conj(g_x)): the adjoint solve is the
forward solver on conjugated data.  The starter (dt/2, T_d/2,
u_prev = u_cur = u^0) is the same step with both contributions on u^0.
"""
from __future__ import annotations

import numpy as np

from . import system, stepping


def step_adjoint(alpha, rho, n, mu_, tau, u_prev, u_cur, u_next, g_next, V=None, **kw):
    """Contributions (g_u_prev, g_u_cur, g_V) of one step, given g_next."""
    D = system.diagonal_D(rho, tau, u_cur, V)
    sol, info = stepping.solve_system(alpha, n, mu_, D, np.conj(g_next), **kw)
    lam = np.conj(sol)
    g_D = -(np.conj(lam) * u_next).real - (np.conj(lam) * u_prev).real
    g_prev = -1j * lam + system.apply_T(alpha, n, mu_, lam) - D * lam
    g_cur = 2.0 * tau * rho * g_D * u_cur
    g_V = tau * g_D
    return g_prev, g_cur, g_V, info


def first_step_adjoint(alpha, rho, n, mu_, tau, u0, u1, g1, V=None, **kw):
    """Contributions (g_u0, g_V) of the starter u^1 = first_step(u^0)."""
    g_prev, g_cur, g_V, info = step_adjoint(alpha, rho, n, 0.5 * mu_, 0.5 * tau, u0, u0, u1, g1, V, **kw)
    return g_prev + g_cur, g_V, info


def rollout(alpha, rho, n, mu_, tau, u0, V, steps, **kw):
    """States u^0 .. u^steps of the starter and steps - 1 three-level steps."""
    states = [u0]
    u1, _ = stepping.first_step(alpha, rho, n, mu_, tau, u0, V, **kw)
    states.append(u1)
    for _ in range(1, steps):
        un, _ = stepping.step(alpha, rho, n, mu_, tau, states[-2], states[-1], V, **kw)
        states.append(un)
    return states


def rollout_grad(alpha, rho, n, mu_, tau, states, V, g_final, **kw):
    """(g_u0, g_V) of a loss whose gradient with respect to the last state is
    g_final, by the steps' adjoints in reverse order."""
    N = len(states) - 1
    g = [np.zeros_like(states[0]) for _ in range(N + 1)]
    g[N] = g[N] + g_final
    g_V = np.zeros(states[0].shape)
    for k in range(N - 1, 0, -1):   # step k maps (u^{k-1}, u^k) to u^{k+1}
        gp, gc, gv, _ = step_adjoint(alpha, rho, n, mu_, tau, states[k - 1], states[k], states[k + 1], g[k + 1],
                                     V, **kw)
        g[k - 1] += gp
        g[k] += gc
        g_V += gv
    g0, gv, _ = first_step_adjoint(alpha, rho, n, mu_, tau, states[0], states[1], g[1], V, **kw)
    return g[0] + g0, g_V + gv
