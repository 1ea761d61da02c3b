"""CPU pins of the oracle's reverse mode: gradients of a loss of the final
state against central finite differences of the oracle's own forward run
(so a dropped term, a wrong sign or a missing conjugate in the adjoint
formulas fails), on tiny grids with tight solves."""
import numpy as np
import pytest

from oracle import adjoint, fcd, system
from paper_2410_03643_amd import inputs

TOL = 1e-14


def setup(d, n, seed):
    lo, hi = -4.0, 4.0
    h = (hi - lo) / (n + 1)
    rng = np.random.default_rng(seed)
    u0 = inputs.soliton(d, n, lo, hi, noise=0.05, seed=seed)
    V = 0.3 * rng.standard_normal(u0.shape)
    target = u0 + 0.1 * (rng.standard_normal(u0.shape) + 1j * rng.standard_normal(u0.shape))
    return h, u0, V, target, rng


def loss(alpha, rho, n, mu, tau, u0, V, steps, target):
    st = adjoint.rollout(alpha, rho, n, mu, tau, u0, V, steps, tol=TOL)
    r = st[-1] - target
    return float(np.vdot(r, r).real), st


@pytest.mark.parametrize("d,n,steps", [(1, 7, 1), (1, 7, 4), (2, 3, 3), (1, 15, 5)])
def test_rollout_gradient_matches_finite_differences(d, n, steps):
    alpha, rho, tau = 1.5, 2.0, 0.05
    h, u0, V, target, rng = setup(d, n, seed=d * 100 + n)
    mu = fcd.mu(alpha, h, tau)
    L0, st = loss(alpha, rho, n, mu, tau, u0, V, steps, target)
    g_final = 2.0 * (st[-1] - target)          # L = |u^N - t|^2
    g_u0, g_V = adjoint.rollout_grad(alpha, rho, n, mu, tau, st, V, g_final, tol=TOL)
    eps = 1e-6
    for trial in range(3):
        du = rng.standard_normal(u0.shape) + 1j * rng.standard_normal(u0.shape)
        dV = rng.standard_normal(u0.shape)
        Lp, _ = loss(alpha, rho, n, mu, tau, u0 + eps * du, V + eps * dV, steps, target)
        Lm, _ = loss(alpha, rho, n, mu, tau, u0 - eps * du, V - eps * dV, steps, target)
        fd = (Lp - Lm) / (2 * eps)
        ad = float(np.vdot(g_u0, du).real) + float(np.sum(g_V * dV))
        assert abs(fd - ad) <= 1e-6 * max(abs(fd), 1e-3), (trial, fd, ad)


def test_adjoint_solve_is_the_conjugate_transpose_solve():
    """lam = conj(A^{-1} conj(g)) solves A^H lam = g (dense check)."""
    d, n, alpha, rho, tau = 2, 3, 1.4, 2.0, 0.05
    h, u0, V, target, rng = setup(d, n, seed=7)
    mu = fcd.mu(alpha, h, tau)
    D = system.diagonal_D(rho, tau, u0, V)
    A = system.dense_A(alpha, n, mu, d, D.ravel())
    g = rng.standard_normal(u0.shape) + 1j * rng.standard_normal(u0.shape)
    u_next = u0 * 0.9
    gp, gc, gv, _ = adjoint.step_adjoint(alpha, rho, n, mu, tau, u0, u0, u_next, g, V, tol=TOL)
    lam = np.linalg.solve(A.conj().T, g.ravel())
    # g_prev = B^H lam with B = iI + T - D
    T = system.dense_T(alpha, n, mu, d)
    B = 1j * np.eye(n ** d) + T - np.diag(D.ravel())
    assert np.allclose(gp.ravel(), B.conj().T @ lam, rtol=1e-10, atol=1e-12)
    gD = -(np.conj(lam) * u_next.ravel()).real - (np.conj(lam) * u0.ravel()).real
    assert np.allclose(gv.ravel(), tau * gD, rtol=1e-10, atol=1e-12)
