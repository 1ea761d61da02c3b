"""Pins for the d-level oracle operators and the preconditioner.

Brute-force loops, numpy.kron dense matrices, the real 2x2 block forms of
Sec. 3-4 built literally, Theorem 3.1 / 4.1 bounds and the exact special case
alpha = 2, rho = 0 (where the preconditioner equals the system matrix).
"""
import itertools

import numpy as np
import pytest

from oracle import fcd, system
from paper_2410_03643_amd import inputs


def brute_T(alpha, n, mu, x):
    """T_d x with explicit loops over every index (tiny grids)."""
    c = fcd.coefficients(alpha, n)
    d = x.ndim
    y = np.zeros_like(x)
    for idx in itertools.product(range(n), repeat=d):
        acc = 0j
        for ax in range(d):
            for k in range(n):
                src = list(idx)
                src[ax] = k
                acc += mu * c[abs(idx[ax] - k)] * x[tuple(src)]
        y[idx] = acc
    return y


@pytest.mark.parametrize("d,n", [(1, 13), (2, 5), (3, 4)])
@pytest.mark.parametrize("alpha", [1.3, 1.8])
def test_apply_T_matches_brute_force_and_kron(d, n, alpha):
    mu = 0.45
    x = inputs.random_field((n,) * d, seed=7)
    y = system.apply_T(alpha, n, mu, x)
    assert np.allclose(y, brute_T(alpha, n, mu, x), atol=1e-13)
    Td = system.dense_T(alpha, n, mu, d)
    assert np.allclose(y.ravel(), Td @ x.ravel(), atol=1e-13)


def test_kron_order_matches_paper_2d():
    """T_2 = I (x) T_x + T_y (x) I with x the fastest (last) index."""
    n, mu, alpha = 4, 0.3, 1.5
    T1 = fcd.toeplitz_T1(alpha, n, mu)
    I = np.eye(n)
    assert np.allclose(system.dense_T(alpha, n, mu, 2), np.kron(I, T1) + np.kron(T1, I))


@pytest.mark.parametrize("d,n", [(1, 9), (2, 4), (3, 3)])
def test_apply_S_is_kron_power(d, n):
    x = inputs.random_field((n,) * d, seed=3)
    Sd = system.kron_power(fcd.dst_matrix(n), d)
    assert np.allclose(system.apply_S(x).ravel(), Sd @ x.ravel(), atol=1e-13)
    assert np.allclose(system.apply_S(system.apply_S(x)), x, atol=1e-13)


@pytest.mark.parametrize("d,n", [(1, 15), (2, 6), (3, 3)])
@pytest.mark.parametrize("omega", [1.0, 1.3])
def test_preconditioner_inverse_matches_dense(d, n, omega):
    alpha, mu, rho, tau = 1.6, 0.8, 2.0, 0.05
    u = inputs.soliton(d, n, -4, 4, noise=1e-2, seed=1)
    D = system.diagonal_D(rho, tau, u)
    r = inputs.random_field((n,) * d, seed=11)
    z = system.apply_precond_inverse(alpha, n, mu, D, r, omega)
    P = system.dense_Ptilde(alpha, n, mu, d, D, omega)
    assert np.allclose(P @ z.ravel(), r.ravel(), atol=1e-12)


@pytest.mark.parametrize("d,n", [(1, 10), (2, 4)])
@pytest.mark.parametrize("omega", [1.0, 0.7])
def test_complex_form_matches_real_block_forms(d, n, omega):
    """Map [z; y] <-> y + i z (Sec. 3): R x <-> -i A u, and
    Ftilde^{-1} y <-> i Ptilde^{-1} (mapped y); the spectra of Ftilde^{-1} R
    and Ptilde^{-1} A agree (real spectrum = complex one and its conjugate)."""
    alpha, mu, rho, tau = 1.4, 0.6, 2.0, 0.1
    u = inputs.soliton(d, n, -3, 3, noise=1e-2, seed=2)
    D = system.diagonal_D(rho, tau, u)
    R = system.dense_R(alpha, n, mu, d, D)
    A = system.dense_A(alpha, n, mu, d, D)
    v = inputs.random_field((n,) * d, seed=5).ravel()
    assert np.allclose(system.from_real(R @ system.to_real(v)), -1j * (A @ v), atol=1e-12)
    # right-hand side map: R x = f  <=>  A u = b
    b = A @ v
    xr = np.linalg.solve(R, system.rhs_to_real(b))
    assert np.allclose(system.from_real(xr), v, atol=1e-11)
    Ft = system.dense_F(alpha, n, mu, d, D, omega, tau_version=True)
    y = np.random.default_rng(4).standard_normal(2 * n ** d)
    lhs = system.from_real(np.linalg.solve(Ft, y))
    rhs = 1j * system.apply_precond_inverse(alpha, n, mu, D,
                                            system.from_real(y).reshape((n,) * d), omega).ravel()
    assert np.allclose(lhs, rhs, atol=1e-12)
    ev_real = np.sort_complex(np.linalg.eigvals(np.linalg.solve(Ft, R)))
    P = system.dense_Ptilde(alpha, n, mu, d, D, omega)
    ev_c = np.linalg.eigvals(np.linalg.solve(P, A))
    ev_both = np.sort_complex(np.concatenate([ev_c, ev_c.conj()]))
    assert np.allclose(ev_real, ev_both, atol=1e-9)


@pytest.mark.parametrize("omega", [0.5, 1.0, 1.3, None])
def test_theorem_3_1_and_4_1_bounds(omega):
    """R = F - G; rho(F^{-1} G) <= sigma(omega) < 1; eigenvalues of F^{-1} R
    lie in the disc of radius sigma(omega) about 1 (exact T)."""
    d, n, alpha, mu, rho, tau = 2, 5, 1.5, 1.2, 2.0, 0.2
    u = inputs.soliton(d, n, -3, 3, noise=1e-2, seed=9)
    D = system.diagonal_D(rho, tau, u)
    lam_max = D.max()
    if omega is None:
        omega = np.sqrt(lam_max ** 2 + 1)   # Remark 3.1 optimum
    R = system.dense_R(alpha, n, mu, d, D)
    F = system.dense_F(alpha, n, mu, d, D, omega)
    G = system.dense_G(alpha, n, mu, d, D, omega)
    assert np.allclose(F - G, R, atol=1e-12)
    sig = system.sigma_bound(omega, lam_max)
    assert sig < 1
    rad = np.abs(np.linalg.eigvals(np.linalg.solve(F, G))).max()
    assert rad <= sig * (1 + 1e-10)
    ev = np.linalg.eigvals(np.linalg.solve(F, R))
    assert np.abs(ev - 1).max() <= sig * (1 + 1e-10)


def test_exact_preconditioner_special_case():
    """alpha = 2, D = 0, omega = 1: tau(T) = T and Ptilde = i I - T = A."""
    for d, n in [(1, 12), (2, 5)]:
        mu = 0.9
        D = np.zeros((n,) * d)
        P = system.dense_Ptilde(2.0, n, mu, d, D, 1.0)
        A = system.dense_A(2.0, n, mu, d, D)
        assert np.allclose(P, A, atol=1e-13)


def test_rhs_matches_dense():
    d, n, alpha, mu, rho, tau = 2, 5, 1.7, 0.5, 1.0, 0.02
    u = inputs.soliton(d, n, -2, 2, noise=1e-2, seed=4)
    D = system.diagonal_D(rho, tau, u)
    b = system.scheme_rhs(alpha, n, mu, D, u)
    Td = system.dense_T(alpha, n, mu, d)
    ref = 1j * u.ravel() + Td @ u.ravel() - D.ravel() * u.ravel()
    assert np.allclose(b.ravel(), ref, atol=1e-13)
    # A is complex symmetric and normal: B = D - T real symmetric, A = B + i I.
    A = system.dense_A(alpha, n, mu, d, D)
    assert np.allclose(A, A.T)
    assert np.allclose(A @ A.conj().T, A.conj().T @ A, atol=1e-12)


@pytest.mark.parametrize("d,ns", [(1, (32, 64)), (2, (8, 16))])
def test_clustering_does_not_degrade_with_mesh(d, ns):
    """Soft check of the clustering remark after Theorem 4.3: the 95th
    percentile of |eig(Ptilde^{-1} A) - 1| does not grow when n doubles."""
    alpha, rho, tau = 1.5, 2.0, 0.01
    q = []
    for n in ns:
        h = 20.0 / (n + 1)
        mu = fcd.mu(alpha, h, tau)
        u = inputs.soliton(d, n, -10, 10)
        D = system.diagonal_D(rho, tau, u)
        ev = np.linalg.eigvals(np.linalg.solve(system.dense_Ptilde(alpha, n, mu, d, D),
                                               system.dense_A(alpha, n, mu, d, D)))
        q.append(np.percentile(np.abs(ev - 1), 95))
    assert q[1] <= 1.5 * q[0] + 1e-3
    assert max(q) < 0.5


def test_diagonal_is_rho_dt_conj_u_times_u():
    """Sec. 2.2: D_2 = rho dt diag(vec(conj(U) . U)) (Hadamard product)."""
    u = inputs.soliton(2, 6, -3, 3, noise=1e-2, seed=8)
    D = system.diagonal_D(1.7, 0.03, u)
    ref = 1.7 * 0.03 * (np.conj(u) * u)
    assert np.allclose(D, ref.real, rtol=1e-14, atol=0) and np.abs(ref.imag).max() < 1e-17
