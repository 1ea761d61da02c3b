"""Pins for the one-level oracle pieces (coefficients, Toeplitz, tau, DST).

Each check compares the oracle with something other than itself: the
generating function of the fractional centred difference (quadrature), the
Gamma-function recurrence, the paper's sign/sum properties and Lemma 4.1-4.5
bounds, the alpha = 2 textbook second difference, scipy's DST-I, and dense
eigen-decompositions.
"""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.integrate
from hypothesis import given, settings, strategies as st

from oracle import fcd, system

ALPHAS = [1.1, 1.3, 1.5, 1.7, 1.9]


@pytest.mark.parametrize("alpha", [1.1, 1.5, 1.9])
@pytest.mark.parametrize("k", [0, 1, 2, 5, 17])
def test_coefficients_match_generating_function(alpha, k):
    """c_k are the Fourier coefficients of |2 sin(theta/2)|^alpha, the symbol of
    the fractional centred difference (Ortigueira 2006, Celik-Duman 2012,
    cited in Sec. 2.1).  Independent of the Gamma closed form."""
    f = lambda th: (2 * math.sin(th / 2)) ** alpha  # noqa: E731
    val, err = scipy.integrate.quad(f, 0, math.pi, weight="cos", wvar=k, limit=400)
    ck = val / math.pi
    c = fcd.coefficients(alpha, k + 1)
    assert abs(c[k] - ck) < 1e-12 * max(1.0, abs(ck)) + 5 * err


@pytest.mark.parametrize("alpha", ALPHAS)
def test_coefficient_ratio_recurrence(alpha):
    """Gamma(z+1) = z Gamma(z) gives c_{k+1}/c_k = (k - alpha/2)/(k + 1 + alpha/2)."""
    c = fcd.coefficients(alpha, 300)
    k = np.arange(299)
    ratio = c[1:] / c[:-1]
    assert np.allclose(ratio, (k - alpha / 2) / (k + 1 + alpha / 2), rtol=1e-13, atol=0)
    assert abs(c[0] - math.gamma(alpha + 1) / math.gamma(alpha / 2 + 1) ** 2) < 1e-14


@pytest.mark.parametrize("alpha", ALPHAS)
def test_coefficient_signs_sum_and_tail(alpha):
    """Sec. 2.1: c_0 >= 0, c_k = c_{-k} <= 0, sum_{k != 0} |c_k| = c_0, and the
    tail of the sum lies between the Lemma 4.1 bounds."""
    n = 2000
    c = fcd.coefficients(alpha, n)
    assert c[0] > 0 and np.all(c[1:] < 0)
    for k0 in (3, 10, 100, n - 1):
        tail = c[0] / 2 - np.sum(np.abs(c[1:k0 + 1]))
        lo, hi, _, _ = fcd.tail_bounds(alpha, k0)
        assert lo < tail < hi, (k0, lo, tail, hi)


def test_alpha2_is_second_difference():
    """alpha = 2: c = (2, -1, 0, ...), T_0 = tridiag(-1, 2, -1), HC = 0,
    tau(T) = T and lambda_k = 4 mu sin^2(k pi / (2(n+1))) (textbook)."""
    n, mu = 20, 0.37
    c = fcd.coefficients(2.0, n)
    assert c[0] == 2.0 and c[1] == -1.0 and np.all(c[2:] == 0.0)
    T0 = fcd.toeplitz_T0(2.0, n)
    ref = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    assert np.array_equal(T0, ref)
    assert np.all(fcd.hankel_correction(2.0, n, mu) == 0)
    lam = fcd.tau_eigenvalues(2.0, n, mu)
    k = np.arange(1, n + 1)
    assert np.allclose(lam, 4 * mu * np.sin(k * np.pi / (2 * (n + 1))) ** 2, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 7, 16, 31, 64])
def test_dst_matrix_is_orthonormal_dst1(n):
    """S equals scipy's orthonormal DST-I, is symmetric, and S^2 = I."""
    S = fcd.dst_matrix(n)
    ref = scipy.fft.dst(np.eye(n), type=1, norm="ortho", axis=0)
    assert np.allclose(S, ref, atol=1e-14)
    assert np.allclose(S, S.T, atol=0)
    assert np.allclose(S @ S, np.eye(n), atol=1e-13)


def test_printed_dst_scaling_is_not_orthonormal():
    """The printed sqrt(1/(M+1)) scaling gives S^2 = I/2 (recorded reading)."""
    n = 9
    S_printed = fcd.dst_matrix(n) / math.sqrt(2.0)
    assert np.allclose(S_printed @ S_printed, 0.5 * np.eye(n), atol=1e-14)


@pytest.mark.parametrize("n", [5, 8, 16, 17, 33, 64])
@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.9, 2.0])
def test_tau_matrix_diagonalised_by_dst(n, alpha):
    """tau(T_1) = S Lambda S (Sec. 4): S tau(T) S is diagonal, its diagonal is
    the cosine formula, and equals (S tau(T) e_1) / (S e_1) ("determined by its
    first column")."""
    mu = 0.7
    S = fcd.dst_matrix(n)
    M = S @ fcd.tau_T1(alpha, n, mu) @ S
    lam = fcd.tau_eigenvalues(alpha, n, mu)
    off = M - np.diag(np.diag(M))
    assert np.abs(off).max() <= 1e-13 * np.abs(lam).max()
    assert np.allclose(np.diag(M), lam, rtol=1e-12, atol=1e-13)
    e1 = np.zeros(n)
    e1[0] = 1
    first_col = (S @ (fcd.tau_T1(alpha, n, mu) @ e1)) / (S @ e1)
    assert np.allclose(first_col, lam, rtol=1e-10, atol=1e-12)


def test_other_hankel_layout_breaks_diagonalisation():
    """A plausible misreading (c_n on the anti-diagonal r+s = n+2) breaks the
    tau property, so the pinned layout is the only one that passes."""
    n, alpha, mu = 16, 1.5, 1.0
    c = fcd.coefficients(alpha, n + 1)
    H = fcd.hankel_correction(alpha, n, mu).copy()
    for r in range(1, n + 1):
        s = n + 2 - r
        if 1 <= s <= n:
            H[r - 1, s - 1] = c[n]
    S = fcd.dst_matrix(n)
    M = S @ (fcd.toeplitz_T1(alpha, n, mu) - H) @ S
    off = M - np.diag(np.diag(M))
    assert np.abs(off).max() > 1e-6


@pytest.mark.parametrize("alpha", [1.2, 1.6, 2.0])
@pytest.mark.parametrize("n", [6, 10, 24])
def test_lemma_eigenvalue_bounds(alpha, n):
    """Lemmas 4.2-4.5 (n even >= 6): eigenvalues of T_1, T_2, tau(T_1), tau(T_2)
    lie inside the stated bounds."""
    lo_x, hi_x = -3.0, 4.0
    h = (hi_x - lo_x) / (n + 1)
    dt = 0.05
    mu = fcd.mu(alpha, h, dt)
    _, _, theta, _ = fcd.tail_bounds(alpha, 3)
    c0 = math.gamma(alpha + 1) / math.gamma(alpha / 2 + 1) ** 2
    c2 = fcd.coefficients(alpha, 3)[2]
    L = (hi_x - lo_x) ** alpha
    lo1 = 2 * dt * theta / L
    hi1 = 2 * dt / h ** alpha * (c0 - theta * h ** alpha / L)
    e_T1 = np.linalg.eigvalsh(fcd.toeplitz_T1(alpha, n, mu))
    e_tau1 = np.linalg.eigvalsh(fcd.tau_T1(alpha, n, mu))
    assert lo1 < e_T1.min() and e_T1.max() < hi1
    assert lo1 < e_tau1.min() and e_tau1.max() < hi1 - c2 * dt / h ** alpha
    e_T2 = np.linalg.eigvalsh(system.dense_T(alpha, n, mu, 2))
    e_tau2 = np.linalg.eigvalsh(system.dense_tauT(alpha, n, mu, 2))
    assert 2 * lo1 < e_T2.min() and e_T2.max() < 2 * hi1
    assert 2 * lo1 < e_tau2.min() and e_tau2.max() < 2 * hi1 - 2 * c2 * dt / h ** alpha


@settings(max_examples=25, deadline=None)
@given(alpha=st.floats(1.01, 2.0), n=st.integers(2, 24), mu=st.floats(0.01, 5.0))
def test_tau_is_antisymmetric_part_of_circulant_embedding(alpha, n, mu):
    """Property: tau(T_1) x equals, on points 1..n, the circulant of length
    2(n+1) (first column mu c_|k|, zero at k = n, n+1, n+2) applied to the odd
    extension of x.  Uses numpy's FFT, not the oracle's sine transform."""
    x = np.random.default_rng(n).standard_normal(n)
    c = fcd.coefficients(alpha, n)
    L = 2 * (n + 1)
    col = np.zeros(L)
    col[:n] = mu * c
    col[L - n + 1:] = mu * c[1:][::-1]
    xe = np.zeros(L)
    xe[1:n + 1] = x
    xe[L - n:] = -x[::-1]
    y = np.fft.ifft(np.fft.fft(col) * np.fft.fft(xe)).real[1:n + 1]
    ref = fcd.tau_T1(alpha, n, mu) @ x
    assert np.allclose(y, ref, atol=1e-12 * (1 + np.abs(ref).max()))


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8, 2.0])
def test_mu_scales_T1_to_the_riesz_operator(alpha):
    """mu = dt / h^alpha (Sec. 2.1, T_1 = mu T_0) makes T_1 u approximate
    dt (-Laplacian)^(alpha/2) u, the operator whose Fourier symbol is
    |omega|^alpha (the Riesz derivative the centred differences discretise,
    with second-order accuracy).  Reference: numpy's FFT of a Gaussian on the
    same grid, multiplied by |omega|^alpha (the Gaussian is ~e^-400 at the
    ends, so the periodic transform sees the whole function).  mu is taken
    from fcd.mu; a slip to dt/h^2, h^alpha/dt or dt h^alpha is off by a
    factor 100 times the discretisation error or more (checked below), and the
    error must shrink under refinement."""
    lo, hi, dt = -20.0, 20.0, 0.01

    def err(n, mu_of):
        h = (hi - lo) / (n + 1)
        x = lo + h * np.arange(1, n + 1)
        u = np.exp(-x ** 2)
        y = fcd.toeplitz_T1(alpha, n, mu_of(h)) @ u
        w = 2 * np.pi * np.fft.fftfreq(n, h)
        ref = dt * np.fft.ifft(np.abs(w) ** alpha * np.fft.fft(u)).real
        centre = np.abs(x) < 5
        return float(np.abs(y - ref)[centre].max() / np.abs(ref).max())

    e1023 = err(1023, lambda h: fcd.mu(alpha, h, dt))
    e511 = err(511, lambda h: fcd.mu(alpha, h, dt))
    e2047 = err(2047, lambda h: fcd.mu(alpha, h, dt))
    assert e1023 < 2e-3, e1023
    assert e2047 < 0.5 * e511, (e511, e2047)
    for slip in (lambda h: h ** alpha / dt, lambda h: dt * h ** alpha):
        assert err(1023, slip) > 0.2
    if alpha != 2.0:
        assert err(1023, lambda h: dt / h ** 2) > 0.2
