"""One-level building blocks, written out from their definitions.

Test infrastructure only (see the package docstring).

* c_k: the fractional centred-difference coefficients (Sec. 2.1), evaluated
  from their closed Gamma-function form in 40-digit arithmetic and rounded to
  FP64.  The reciprocal Gamma function is used so that the poles at
  alpha = 2 give exact zeros.
* T_1 = mu * T_0, T_0 the symmetric Toeplitz matrix with first row
  (c_0, ..., c_{M-1}), mu = dt / h^alpha (Sec. 2.1).
* HC(T_1), tau(T_1) = T_1 - HC(T_1) (Sec. 4, tau-matrix definition and
  Hankel-correction layout; the garbled middle rows are read as three zero
  anti-diagonals r + s in {M, M+1, M+2}, the one reading under which the sine
  transform diagonalises tau(T_1)).
* S, the sine transform (Sec. 4), with the orthonormal scaling sqrt(2/(M+1))
  (the printed sqrt(1/(M+1)) would make S^2 = I/2, so tau = S Lambda S could
  not hold).
* lambda_k, the eigenvalues of tau(T_1), from the cosine sum of its first
  row (Sec. 4: "determined by its first column").
"""
from __future__ import annotations

import functools

import mpmath
import numpy as np


@functools.lru_cache(maxsize=128)
def _coefficients_cached(alpha: float, n: int) -> tuple:
    with mpmath.workdps(40):
        a = mpmath.mpf(alpha)
        g = mpmath.gamma(a + 1)
        vals = []
        for k in range(n):
            ck = (-1) ** k * g * mpmath.rgamma(a / 2 - k + 1) * mpmath.rgamma(a / 2 + k + 1)
            vals.append(float(ck))
    return tuple(vals)


def coefficients(alpha: float, n: int) -> np.ndarray:
    """c_k = (-1)^k Gamma(alpha+1) / (Gamma(alpha/2-k+1) Gamma(alpha/2+k+1)),
    k = 0..n-1 (Sec. 2.1, coefficient formula)."""
    if n <= 0:
        return np.zeros(0)
    return np.array(_coefficients_cached(float(alpha), int(n)), dtype=np.float64)


def mu(alpha: float, h: float, tau: float) -> float:
    """mu = dt / h^alpha (Sec. 2.1)."""
    return tau / h ** alpha


def toeplitz_T0(alpha: float, n: int) -> np.ndarray:
    """T_0[j, k] = c_{j-k} = c_{|j-k|} (Sec. 2.1, the matrix T_0)."""
    c = coefficients(alpha, n)
    idx = np.arange(n)
    return c[np.abs(idx[:, None] - idx[None, :])]


def toeplitz_T1(alpha: float, n: int, mu_: float) -> np.ndarray:
    """T_1 = mu T_0 (Sec. 2.1)."""
    return mu_ * toeplitz_T0(alpha, n)


def hankel_correction(alpha: float, n: int, mu_: float) -> np.ndarray:
    """HC(T_1) with 1-based (r, s): mu c_{r+s} for r+s <= n-1, zero for
    n <= r+s <= n+2, mu c_{2n+2-r-s} for r+s >= n+3 (Sec. 4)."""
    c = coefficients(alpha, n)
    H = np.zeros((n, n))
    for r in range(1, n + 1):
        for s in range(1, n + 1):
            q = r + s
            if q <= n - 1:
                H[r - 1, s - 1] = c[q]
            elif q >= n + 3:
                H[r - 1, s - 1] = c[2 * n + 2 - q]
    return mu_ * H


def tau_T1(alpha: float, n: int, mu_: float) -> np.ndarray:
    """tau(T_1) = T_1 - HC(T_1) (Sec. 4)."""
    return toeplitz_T1(alpha, n, mu_) - hankel_correction(alpha, n, mu_)


def dst_matrix(n: int) -> np.ndarray:
    """[S]_{jk} = sqrt(2/(n+1)) sin(pi j k / (n+1)), 1 <= j, k <= n (Sec. 4,
    with the orthonormal scaling)."""
    j = np.arange(1, n + 1)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(j, j) / (n + 1))


def tau_eigenvalues(alpha: float, n: int, mu_: float) -> np.ndarray:
    """lambda_k = mu (c_0 + 2 sum_{j=1}^{n-1} c_j cos(pi j k/(n+1))), k = 1..n:
    the eigenvalues of tau(T_1) = S Lambda S (Sec. 4)."""
    c = coefficients(alpha, n)
    k = np.arange(1, n + 1)
    j = np.arange(1, n)
    cosm = np.cos(np.pi * np.outer(k, j) / (n + 1))
    return mu_ * (c[0] + 2.0 * cosm @ c[1:])


def tail_bounds(alpha: float, k0: int):
    """Lemma 4.1: theta/(k0+1/2)^alpha < sum_{j>k0} |c_j| < theta0/(k0-1)^alpha."""
    from math import gamma, sin, pi, e, sqrt
    a = alpha
    theta = ((1 - (1 + a) / (5 + a / 2)) ** (5 + a / 2) * e ** (1 + a) * gamma(a + 1)
             * sin(pi * a / 2) / (pi * a))
    theta0 = sqrt(2) * e ** (13.0 / 12.0) * gamma(a + 1) * sin(pi * a / 2) / (pi * a)
    return theta / (k0 + 0.5) ** a, theta0 / (k0 - 1) ** a, theta, theta0
