"""d-level operators of the linear systems, written out from their definitions.

Test infrastructure only (see the package docstring).

Vectors are C-ordered complex128 arrays of shape (n,)*d; the last axis is the
fastest one (x_1), matching the column-stacking vec() of Sec. 2.2, so that the
flattened Kronecker sum is T_2 = I (x) T_x + T_y (x) I.

Matrix-free operators apply the dense one-level matrices (T_1, S) along each
axis in turn: that is the Kronecker-sum / Kronecker-product definition itself,
with no FFT.  The dense builders (small n only) form the same matrices with
numpy.kron.
"""
from __future__ import annotations

import numpy as np

from . import fcd


# ----------------------------------------------------------------------------
# per-axis application of a real n x n matrix
# ----------------------------------------------------------------------------

def along_axis(M: np.ndarray, x: np.ndarray, axis: int) -> np.ndarray:
    """(I (x) .. (x) M (x) .. (x) I) x, M acting on index `axis`."""
    xm = np.moveaxis(x, axis, 0)
    shape = xm.shape
    flat = xm.reshape(shape[0], -1)
    if np.iscomplexobj(flat):
        y = (M @ np.ascontiguousarray(flat.real)) + 1j * (M @ np.ascontiguousarray(flat.imag))
    else:
        y = M @ flat
    return np.ascontiguousarray(np.moveaxis(y.reshape(shape), 0, axis))


def apply_T(alpha: float, n: int, mu_: float, x: np.ndarray) -> np.ndarray:
    """T_d x = sum over axes of T_1 applied along that axis (Sec. 2.2,
    Kronecker sum; d = 1 gives T_1 x of Sec. 2.1; d = 3 extends the sum)."""
    T1 = fcd.toeplitz_T1(alpha, n, mu_)
    y = np.zeros_like(x, dtype=np.complex128)
    for ax in range(x.ndim):
        y += along_axis(T1, x, ax)
    return y


def diagonal_D(rho: float, tau: float, u: np.ndarray, V: np.ndarray | None = None) -> np.ndarray:
    """d_j = rho dt |u_j|^2 (Sec. 2.1 / 2.2), plus dt V_j for an optional real
    potential."""
    D = rho * tau * (u.real ** 2 + u.imag ** 2)
    if V is not None:
        D = D + tau * V
    return D


def apply_A(alpha: float, n: int, mu_: float, D: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A x = (D - T_d + i I) x (Sec. 2, the system matrix)."""
    return D * x - apply_T(alpha, n, mu_, x) + 1j * x


def scheme_rhs(alpha: float, n: int, mu_: float, D: np.ndarray, u_prev: np.ndarray) -> np.ndarray:
    """b = (i I + T_d - D) u^{n-1}: the three-level schemes of Sec. 2.1 and
    2.2 multiplied by 2 dt, with the u^{n-1} terms moved to the right."""
    return 1j * u_prev + apply_T(alpha, n, mu_, u_prev) - D * u_prev


def apply_S(x: np.ndarray) -> np.ndarray:
    """S_d x = (S (x) ... (x) S) x, the d-dimensional sine transform."""
    n = x.shape[0]
    S = fcd.dst_matrix(n)
    y = x
    for ax in range(x.ndim):
        y = along_axis(S, y, ax)
    return y


def tau_eigen_grid(alpha: float, n: int, mu_: float, d: int) -> np.ndarray:
    """Eigenvalues of tau(T_d) on the (n,)*d grid: the Kronecker sum of the
    one-level lambda_k (Sec. 4, d-level tau matrix)."""
    lam = fcd.tau_eigenvalues(alpha, n, mu_)
    L = np.zeros((n,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = n
        L = L + lam.reshape(shape)
    return L


def apply_precond_inverse(alpha: float, n: int, mu_: float, D: np.ndarray, r: np.ndarray,
                          omega: float = 1.0) -> np.ndarray:
    """z = Ptilde^{-1} r for the sine-transform TBAN preconditioner in complex
    form.

    The real 2x2 block system of Sec. 3 maps to the complex one through
    [z; y] -> y + i z.  Under that map a block [[P, -Q], [Q, P]] acts as
    P - i Q, so omega I + tau(calT_d) -> omega I + i tau(T_d) and
    omega I + calD_d -> (omega+1) I - i D, and the preconditioner of Sec. 4
    becomes Mt = (1/2 omega)(omega I + i tau(T_d))((omega+1) I - i D).  The
    real preconditioned matrix Ft^{-1} R corresponds to Mt^{-1}(-i A), i.e.
    the complex preconditioner is Ptilde = i Mt, whose inverse is

        z = -2 i omega ((omega+1) - i D)^{-1} . S_d (omega + i Lambda_d)^{-1} . S_d r.
    """
    Lam = tau_eigen_grid(alpha, n, mu_, r.ndim)
    t = apply_S(r)
    t = t / (omega + 1j * Lam)
    t = apply_S(t)
    return (-2j * omega) * t / ((omega + 1.0) - 1j * D)


# ----------------------------------------------------------------------------
# dense builders (tiny grids only)
# ----------------------------------------------------------------------------

def kron_sum(M: np.ndarray, d: int) -> np.ndarray:
    """sum over axes of I (x) .. (x) M (x) .. (x) I for C-ordered flattening."""
    n = M.shape[0]
    I = np.eye(n)
    out = np.zeros((n ** d, n ** d))
    for ax in range(d):
        term = np.array([[1.0]])
        for k in range(d):
            term = np.kron(term, M if k == ax else I)
        out += term
    return out


def kron_power(M: np.ndarray, d: int) -> np.ndarray:
    out = np.array([[1.0]])
    for _ in range(d):
        out = np.kron(out, M)
    return out


def dense_T(alpha, n, mu_, d):
    return kron_sum(fcd.toeplitz_T1(alpha, n, mu_), d)


def dense_tauT(alpha, n, mu_, d):
    return kron_sum(fcd.tau_T1(alpha, n, mu_), d)


def dense_A(alpha, n, mu_, d, D):
    return np.diag(D.ravel()).astype(np.complex128) - dense_T(alpha, n, mu_, d) + 1j * np.eye(n ** d)


def dense_Ptilde(alpha, n, mu_, d, D, omega=1.0):
    """Ptilde = (i/2 omega)(omega I + i tau(T_d))((omega+1) I - i D) (dense)."""
    Nn = n ** d
    I = np.eye(Nn)
    return (1j / (2 * omega)) * (omega * I + 1j * dense_tauT(alpha, n, mu_, d)) @ \
        ((omega + 1.0) * I - 1j * np.diag(D.ravel()))


# real 2x2 block forms (Sec. 3 and 4) -----------------------------------------

def block(P11, P12, P21, P22):
    return np.block([[P11, P12], [P21, P22]])


def dense_R(alpha, n, mu_, d, D):
    """R = [[I, T - D], [D - T, I]] (Sec. 3, real block form)."""
    T = dense_T(alpha, n, mu_, d)
    Dm = np.diag(D.ravel())
    I = np.eye(T.shape[0])
    return block(I, T - Dm, Dm - T, I)


def dense_calT(T):
    Z = np.zeros_like(T)
    return block(Z, T, -T, Z)


def dense_calD(D):
    Dm = np.diag(D.ravel())
    I = np.eye(Dm.shape[0])
    return block(I, -Dm, Dm, I)


def dense_F(alpha, n, mu_, d, D, omega, tau_version=False):
    """F_omega = (1/2 omega)(omega I + calT)(omega I + calD) (Sec. 3); with
    tau_version, T is replaced by tau(T_d) (Sec. 4, the sine-transform
    preconditioner Ftilde)."""
    T = dense_tauT(alpha, n, mu_, d) if tau_version else dense_T(alpha, n, mu_, d)
    calT = dense_calT(T)
    calD = dense_calD(D)
    I = np.eye(calT.shape[0])
    return (omega * I + calT) @ (omega * I + calD) / (2 * omega)


def dense_G(alpha, n, mu_, d, D, omega):
    """G_omega = (1/2 omega)(omega I - calT)(omega I - calD) (Sec. 3)."""
    calT = dense_calT(dense_T(alpha, n, mu_, d))
    calD = dense_calD(D)
    I = np.eye(calT.shape[0])
    return (omega * I - calT) @ (omega * I - calD) / (2 * omega)


def sigma_bound(omega: float, lam_max: float) -> float:
    """sigma(omega) of Theorem 3.1."""
    return np.sqrt(((omega - 1) ** 2 + lam_max ** 2) / ((omega + 1) ** 2 + lam_max ** 2))


def to_real(u: np.ndarray) -> np.ndarray:
    """u = y + i z  ->  x = [z; y] (Sec. 3)."""
    u = u.ravel()
    return np.concatenate([u.imag, u.real])


def rhs_to_real(b: np.ndarray) -> np.ndarray:
    """b = p + i q  ->  f = [-p; q] (Sec. 3)."""
    b = b.ravel()
    return np.concatenate([-b.real, b.imag])


def from_real(x: np.ndarray) -> np.ndarray:
    """[z; y] -> y + i z."""
    N = x.size // 2
    return x[N:] + 1j * x[:N]
