"""Right-preconditioned restarted GMRES (textbook form), complex FP64.

Test infrastructure only (see the package docstring).

Follows the protocol of Sec. 5: zero initial guess, stopping on the l2
relative residual ||b - A x|| / ||b||, at most 2000 iterations.  The paper
leaves open the side of the preconditioner, the Arnoldi variant, the Givens
convention, the restart length and the breakdown test; this loop takes right
preconditioning (so the monitored residual is the true one), classical
Gram-Schmidt applied twice, restart 30 and the conventions below, so that the
GPU solver's intermediate quantities are directly comparable:

* Arnoldi step j: w = A (P^{-1} v_j); h1 = V^H w; w -= V h1; h2 = V^H w;
  w -= V h2; h_{:, j} = h1 + h2; h_{j+1, j} = ||w||; v_{j+1} = w / h_{j+1, j}.
* Givens: for the pair (a, b) = (H_jj after the earlier rotations, h_{j+1,j}),
  c = |a| / sqrt(|a|^2 + |b|^2), s = (a/|a|) conj(b) / sqrt(|a|^2 + |b|^2)
  (c = 0, s = 1 when a = 0); the rotation maps (x, y) to
  (c x + s y, -conj(s) x + c y); g_{j+1} = -conj(s) g_j, g_j = c g_j.
* Converged when |g_{j+1}| / ||b|| < tol; at the end of a cycle
  x += P^{-1} (V y) with y = H^{-1} g, the true residual is recomputed, and
  the method restarts if it is still >= tol.
* Happy breakdown when h_{j+1,j} <= 1e-14 ||A P^{-1} v_j||.
* fixed_iters = k > 0 runs exactly k iterations (no tolerance test).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

OK = 0
NOT_CONVERGED = 1
BREAKDOWN_EPS = 1e-14


@dataclass
class GmresInfo:
    iters: int = 0
    cycles: int = 0
    status: int = OK
    relres_true: float = 0.0
    relres_hist: list = field(default_factory=list)


def _vdot(a: np.ndarray, b: np.ndarray) -> complex:
    return complex(np.vdot(a.ravel(), b.ravel()))


def _norm(a: np.ndarray) -> float:
    return float(np.sqrt(np.vdot(a.ravel(), a.ravel()).real))


def givens(a: complex, b: float):
    """Rotation (c, s) that zeroes b below a (convention in the module doc)."""
    aa = abs(a)
    if aa == 0.0:
        return 0.0, 1.0 + 0.0j
    r = np.hypot(aa, abs(b))
    return aa / r, (a / aa) * np.conj(b) / r


def pgmres(apply_A, apply_Pinv, b: np.ndarray, *, tol: float = 1e-10, restart: int = 30,
           maxit: int = 2000, fixed_iters: int = 0):
    """Solve A x = b with right preconditioning, x0 = 0.  Returns (x, info)."""
    info = GmresInfo()
    x = np.zeros_like(b, dtype=np.complex128)
    bnorm = _norm(b)
    if bnorm == 0.0:
        return x, info
    r = b.astype(np.complex128, copy=True)
    total = 0
    while True:
        info.cycles += 1
        beta = _norm(r)
        V = [r / beta]
        R = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        k = 0
        breakdown = False
        for j in range(restart):
            w = apply_A(apply_Pinv(V[j]))
            w_norm0 = _norm(w)
            h1 = np.array([_vdot(V[i], w) for i in range(j + 1)])
            for i in range(j + 1):
                w = w - h1[i] * V[i]
            h2 = np.array([_vdot(V[i], w) for i in range(j + 1)])
            for i in range(j + 1):
                w = w - h2[i] * V[i]
            col = np.zeros(j + 2, dtype=np.complex128)
            col[: j + 1] = h1 + h2
            hn = _norm(w)
            col[j + 1] = hn
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -np.conj(sn[i]) * col[i] + cs[i] * col[i + 1]
                col[i] = t
            c, s = givens(col[j], hn)
            cs[j], sn[j] = c, s
            col[j] = c * col[j] + s * hn
            col[j + 1] = 0.0
            R[: j + 2, j] = col
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            total += 1
            k = j + 1
            est = abs(g[j + 1]) / bnorm
            info.relres_hist.append(est)
            breakdown = hn <= BREAKDOWN_EPS * w_norm0
            if fixed_iters:
                stop = total >= fixed_iters
            else:
                stop = est < tol
            if stop or breakdown or total >= maxit:
                break
            V.append(w / hn)
        # y = R_k^{-1} g_k (back substitution on the rotated Hessenberg)
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            acc = g[i] - np.dot(R[i, i + 1:k], y[i + 1:k])
            y[i] = acc / R[i, i]
        t = np.zeros_like(x)
        for i in range(k):
            t = t + y[i] * V[i]
        x = x + apply_Pinv(t)
        r = b - apply_A(x)
        info.relres_true = _norm(r) / bnorm
        info.iters = total
        if fixed_iters:
            if total >= fixed_iters or breakdown:
                break
        elif info.relres_true < tol:
            break
        if total >= maxit:
            info.status = NOT_CONVERGED
            break
    if not fixed_iters and info.relres_true >= tol:
        info.status = NOT_CONVERGED
    return x, info
