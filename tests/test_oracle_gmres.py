"""Pins for the oracle's GMRES and time stepping.

Dense LU (numpy.linalg.solve), a brute-force Krylov least-squares minimiser,
the exact-preconditioner special case, the unitarity of the three-level step,
and the paper's printed mass-error table and iteration counts.
"""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import fcd, system, stepping
from oracle.gmres import pgmres, givens, NOT_CONVERGED, OK
from paper_2410_03643_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def make_system(d, n, alpha=1.5, rho=2.0, tau=0.05, lo=-6.0, hi=6.0, seed=0):
    h = (hi - lo) / (n + 1)
    mu = fcd.mu(alpha, h, tau)
    u = inputs.soliton(d, n, lo, hi, noise=1e-2, seed=seed)
    D = system.diagonal_D(rho, tau, u)
    A = lambda x: system.apply_A(alpha, n, mu, D, x)  # noqa: E731
    P = lambda r: system.apply_precond_inverse(alpha, n, mu, D, r)  # noqa: E731
    b = system.scheme_rhs(alpha, n, mu, D, u)
    return A, P, b, (alpha, n, mu, D)


@pytest.mark.parametrize("d,n", [(1, 63), (2, 15), (3, 7)])
@pytest.mark.parametrize("alpha", [1.2, 1.8])
def test_gmres_matches_dense_lu(d, n, alpha):
    A, P, b, (a, n_, mu, D) = make_system(d, n, alpha)
    x, info = pgmres(A, P, b, tol=1e-12)
    Ad = system.dense_A(a, n_, mu, d, D)
    xs = np.linalg.solve(Ad, b.ravel())
    kappa = np.linalg.cond(Ad)
    assert info.status == OK
    assert info.relres_true < 1e-12
    assert np.linalg.norm(x.ravel() - xs) / np.linalg.norm(xs) < 10 * kappa * 1e-12
    # recomputed residual agrees with a dense product
    assert np.linalg.norm(b.ravel() - Ad @ x.ravel()) / np.linalg.norm(b) < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_fixed_iters_is_krylov_minimiser(k):
    """After k steps, x_k = P^{-1} y with y in K_k(A P^{-1}, b) minimising
    ||b - A P^{-1} y||: checked by an explicit least-squares solve."""
    d, n = 1, 40
    A, P, b, _ = make_system(d, n, 1.7, tau=0.2)
    x, info = pgmres(A, P, b, fixed_iters=k)
    assert info.iters == k
    cols = []
    v = b.ravel().copy()
    for _ in range(k):
        cols.append(v.copy())
        v = A(P(v.reshape(b.shape))).ravel()
    Q, _ = np.linalg.qr(np.array(cols).T)
    AQ = np.array([A(P(Q[:, i].reshape(b.shape))).ravel() for i in range(k)]).T
    c, *_ = np.linalg.lstsq(AQ, b.ravel(), rcond=None)
    xref = P((Q @ c).reshape(b.shape))
    assert np.linalg.norm(x - xref) / np.linalg.norm(xref) < 1e-10


def test_givens_convention():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a = complex(rng.standard_normal(), rng.standard_normal())
        bb = abs(rng.standard_normal())
        c, s = givens(a, bb)
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-15
        assert abs(-np.conj(s) * a + c * bb) < 1e-15
        top = c * a + s * bb
        assert abs(abs(top) - np.hypot(abs(a), bb)) < 1e-14
    c, s = givens(0j, 2.0)
    assert c == 0.0 and s == 1.0


def test_exact_preconditioner_converges_in_one_iteration():
    """alpha = 2, D = 0: Ptilde = A, so A P^{-1} = I and GMRES stops after one
    step (happy breakdown) with the exact solution."""
    for d, n in [(1, 31), (2, 15)]:
        mu = 0.8
        D = np.zeros((n,) * d)
        A = lambda x: system.apply_A(2.0, n, mu, D, x)  # noqa: E731
        P = lambda r: system.apply_precond_inverse(2.0, n, mu, D, r)  # noqa: E731
        b = inputs.random_field((n,) * d, seed=2)
        x, info = pgmres(A, P, b, tol=1e-14)
        assert info.iters == 1
        xs = np.linalg.solve(system.dense_A(2.0, n, mu, d, D), b.ravel())
        assert np.allclose(x.ravel(), xs, atol=1e-12)


def test_not_converged_and_zero_rhs():
    A, P, b, _ = make_system(1, 31)
    x, info = pgmres(A, P, b, tol=1e-30, maxit=3)
    assert info.status == NOT_CONVERGED and info.iters == 3
    x0, info0 = pgmres(A, P, np.zeros_like(b))
    assert info0.iters == 0 and np.all(x0 == 0)


def test_restart_reaches_same_solution():
    A, P, b, _ = make_system(1, 63, 1.9, tau=0.5)
    x1, i1 = pgmres(A, P, b, tol=1e-12)
    x2, i2 = pgmres(A, P, b, tol=1e-12, restart=2)
    assert i2.cycles > 1
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-10


@settings(max_examples=10, deadline=None)
@given(alpha=st.floats(1.05, 2.0), d=st.integers(1, 3), seed=st.integers(0, 100))
def test_gmres_random_params_vs_lu(alpha, d, seed):
    n = {1: 24, 2: 6, 3: 4}[d]
    A, P, b, (a, n_, mu, D) = make_system(d, n, alpha, seed=seed)
    x, info = pgmres(A, P, b, tol=1e-12)
    xs = np.linalg.solve(system.dense_A(a, n_, mu, d, D), b.ravel())
    assert np.linalg.norm(x.ravel() - xs) / np.linalg.norm(xs) < 1e-9


def test_iterations_independent_of_mesh():
    """Sec. 5: IT essentially constant under mesh refinement (fixed domain and
    time step), here within +-1 over n = 63..511 in 1-D."""
    its = []
    for n in (63, 127, 255, 511):
        h = 40.0 / (n + 1)
        mu = fcd.mu(1.5, h, 0.01)
        u = inputs.soliton(1, n, -20, 20)
        x, info = stepping.step(1.5, 2.0, n, mu, 0.01, u, u, tol=1e-10)
        its.append(info.iters)
    assert max(its) - min(its) <= 1


def test_paper_1d_iteration_counts_are_an_upper_bound():
    """Sec. 5.1 tables print IT = 6 at tol 1e-8 for M = 6400 with N = 200
    time steps and an unstated final time.  For the time steps of final times
    1, 2 and 4 over those 200 steps (dt = 0.005, 0.01, 0.02) the oracle needs
    at most that many iterations (complex GMRES never needs more than the
    real block form: the real Krylov space maps isometrically into the
    complex one)."""
    table = json.load(open(os.path.join(GOLDEN, "paper_iteration_counts.json")))
    it_paper = table["tau_gmres_IT_1d"]["1.4"][0]
    n = table["tau_gmres_IT_1d"]["M"][0]
    u = inputs.soliton(1, n, -20, 20, kx=2.0)
    h = 40.0 / (n + 1)
    for dt in (0.005, 0.01, 0.02):
        mu = fcd.mu(1.4, h, dt)
        x, info = stepping.step(1.4, 2.0, n, mu, dt, u, u, tol=1e-8)
        assert info.iters <= it_paper


def test_step_is_unitary_and_starter_conserves_norm():
    """The three-level step is a Cayley map: ||u^{n+1}|| = ||u^{n-1}||."""
    d, n = 2, 15
    alpha, rho, tau = 1.6, 2.0, 0.02
    h = 12.0 / (n + 1)
    mu = fcd.mu(alpha, h, tau)
    u0 = inputs.soliton(d, n, -6, 6)
    u1, _ = stepping.first_step(alpha, rho, n, mu, tau, u0, tol=1e-14)
    assert abs(np.linalg.norm(u1) - np.linalg.norm(u0)) < 1e-12
    u2, _ = stepping.step(alpha, rho, n, mu, tau, u0, u1, tol=1e-14)
    assert abs(np.linalg.norm(u2) - np.linalg.norm(u0)) < 1e-12


@pytest.mark.parametrize("alpha", ["1.4", "1.7", "1.9", "2.0"])
def test_paper_mass_error_table(alpha):
    """Reproduce the Sec. 5.1 mass-conservation protocol; the relative mass
    errors are at the rounding level printed by the paper (all <= 5.6e-16)."""
    table = json.load(open(os.path.join(GOLDEN, "paper_mass_error_table.json")))
    paper = table["rows"][alpha]
    a = float(alpha)
    p = inputs.paper_1d_mass_case(a)
    assert abs(p.h - 0.2) < 1e-15 and p.tau == 0.05
    mu = fcd.mu(a, p.h, p.tau)
    u0 = p.u
    u1, _ = stepping.first_step(a, p.rho, p.n, mu, p.tau, u0, tol=1e-15)
    Q0 = stepping.mass(p.h, u1, u0)
    up, uc = u0, u1
    errs = []
    spt = table["steps_per_unit_time"]
    for k in range(1, spt * len(table["t"])):
        un, info = stepping.step(a, p.rho, p.n, mu, p.tau, up, uc, tol=1e-15)
        up, uc = uc, un
        if (k + 1) % spt == 0:
            errs.append(abs(stepping.mass(p.h, un, up) - Q0) / Q0)
    assert len(errs) == len(paper)
    assert max(errs) <= 10 * max(max(paper), 2.3e-16)
