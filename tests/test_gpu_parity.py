"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Element-wise comparison on the same seeded inputs.  Operators: relative
max-norm error <= 1e-12 (FP64 FFT/DST rounding against the dense oracle).
Solves (parity rule): IT within 1 of the oracle's at the same tolerance, and
||x_gpu - x_oracle(fixed_iters = IT_gpu)|| / ||x_oracle|| <= 1e-10; the
recomputed residual of the GPU solution (by the oracle's own operator) below
the tolerance.  FP32-IR: oracle residual of x_IR below the tolerance and its
error against the FP64 oracle solution reported and bounded by cond * tol.
"""
import numpy as np
import pytest

import oracle
from oracle import fcd
from paper_2410_03643_amd import inputs

pytestmark = pytest.mark.gpu

OP_TOL = 1e-12
X_TOL = 1e-10


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda", 0)


def make(torch_dev, d, n, lo, hi, alpha, rho, tau, noise=1e-3, seed=0, restart=30):
    from paper_2410_03643_amd.fnls import Solver
    torch, dev = torch_dev
    h = (hi - lo) / (n + 1)
    u = inputs.soliton(d, n, lo, hi, noise=noise, seed=seed)
    s = Solver(alpha, rho, d, n, h, tau, device=dev, restart=restart)
    o = oracle.OracleSolver(alpha, rho, d, n, h, tau)
    ut = torch.from_numpy(u).to(dev)
    s.precond_setup(ut)
    o.precond_setup(u)
    return s, o, u, ut


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


OP_CASES = [(1, 1), (1, 3), (1, 7), (1, 15), (1, 63), (1, 255), (1, 511), (1, 1023),
            (2, 1), (2, 3), (2, 7), (2, 31), (2, 127), (2, 255), (2, 511),
            (3, 1), (3, 3), (3, 7), (3, 15), (3, 31)]


@pytest.mark.parametrize("d,n", OP_CASES)
def test_apply_A(torch_dev, d, n):
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, d, n, -6.0, 6.0, 1.5, 2.0, 0.05)
    x = inputs.random_field((n,) * d, seed=3)
    y = to_np(s.apply_A(torch.from_numpy(x).to(dev)))
    assert relerr(y, o.apply_A(x)) < OP_TOL


@pytest.mark.parametrize("d,n", OP_CASES)
def test_apply_precond(torch_dev, d, n):
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, d, n, -6.0, 6.0, 1.7, 2.0, 0.05)
    r = inputs.random_field((n,) * d, seed=4)
    z = to_np(s.apply_precond(torch.from_numpy(r).to(dev)))
    assert relerr(z, o.apply_Pinv(r)) < OP_TOL


@pytest.mark.parametrize("d,n", [(1, 63), (2, 31), (3, 15)])
def test_rhs(torch_dev, d, n):
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, d, n, -6.0, 6.0, 1.3, 1.0, 0.02)
    b = to_np(s.rhs(ut))
    assert relerr(b, o.rhs(u)) < OP_TOL


@pytest.mark.parametrize("alpha", [1.1, 1.5, 2.0])
def test_apply_A_alpha_range(torch_dev, alpha):
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 63, -10.0, 10.0, alpha, 2.0, 0.01)
    x = inputs.random_field((63, 63), seed=5)
    assert relerr(to_np(s.apply_A(torch.from_numpy(x).to(dev))), o.apply_A(x)) < OP_TOL
    assert relerr(to_np(s.apply_precond(torch.from_numpy(x).to(dev))), o.apply_Pinv(x)) < OP_TOL


def check_solve(torch_dev, s, o, u, ut, tol=1e-10, **kw):
    torch, dev = torch_dev
    b = o.rhs(u)
    bt = torch.from_numpy(b).to(dev)
    x_t, info = s.solve(bt, tol=tol, **kw)
    x = to_np(x_t)
    xo, io = o.solve(b, tol=tol)
    xf, _ = o.solve(b, fixed_iters=info.iters)
    res = np.linalg.norm(b - o.apply_A(x)) / np.linalg.norm(b)
    print("IT gpu %d oracle %d | relres gpu %.3e oracle-recomputed %.3e | |x-x_fixed| %.3e"
          % (info.iters, io.iters, info.relres_true, res,
             np.linalg.norm(x - xf) / np.linalg.norm(xf)), flush=True)
    assert info.status == 0
    assert abs(info.iters - io.iters) <= 1
    assert res < tol
    assert np.linalg.norm(x - xf) / np.linalg.norm(xf) < X_TOL
    return x, info


@pytest.mark.parametrize("d,n,lo,hi", [(1, 63, -20, 20), (1, 1023, -20, 20), (2, 31, -10, 10),
                                       (2, 127, -10, 10), (3, 15, -8, 8), (3, 31, -8, 8)])
def test_solve_fp64(torch_dev, d, n, lo, hi):
    s, o, u, ut = make(torch_dev, d, n, lo, hi, 1.5, 2.0, 0.01)
    check_solve(torch_dev, s, o, u, ut)


def test_solve_metric_case(torch_dev):
    """d = 2, n = 1023 on [-10, 10]^2, alpha 1.5, rho 2, dt 0.01 (full size)."""
    p = inputs.metric_case()
    s, o, u, ut = make(torch_dev, p.d, p.n, p.lo, p.hi, p.alpha, p.rho, p.tau)
    check_solve(torch_dev, s, o, u, ut)


@pytest.mark.parametrize("d,n", [(1, 255), (2, 63), (3, 15)])
def test_solve_fp32_ir(torch_dev, d, n):
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, d, n, -10.0, 10.0, 1.6, 2.0, 0.01)
    b = o.rhs(u)
    x_t, info = s.solve(torch.from_numpy(b).to(dev), tol=1e-10, precision="fp32_ir")
    x = to_np(x_t)
    res = np.linalg.norm(b - o.apply_A(x)) / np.linalg.norm(b)
    xo, _ = o.solve(b, tol=1e-13)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    _, i64 = s.solve(torch.from_numpy(b).to(dev), tol=1e-10)
    print("IR: inner IT %d outer %d (FP64 IT %d) relres %.3e (oracle %.3e) err vs FP64 oracle %.3e"
          % (info.iters, info.outer_iters, i64.iters, info.relres_true, res, err), flush=True)
    assert info.status == 0
    assert res < 1e-10
    assert err < 1e-8
    # a degraded FP32 kernel would show as extra refinement steps / inner iterations
    assert info.outer_iters <= 3
    assert info.iters <= 2 * i64.iters + 2


def test_solve_metric_case_fp32_ir(torch_dev):
    """GMRES-IR at the metric case: the oracle's residual below 1e-10, the
    error against the oracle's FP64 solution (to 1e-13) within cond(A) * tol,
    at most 3 refinement steps and at most 2 inner iterations more than the
    FP64 solve's."""
    torch, dev = torch_dev
    p = inputs.metric_case()
    s, o, u, ut = make(torch_dev, p.d, p.n, p.lo, p.hi, p.alpha, p.rho, p.tau)
    b = o.rhs(u)
    bt = torch.from_numpy(b).to(dev)
    x_t, info = s.solve(bt, tol=1e-10, precision="fp32_ir")
    _, i64 = s.solve(bt, tol=1e-10)
    x = to_np(x_t)
    res = np.linalg.norm(b - o.apply_A(x)) / np.linalg.norm(b)
    xo, _ = o.solve(b, tol=1e-13)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    c0 = fcd.coefficients(p.alpha, 2)[0]
    kap = np.sqrt(1.0 + (p.d * fcd.mu(p.alpha, p.h, p.tau) * 2 * c0 + p.rho * p.tau * np.abs(u).max() ** 2) ** 2)
    print("metric IR: inner IT %d outer %d (FP64 IT %d) relres %.2e oracle %.2e err vs FP64 oracle %.2e "
          "(cond bound %.1f)" % (info.iters, info.outer_iters, i64.iters, info.relres_true, res, err, kap), flush=True)
    assert info.status == 0 and res < 1e-10
    assert err <= kap * 1e-10
    assert info.outer_iters <= 3 and info.iters <= i64.iters + 2


def test_zero_rhs_gives_zero(torch_dev):
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 31, -10, 10, 1.5, 2.0, 0.01)
    x_t, info = s.solve(torch.zeros_like(ut))
    assert info.iters == 0 and float(x_t.abs().max()) == 0.0


def test_nonfinite_rhs_is_reported(torch_dev):
    from paper_2410_03643_amd.fnls import FnlsError, ERR_NONFINITE
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 31, -10, 10, 1.5, 2.0, 0.01)
    b = ut.clone()
    b[3, 5] = complex(float("nan"), 0.0)
    with pytest.raises(FnlsError) as e:
        s.solve(b)
    assert e.value.code == ERR_NONFINITE


def test_option_limits_are_checked_before_any_work(torch_dev):
    """maxit beyond 2^21 (the bound that keeps a solve's status reports inside
    its window of the status sequence) and restart beyond the workspace are
    rejected on the host; the context still solves afterwards."""
    from paper_2410_03643_amd.fnls import FnlsError, ERR_INVALID_ARG, ERR_WORKSPACE
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 31, -10, 10, 1.5, 2.0, 0.01)
    b = s.rhs(ut)
    with pytest.raises(FnlsError) as e:
        s.solve(b, maxit=(1 << 21) + 1)
    assert e.value.code == ERR_INVALID_ARG
    with pytest.raises(FnlsError) as e:
        s.solve(b, restart=31)
    assert e.value.code == ERR_WORKSPACE
    x, info = s.solve(b, maxit=1 << 21)
    assert info.status == 0


def test_exact_preconditioner_one_iteration(torch_dev):
    """alpha = 2, rho = 0: Ptilde = A, GMRES stops after one iteration."""
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 31, -5, 5, 2.0, 0.0, 0.05)
    b = inputs.random_field((31, 31), seed=9)
    x_t, info = s.solve(torch.from_numpy(b).to(dev), tol=1e-13)
    assert info.iters == 1
    x = to_np(x_t)
    assert np.linalg.norm(b - o.apply_A(x)) / np.linalg.norm(b) < 1e-13


def test_restart_and_maxit(torch_dev):
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 1, 127, -20, 20, 1.9, 2.0, 0.5)
    b = o.rhs(u)
    bt = torch.from_numpy(b).to(dev)
    x_t, info = s.solve(bt, tol=1e-10, restart=2)
    assert info.status == 0 and info.outer_iters > 1
    x = to_np(x_t)
    assert np.linalg.norm(b - o.apply_A(x)) / np.linalg.norm(b) < 1e-10
    x_t, info = s.solve(bt, tol=1e-30, maxit=3)
    assert info.status == 1 and info.iters == 3


@pytest.mark.parametrize("restart", [64, 30])
def test_long_cycles_match_oracle(torch_dev, restart):
    """A weak preconditioner (omega = 0.02, 1-D, n = 1023) takes GMRES over 50
    iterations: in one cycle of the largest basis (restart 64, where the
    stopping workgroup back-substitutes a triangle of that size) and across
    restart boundaries (30).  The iteration count is the oracle's within one,
    and the solution equals the oracle's after the same number of iterations
    and restart length."""
    from paper_2410_03643_amd.fnls import Solver
    torch, dev = torch_dev
    n, lo, hi, alpha, rho, dt, om = 1023, -20.0, 20.0, 1.5, 2.0, 0.01, 0.02
    h = (hi - lo) / (n + 1)
    u = inputs.soliton(1, n, lo, hi, kx=2.0)
    s = Solver(alpha, rho, 1, n, h, dt, device=dev, restart=restart)
    s.precond_setup(torch.from_numpy(u).to(dev), omega=om)
    o = oracle.OracleSolver(alpha, rho, 1, n, h, dt)
    o.precond_setup(u, omega=om)
    b = o.rhs(u)
    x_t, info = s.solve(torch.from_numpy(b).to(dev), tol=1e-10, restart=restart)
    x = to_np(x_t)
    _, io = o.solve(b, tol=1e-10, restart=restart)
    xf, _ = o.solve(b, restart=restart, fixed_iters=info.iters)
    res = np.linalg.norm(b - o.apply_A(x)) / np.linalg.norm(b)
    err = np.linalg.norm(x - xf) / np.linalg.norm(xf)
    print("restart %d: IT gpu %d (%d cycles) oracle %d | relres %.3e | |x-x_fixed| %.3e"
          % (restart, info.iters, info.outer_iters, io.iters, res, err), flush=True)
    assert info.status == 0 and info.iters > 50
    assert (info.outer_iters == 1) == (restart == 64)
    assert abs(info.iters - io.iters) <= 1
    assert res < 1e-10
    assert err < X_TOL


@pytest.mark.parametrize("k", [1, 2, 4])
def test_fixed_iters_matches_oracle(torch_dev, k):
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 63, -10, 10, 1.4, 2.0, 0.05)
    b = o.rhs(u)
    x_t, info = s.solve(torch.from_numpy(b).to(dev), fixed_iters=k)
    assert info.iters == k
    xf, _ = o.solve(b, fixed_iters=k)
    assert np.linalg.norm(to_np(x_t) - xf) / np.linalg.norm(xf) < 1e-12


def test_solve_is_deterministic(torch_dev):
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 127, -10, 10, 1.5, 2.0, 0.01)
    b = s.rhs(ut)
    x1, i1 = s.solve(b)
    x2, i2 = s.solve(b)
    assert i1.iters == i2.iters and torch.equal(x1, x2)


def test_lookahead_settings_agree(torch_dev):
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 63, -10, 10, 1.5, 2.0, 0.01)
    b = s.rhs(ut)
    xs = [s.solve(b, lookahead=la)[0] for la in (0, 1, 3)]
    assert torch.equal(xs[0], xs[1]) and torch.equal(xs[0], xs[2])


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_lookahead_settings_agree_uneven_convergence(torch_dev, precision):
    """A random right-hand side converges at an uneven rate, so the host's
    prediction of the stopping iteration (which issues only the next first
    pass ahead) is sometimes wrong and the iteration is completed afterwards:
    lookahead 0, 1 and 3 must still give bitwise equal results, over several
    restart cycles, with the oracle's iteration count."""
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 255, -10, 10, 1.3, 2.0, 0.02)
    bn = inputs.random_field(u.shape, seed=17)
    b = torch.from_numpy(bn).to(dev)
    tol = 1e-13 if precision == "fp64" else 1e-11
    runs = [s.solve(b, tol=tol, restart=3, lookahead=la, precision=precision) for la in (0, 1, 3)]
    its = [r[1].iters for r in runs]
    print("%s: IT %s, outer %s" % (precision, its, [r[1].outer_iters for r in runs]), flush=True)
    assert all(r[1].status == 0 for r in runs)
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][0], runs[2][0])
    assert its[0] == its[1] == its[2]
    if precision == "fp64":
        _, io = o.solve(bn, tol=tol, restart=3)
        assert abs(io.iters - its[0]) <= 1


def test_status_sequence_across_solves(torch_dev):
    """The host takes each Arnoldi iteration's status from a sequence number
    the device publishes in pinned memory (no event per iteration).  Many
    solves in a row on one context, alternating precision and restart length
    (so with and without restarts), must repeat their iteration counts and
    solutions bitwise."""
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 63, -10, 10, 1.5, 2.0, 0.01)
    b = s.rhs(ut)
    ref = {}
    for k in range(24):
        key = (("fp64", "fp32_ir")[k % 2], (30, 3)[(k // 2) % 2])
        x, info = s.solve(b, precision=key[0], restart=key[1])
        assert info.status == 0
        if key in ref:
            assert info.iters == ref[key][1] and torch.equal(x, ref[key][0])
        else:
            ref[key] = (x.clone(), info.iters)
    print({k: v[1] for k, v in ref.items()}, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_end_of_cycle_enqueued_ahead_matches(torch_dev, precision):
    """Near a predicted stop the end-of-cycle passes are enqueued ahead,
    guarded by the device's stop flag (not while per-launch timing is on).
    With timing on and off, and over restart cycles of 3 where the prediction
    is sometimes wrong, the results must be bitwise equal."""
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 127, -10, 10, 1.3, 2.0, 0.02)
    b = torch.from_numpy(inputs.random_field(u.shape, seed=23)).to(dev)
    for restart in (30, 3):
        x1, i1 = s.solve(b, tol=1e-12, restart=restart, precision=precision)
        s.timing(True)
        x2, i2 = s.solve(b, tol=1e-12, restart=restart, precision=precision)
        s.timing(False)
        assert i1.status == 0 and i1.iters == i2.iters and i1.outer_iters == i2.outer_iters
        assert torch.equal(x1, x2)


def test_refinement_step_limit(torch_dev):
    """FP32-IR with max_outer refinement steps: one step cannot reach 1e-10
    (status NOT_CONVERGED after exactly one step, with the step's true
    residual reported), while the default limit converges.  The next step is
    never enqueued ahead past the limit."""
    torch, dev = torch_dev
    s, o, u, ut = make(torch_dev, 2, 127, -10, 10, 1.5, 2.0, 0.01)
    b = s.rhs(ut)
    x1, i1 = s.solve(b, precision="fp32_ir", max_outer=1)
    assert i1.status == 1 and i1.outer_iters == 1 and 1e-10 < i1.relres_true < 1e-3
    x2, i2 = s.solve(b, precision="fp32_ir")
    assert i2.status == 0 and i2.outer_iters >= 2 and i2.relres_true < 1e-10
    bn = to_np(b)
    r = to_np(s.apply_A(x2)) - bn
    assert np.linalg.norm(r) / np.linalg.norm(bn) < 1e-10


def test_step_and_first_step(torch_dev):
    torch, dev = torch_dev
    d, n, lo, hi, alpha, rho, tau = 2, 63, -10.0, 10.0, 1.5, 2.0, 0.005
    s, o, u, ut = make(torch_dev, d, n, lo, hi, alpha, rho, tau, noise=0.0)
    u1t, i1 = s.first_step(ut)
    u1 = to_np(u1t)
    u1o, _ = o.first_step(u, tol=1e-13)
    assert np.linalg.norm(u1 - u1o) / np.linalg.norm(u1o) < 1e-9
    u2t, i2 = s.step(ut, u1t)
    u2o, _ = o.step(u, u1o, tol=1e-13)
    u2 = to_np(u2t)
    assert np.linalg.norm(u2 - u2o) / np.linalg.norm(u2o) < 1e-9
    # unitarity of the three-level step (mass invariant)
    assert abs(np.linalg.norm(u2) - np.linalg.norm(u)) / np.linalg.norm(u) < 1e-9
