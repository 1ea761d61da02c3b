"""The host's GMRES sequencing on the GPU: iterations enqueued ahead of their
stopping decisions, stop predictions, cycle ends enqueued ahead and guarded
on the device, and the status reports read from pinned memory.  Every
setting must give bitwise the same iterates, iteration counts and cycle
counts as the fully synchronous loop (lookahead 0); the host's counters
(fnls_get_host_stats) show that each mechanism actually ran.

* Late read of a stop report: the testing option poll_delay_us makes the
  host sleep before each status wait, so the cycle end that was enqueued
  behind a predicted stop has already run, and its residual report has
  replaced the stop report, when the host reads.  The host must recognise
  that (late_reads > 0) and still return the right x.
* Several iterations in flight (lookahead 3) with restart cycles and the stop
  predictor firing: a guarded cycle end runs only when the cycle stops with
  the basis size it was enqueued for, so an earlier stop among the
  iterations in flight cannot apply the update twice.
"""
import numpy as np
import pytest

import oracle
from paper_2410_03643_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda", 0)


def make(torch_dev, d, n, alpha, rho, tau, lo=-10.0, hi=10.0):
    from paper_2410_03643_amd.fnls import Solver
    torch, dev = torch_dev
    h = (hi - lo) / (n + 1)
    u = inputs.soliton(d, n, lo, hi, noise=1e-3, seed=0)
    s = Solver(alpha, rho, d, n, h, tau, device=dev)
    ut = torch.from_numpy(u).to(dev)
    s.precond_setup(ut)
    return s, ut, u


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_late_read_of_stop_report(torch_dev, precision):
    torch, dev = torch_dev
    s, ut, u = make(torch_dev, 2, 255, 1.5, 2.0, 0.01)
    b = s.rhs(ut)
    x0, i0 = s.solve(b, precision=precision)
    s.host_stats(reset=True)
    x1, i1 = s.solve(b, precision=precision, poll_delay_us=20000)
    st = s.host_stats(reset=True)
    print("%s: IT %d/%d outer %d/%d stats %s" % (precision, i0.iters, i1.iters, i0.outer_iters, i1.outer_iters, st),
          flush=True)
    assert i0.status == 0 and i1.status == 0
    assert i0.iters == i1.iters and i0.outer_iters == i1.outer_iters
    assert torch.equal(x0, x1)
    assert st["stop_predictions"] >= 1 and st["ends_ahead"] >= 1
    assert st["late_reads"] >= 1
    # and the answer is right: the oracle's residual of x
    o = oracle.OracleSolver(1.5, 2.0, 2, 255, 20.0 / 256, 0.01)
    o.precond_setup(u)
    bn = b.cpu().numpy()
    xn = x1.cpu().numpy()
    assert np.linalg.norm(bn - o.apply_A(xn)) / np.linalg.norm(bn) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_lookahead3_restart_cycles_with_predictions(torch_dev, precision):
    torch, dev = torch_dev
    s, ut, u = make(torch_dev, 2, 255, 1.3, 2.0, 0.02)
    tol = 1e-13 if precision == "fp64" else 1e-11
    tot = {"stop_predictions": 0, "ends_ahead": 0, "early_stops": 0}
    for restart in (6, 8, 12):
        for seed in (41, 42, 43):
            b = torch.from_numpy(inputs.random_field(u.shape, seed=seed)).to(dev)
            ref, iref = s.solve(b, tol=tol, restart=restart, lookahead=0, precision=precision)
            assert iref.status == 0
            for la in (1, 3):
                s.host_stats(reset=True)
                x, info = s.solve(b, tol=tol, restart=restart, lookahead=la, precision=precision)
                st = s.host_stats(reset=True)
                print("seed %d restart %d lookahead %d: IT %d outer %d | %s"
                      % (seed, restart, la, info.iters, info.outer_iters, st), flush=True)
                assert info.status == 0
                assert info.iters == iref.iters and info.outer_iters == iref.outer_iters
                assert torch.equal(x, ref)
                if la == 3:
                    for k in tot:
                        tot[k] += st[k]
    # the predictor fired with three iterations in flight; its guarded cycle
    # ends mostly do not match the actual stop (an earlier iteration stops
    # the cycle), and the results above are still those of lookahead 0
    print("lookahead 3 totals: %s" % tot, flush=True)
    assert tot["stop_predictions"] >= 1
    if precision == "fp32_ir":
        assert tot["early_stops"] >= 1
