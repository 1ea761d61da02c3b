"""The transform-schedule autotuner (fnls_autotune) on the GPU: it returns a
valid schedule, and solves with the tuned schedule agree with the default
schedule's and satisfy the oracle's residual test (d = 2, n = 1023 in FP64
and FP32-IR; d = 3, n = 63, which runs the generic line-length path)."""
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


@pytest.mark.parametrize("d,n,precision", [(2, 1023, "fp64"), (2, 1023, "fp32_ir"), (3, 63, "fp64")])
def test_autotune(torch_dev, d, n, precision):
    from paper_2410_03643_amd.fnls import Solver
    torch, dev = torch_dev
    lo, hi, alpha, rho, dt = -10.0, 10.0, 1.5, 2.0, 0.01
    h = (hi - lo) / (n + 1)
    u = inputs.soliton(d, n, lo, hi, noise=1e-3, seed=0)
    s = Solver(alpha, rho, d, n, h, dt, device=dev)
    ut = torch.from_numpy(u).to(dev)
    s.precond_setup(ut)
    b = s.rhs(ut)
    x0, i0 = s.solve(b, tol=1e-10, precision=precision)
    x0 = x0.cpu().numpy()
    cfg, ms = s.autotune(b, precision=precision, reps=3)
    x1, i1 = s.solve(b, tol=1e-10, precision=precision)
    x1 = x1.cpu().numpy()
    print("d=%d n=%d %s: tuned schedule %s, %.3f ms per solve, IT %d -> %d"
          % (d, n, precision, cfg, ms, i0.iters, i1.iters), flush=True)
    for kind in ("contiguous", "strided"):
        rm, li = cfg[kind]
        assert rm in (4, 8, 16) and li in (1, 2, 4)
    assert ms > 0.0
    o = oracle.OracleSolver(alpha, rho, d, n, h, dt)
    o.precond_setup(u)
    bo = b.cpu().numpy()
    res = np.linalg.norm(bo - o.apply_A(x1)) / np.linalg.norm(bo)
    assert i1.status == 0 and res < 1e-10 and abs(i1.iters - i0.iters) <= 1
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) <= 1e-8
