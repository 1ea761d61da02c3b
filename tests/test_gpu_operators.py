"""Operator parity at the full workload sizes, the complex64 operators of the
GMRES-IR inner solve, and the boundary's error paths on a real context.

* FP64 y = A x (Sec. 2.1 / 2.2, Kronecker sum) and z = Ptilde^{-1} r (the
  complex form of the Sec. 4 preconditioner) at d = 2, n = 1023 (the strided
  m = 1024 plan over 1,023 lines) and d = 3, n = 255 (more than 1,024
  workgroups per pass), element by element against the oracle: max-norm
  relative error <= 1e-12.
* The same operators on complex64 vectors (fnls_apply_A_c64 /
  fnls_apply_precond_c64: the FP32 kernels, tables and diagonal of the inner
  iteration) against the oracle applied to the same (rounded) input in FP64,
  max-norm error relative to the largest output.  A x: each m-point FFT
  stage adds a few FP32 roundings relative to the line's magnitude, log2(m)
  stages per transform and d axes, so the bound is 4 d log2(m) 2^-24.
  Ptilde^{-1} r: every sine transform recovers half of its outputs as a
  prefix sum over up to m/2 FFT outputs, so the FFT's rounding errors add up
  like a random walk of m/2 steps, each carrying the FFT's own error of up
  to log2(m) roundings: about sqrt(m/2) log2(m) / 2 roundings per transform,
  normwise (an FP32 emulation of the same recovery with numpy's FFT
  measures 6, 10 and 34 roundings at m = 64, 256, 1024; the kernels, whose
  twiddle powers are products, about three times that).  With two
  transforms per axis the normwise bound is d sqrt(m) log2(m) 2^-24; the
  largest single error is a few times the normwise one (bound: 8 times).
* fnls_assemble on a real context returns the status of the context-free
  checker for bad arguments and leaves the context unassembled; calls made
  before assemble or before precond_setup return FNLS_ERR_STATE.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
from paper_2410_03643_amd import inputs

pytestmark = pytest.mark.gpu

OP_TOL = 1e-12
EPS32 = 2.0 ** -24


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda", 0)


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def make(torch_dev, d, n, lo, hi, alpha, rho, tau, restart=30):
    from paper_2410_03643_amd.fnls import Solver
    torch, dev = torch_dev
    h = (hi - lo) / (n + 1)
    u = inputs.soliton(d, n, lo, hi, noise=1e-3, seed=0)
    s = Solver(alpha, rho, d, n, h, tau, device=dev, restart=restart)
    o = oracle.OracleSolver(alpha, rho, d, n, h, tau)
    s.precond_setup(torch.from_numpy(u).to(dev))
    o.precond_setup(u)
    return s, o


FULL = [(2, 1023, -10.0, 10.0, 1.5, 2.0, 0.01), (3, 255, -8.0, 8.0, 1.6, 1.0, 0.01)]


@pytest.mark.parametrize("case", FULL, ids=["d2_n1023", "d3_n255"])
def test_fp64_operators_full_size(torch_dev, case):
    torch, dev = torch_dev
    d, n = case[:2]
    print("fp64 operators d=%d n=%d" % (d, n), flush=True)
    s, o = make(torch_dev, *case, restart=1)
    x = inputs.random_field((n,) * d, seed=31)
    xt = torch.from_numpy(x).to(dev)
    y = to_np(s.apply_A(xt))
    z = to_np(s.apply_precond(xt))
    del xt
    ey = relerr(y, o.apply_A(x))
    ez = relerr(z, o.apply_Pinv(x))
    print("d=%d n=%d: A x %.2e, Ptilde^-1 r %.2e (bound %.0e)" % (d, n, ey, ez, OP_TOL), flush=True)
    assert ey < OP_TOL and ez < OP_TOL


C64_CASES = [(1, 63, -20.0, 20.0, 1.5, 2.0, 0.01), (1, 1023, -20.0, 20.0, 1.5, 2.0, 0.01),
             (2, 127, -10.0, 10.0, 1.3, 2.0, 0.01), (2, 1023, -10.0, 10.0, 1.5, 2.0, 0.01),
             (3, 31, -8.0, 8.0, 1.8, 1.0, 0.01), (3, 255, -8.0, 8.0, 1.6, 1.0, 0.01)]


def c64_bound_A(d, n):
    return 4.0 * d * math.log2(n + 1) * EPS32


def c64_bound_P(d, n):
    return d * math.sqrt(n + 1) * math.log2(n + 1) * EPS32


def normerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("case", C64_CASES, ids=["d%d_n%d" % c[:2] for c in C64_CASES])
def test_c64_operators_against_oracle(torch_dev, case):
    torch, dev = torch_dev
    d, n = case[:2]
    print("complex64 operators d=%d n=%d" % (d, n), flush=True)
    s, o = make(torch_dev, *case, restart=1)
    x32 = inputs.random_field((n,) * d, seed=37).astype(np.complex64)
    x = x32.astype(np.complex128)            # the input the kernels see, exactly
    xt = torch.from_numpy(x32).to(dev)
    y = to_np(s.apply_A_c64(xt)).astype(np.complex128)
    z = to_np(s.apply_precond_c64(xt)).astype(np.complex128)
    del xt
    zref = o.apply_Pinv(x)
    ey = relerr(y, o.apply_A(x))
    ez, ezn = relerr(z, zref), normerr(z, zref)
    by, bz = c64_bound_A(d, n), c64_bound_P(d, n)
    print("d=%d n=%d: A x max %.2e (%.1f roundings, bound %.2e); Ptilde^-1 r normwise %.2e (%.1f roundings, "
          "bound %.2e), max %.2e (%.1f roundings)" % (d, n, ey, ey / EPS32, by, ezn, ezn / EPS32, bz, ez,
                                                      ez / EPS32), flush=True)
    assert ey < by
    assert ezn < bz and ez < 8 * bz
    # the FP32 kernels do round: far from FP64 agreement, far from garbage
    assert max(ey, ez) > 1e-12


def test_c64_operators_reject_bad_arguments(torch_dev):
    from paper_2410_03643_amd.fnls import FnlsError, ERR_INVALID_ARG
    torch, dev = torch_dev
    s, o = make(torch_dev, 2, 31, -10.0, 10.0, 1.5, 2.0, 0.01, restart=1)
    x = torch.zeros((31, 31), dtype=torch.complex64, device=dev)
    with pytest.raises(FnlsError) as e:
        s.apply_A_c64(x, out=x)
    assert e.value.code == ERR_INVALID_ARG
    with pytest.raises(ValueError):
        s.apply_precond_c64(x.to(torch.complex128))


def test_assemble_errors_on_a_context_match_the_checker(torch_dev):
    """fnls_assemble on a live context returns the checker's status for every
    kind of bad argument (before touching the device), leaves the context
    unassembled (FNLS_ERR_STATE afterwards), and a good call then works."""
    from paper_2410_03643_amd import fnls
    torch, dev = torch_dev
    L = fnls.lib()
    ctx = ctypes.c_void_p()
    assert L.fnls_create(ctypes.byref(ctx), 0, ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)) == 0
    try:
        d, n = 2, 63
        nbytes = L.fnls_workspace_bytes(d, n, 4)
        ws = torch.empty(nbytes + 512, dtype=torch.uint8, device=dev)
        base = (ws.data_ptr() + 255) // 256 * 256
        good = dict(alpha=1.5, rho=2.0, d=d, n=n, h=20.0 / 64, tau=0.01, ws=base, nbytes=nbytes)
        bad = [dict(alpha=0.9), dict(alpha=2.5), dict(rho=-1.0), dict(d=4), dict(n=62), dict(h=0.0),
               dict(tau=-0.01), dict(ws=0), dict(ws=base + 64), dict(nbytes=16)]
        for kw in bad:
            a = dict(good, **kw)
            msg = ctypes.create_string_buffer(256)
            want = L.fnls_check_assemble(a["alpha"], a["rho"], a["d"], a["n"], a["h"], a["tau"],
                                         ctypes.c_void_p(a["ws"]) if a["ws"] else None, a["nbytes"], msg, 256)
            got = L.fnls_assemble(ctx, a["alpha"], a["rho"], a["d"], a["n"], a["h"], a["tau"],
                                  ctypes.c_void_p(a["ws"]) if a["ws"] else None, a["nbytes"])
            assert want < 0 and got == want, (kw, want, got)
            assert msg.value and msg.value == L.fnls_last_error(ctx), (msg.value, L.fnls_last_error(ctx))
        u = torch.zeros((n, n), dtype=torch.complex128, device=dev)
        b = torch.ones((n, n), dtype=torch.complex128, device=dev)
        x = torch.empty_like(b)
        vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        # nothing assembled yet
        assert L.fnls_precond_setup(ctx, vp(u), None, 1.0) == fnls.ERR_STATE
        assert L.fnls_solve(ctx, vp(b), vp(x), None, None) == fnls.ERR_STATE
        a = good
        assert L.fnls_assemble(ctx, a["alpha"], a["rho"], a["d"], a["n"], a["h"], a["tau"],
                               ctypes.c_void_p(a["ws"]), a["nbytes"]) == fnls.OK
        # assembled, but no preconditioner setup yet
        assert L.fnls_solve(ctx, vp(b), vp(x), None, None) == fnls.ERR_STATE
        assert L.fnls_apply_A(ctx, vp(b), vp(x)) == fnls.ERR_STATE
        assert L.fnls_apply_precond(ctx, vp(b), vp(x)) == fnls.ERR_STATE
        assert L.fnls_rhs(ctx, vp(b), vp(x)) == fnls.ERR_STATE
        assert b"precond_setup" in L.fnls_last_error(ctx)
        assert L.fnls_precond_setup(ctx, vp(u), None, 1.0) == fnls.OK
        info = fnls.Info()
        opts = fnls.default_opts()
        opts.restart = 5     # more than the workspace holds (4)
        assert L.fnls_solve(ctx, vp(b), vp(x), ctypes.byref(opts), ctypes.byref(info)) == fnls.ERR_WORKSPACE
        opts.restart = 4
        assert L.fnls_solve(ctx, vp(b), vp(x), ctypes.byref(opts), ctypes.byref(info)) == fnls.OK
        assert info.relres_true < 1e-10
        torch.cuda.synchronize()
    finally:
        L.fnls_destroy(ctx)
