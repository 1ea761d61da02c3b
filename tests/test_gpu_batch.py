"""Batched solves through the C ABI (fnls_batch_*): many instances of uneven
sizes advanced together with one launch per pass for all of them.

* A mixed batch (d = 2, n in {31, 63, 127, 255}, different alpha, rho, and
  one zero right-hand side) against the single-instance path and the oracle:
  each instance's iteration count within 1 of the oracle's, x within 1e-10 of
  the oracle's solution at the same iteration count, oracle residual < tol;
  FP64 and FP32-IR.
* The batched workload at full size: 64 instances on [-10, 10]^2 with n
  drawn from {127, 255, 511, 1023}, alpha ~ U[1.1, 1.9], rho ~ U[0.5, 3],
  dt 0.01, soliton data with random centre and phase (seed 0); one
  three-level step of every instance in FP32-IR to 1e-10; every instance's
  FP64 residual below 1e-10, a sample checked by the oracle's operator; the
  batch timed against the same steps taken one instance at a time.
* Graph mode (opts.graph = 1): each Arnoldi iteration of all instances is one
  replay of a captured hipGraph.  Replays are checked bitwise against the
  direct launches of the same kernels, several times over with other GPU
  work and synchronisations in between; repeated calls with the same vectors
  replay cached graphs without capturing again.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2410_03643_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda", 0)


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


MIXED = [(31, 1.2, 0.5), (63, 1.5, 2.0), (127, 1.8, 1.0), (255, 1.4, 3.0), (63, 1.9, 2.5), (127, 1.1, 0.7),
         (31, 1.6, 2.0)]


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_mixed_batch_matches_single_and_oracle(torch_dev, precision):
    from paper_2410_03643_amd.fnls import Batch, Solver
    torch, dev = torch_dev
    lo, hi, dt = -10.0, 10.0, 0.01
    solvers, us, bs, probs = [], [], [], []
    for k, (n, alpha, rho) in enumerate(MIXED):
        h = (hi - lo) / (n + 1)
        u = inputs.soliton(2, n, lo, hi, center=[0.5 * k - 1.0, 0.3], phase=0.4 * k, noise=1e-3, seed=k)
        s = Solver(alpha, rho, 2, n, h, dt, device=dev)
        ut = torch.from_numpy(u).to(dev)
        s.precond_setup(ut)
        b = s.rhs(ut)
        if k == len(MIXED) - 1:
            b.zero_()                       # a zero right-hand side: x = 0, IT = 0
        solvers.append(s)
        us.append(u)
        bs.append(b)
        probs.append((n, alpha, rho, h))
    batch = Batch(solvers)
    xs, infos = batch.solve(bs, tol=TOL, precision=precision)
    for k, (s, b, x, info) in enumerate(zip(solvers, bs, xs, infos)):
        n, alpha, rho, h = probs[k]
        xn, bn = to_np(x), to_np(b)
        if k == len(MIXED) - 1:
            assert info.status == 0 and info.iters == 0 and np.abs(xn).max() == 0.0
            continue
        # the single-instance path on the same system
        x1, i1 = s.solve(b, tol=TOL, precision=precision)
        o = oracle.OracleSolver(alpha, rho, 2, n, h, dt)
        o.precond_setup(us[k])
        res = np.linalg.norm(bn - o.apply_A(xn)) / np.linalg.norm(bn)
        e1 = np.linalg.norm(xn - to_np(x1)) / np.linalg.norm(to_np(x1))
        msg = "instance %d n=%d: IT batch %d single %d outer %d, relres %.2e, |x - x_single| %.1e" % (
            k, n, info.iters, i1.iters, info.outer_iters, res, e1)
        if precision == "fp64":
            xo, io = o.solve(bn, tol=TOL)
            if io.iters != info.iters:
                xo, _ = o.solve(bn, fixed_iters=info.iters)
            eo = np.linalg.norm(xn - xo) / np.linalg.norm(xo)
            msg += ", oracle IT %d, |x - x_oracle| %.1e" % (io.iters, eo)
            assert abs(info.iters - io.iters) <= 1 and eo <= 1e-10
        print(msg, flush=True)
        assert info.status == 0 and res < TOL
        assert abs(info.iters - i1.iters) <= 1
        assert e1 <= 1e-8
    batch.close()


def test_batched_workload_64_instances(torch_dev):
    from paper_2410_03643_amd.fnls import Batch, Solver
    torch, dev = torch_dev
    cases = inputs.batched_cases(64)
    sizes = sorted(set(p.n for p in cases))
    print("64 instances, n counts %s" % {n: sum(p.n == n for p in cases) for n in sizes}, flush=True)
    solvers = [Solver(p.alpha, p.rho, p.d, p.n, p.h, p.tau, device=dev) for p in cases]
    us = [torch.from_numpy(p.u).to(dev) for p in cases]
    batch = Batch(solvers)
    outs = [torch.empty_like(u) for u in us]
    for _ in range(3):
        batch.step(us, us, outs, tol=TOL, precision="fp32_ir")
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        _, infos = batch.step(us, us, outs, tol=TOL, precision="fp32_ir")
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    # the same steps one instance at a time
    single = [torch.empty_like(u) for u in us]
    for s, u, o in zip(solvers, us, single):
        s.step(u, u, o, tol=TOL, precision="fp32_ir")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sinfos = [s.step(u, u, o, tol=TOL, precision="fp32_ir")[1] for s, u, o in zip(solvers, us, single)]
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / reps
    its = [i.iters for i in infos]
    print("batch: %.2f ms per step of all 64 (%.0f instance-steps/s); one at a time: %.2f ms (%.0f/s); "
          "speed-up %.2f; IT %d-%d, max relres %.2e"
          % (1e3 * tb, 64 / tb, 1e3 * ts, 64 / ts, ts / tb, min(its), max(its), max(i.relres_true for i in infos)),
          flush=True)
    assert all(i.status == 0 and i.relres_true < TOL for i in infos)
    assert all(abs(a.iters - b.iters) <= 1 for a, b in zip(infos, sinfos))
    # one instance of every size class against the oracle's FP64 solution of
    # its system (to 1e-13): within cond(A) * (relres + 1e-13)
    for n in sizes:
        k = next(i for i, p in enumerate(cases) if p.n == n)
        p = cases[k]
        o = oracle.OracleSolver(p.alpha, p.rho, p.d, p.n, p.h, p.tau)
        o.precond_setup(p.u)
        b = o.rhs(p.u)
        xo, io = o.solve(b, tol=1e-13)
        x = to_np(outs[k])
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        kap = kappa_bound(p)
        print("instance %d (n=%d): |x_batch - x_oracle| / |x_oracle| = %.2e (cond bound %.1f, relres %.2e)"
              % (k, n, err, kap, infos[k].relres_true), flush=True)
        assert err <= kap * (infos[k].relres_true + 1e-13)
    # the oracle's residual for a sample of instances, and agreement with the single path
    for k in range(0, 64, 9):
        p = cases[k]
        o = oracle.OracleSolver(p.alpha, p.rho, p.d, p.n, p.h, p.tau)
        o.precond_setup(p.u)
        b = o.rhs(p.u)
        x = to_np(outs[k])
        res = np.linalg.norm(b - o.apply_A(x)) / np.linalg.norm(b)
        e1 = np.linalg.norm(x - to_np(single[k])) / np.linalg.norm(to_np(single[k]))
        print("instance %d (n=%d): oracle residual %.2e, |x_batch - x_single| %.1e" % (k, p.n, res, e1), flush=True)
        assert res < TOL and e1 <= 1e-8
    batch.close()


def kappa_bound(p):
    """cond_2(A) <= sqrt(1 + ||B||^2) for A = B + iI, B = D - T_d real
    symmetric: ||T_d|| <= d mu 2 c_0 (Gershgorin, sum |c_k| = 2 c_0) and
    ||D|| <= rho dt max |u|^2."""
    from oracle import fcd
    c0 = fcd.coefficients(p.alpha, 2)[0]
    nB = p.d * fcd.mu(p.alpha, p.h, p.tau) * 2.0 * c0 + p.rho * p.tau * float(np.abs(p.u).max() ** 2)
    return float(np.sqrt(1.0 + nB * nB))


def test_batched_workload_autotuned(torch_dev):
    """The 64-instance workload with autotuned schedules: fnls_batch_autotune
    times batched solves over radix x lines for each line-length class with a
    compile-time plan (m = 256, 512, 1024) and keeps what is faster, and the
    batch then launches each class with its schedule.  Timed against the
    default schedule (radix 4, 1024 threads) and not slower (5 % for noise);
    every instance still converges, and its solution agrees with the
    default one within cond(A) * (relres + relres)."""
    from paper_2410_03643_amd.fnls import Batch, Solver
    torch, dev = torch_dev
    cases = inputs.batched_cases(64)
    solvers = [Solver(p.alpha, p.rho, p.d, p.n, p.h, p.tau, device=dev) for p in cases]
    us = [torch.from_numpy(p.u).to(dev) for p in cases]
    batch = Batch(solvers)

    def timed(outs):
        batch.step(us, us, outs, tol=TOL, precision="fp32_ir")
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            _, infos = batch.step(us, us, outs, tol=TOL, precision="fp32_ir")
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, infos

    x_def = [torch.empty_like(u) for u in us]
    t_def, i_def = timed(x_def)
    bs = []
    for s, u in zip(solvers, us):
        s.precond_setup(u)
        bs.append(s.rhs(u))
    t0 = time.perf_counter()
    classes = batch.autotune(bs, precision="fp32_ir", reps=2)
    t_tune = time.perf_counter() - t0
    chosen = {n: (batch.schedule(n, "fp32_ir", strided=False), batch.schedule(n, "fp32_ir", strided=True))
              for n in sorted({p.n for p in cases if p.n + 1 in (256, 512, 1024)})}
    print("schedules (contiguous, strided) as (rmax, lines): %s" % chosen, flush=True)
    x_tun = [torch.empty_like(u) for u in us]
    t_tun, i_tun = timed(x_tun)
    print("64 instances, FP32-IR step of all: default schedules %.2f ms, autotuned %.2f ms (%d classes tuned in "
          "%.1f s)" % (1e3 * t_def, 1e3 * t_tun, classes, t_tune), flush=True)
    assert classes == len({p.n for p in cases if p.n + 1 in (256, 512, 1024)})
    assert t_tun <= 1.05 * t_def
    worst = 0.0
    for k, p in enumerate(cases):
        assert i_tun[k].status == 0 and i_tun[k].relres_true < TOL
        assert abs(i_tun[k].iters - i_def[k].iters) <= 2
        e = float(torch.linalg.vector_norm(x_tun[k] - x_def[k]).item() / torch.linalg.vector_norm(x_def[k]).item())
        worst = max(worst, e / kappa_bound(p))
        assert e <= kappa_bound(p) * (i_tun[k].relres_true + i_def[k].relres_true)
    print("largest |x_tuned - x_default| / |x_default| / cond bound: %.2e" % worst, flush=True)
    batch.close()


def bitwise_equal(a, b):
    import torch
    return bool(torch.equal(torch.view_as_real(a), torch.view_as_real(b)))


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_graph_mode_replays_match_direct_launches(torch_dev, precision):
    from paper_2410_03643_amd.fnls import Batch, Solver
    torch, dev = torch_dev
    lo, hi, dt = -10.0, 10.0, 0.01
    solvers, bs = [], []
    for k, (n, alpha, rho) in enumerate(MIXED[:-1]):
        h = (hi - lo) / (n + 1)
        u = inputs.soliton(2, n, lo, hi, center=[0.5 * k - 1.0, 0.3], phase=0.4 * k, noise=1e-3, seed=k)
        s = Solver(alpha, rho, 2, n, h, dt, device=dev)
        ut = torch.from_numpy(u).to(dev)
        s.precond_setup(ut)
        solvers.append(s)
        bs.append(s.rhs(ut))
    batch = Batch(solvers)
    ref, rinfo = batch.solve(bs, tol=TOL, precision=precision)
    ref = [x.clone() for x in ref]
    outs = [torch.empty_like(x) for x in ref]
    counts = []
    for rep in range(4):
        for x in outs:
            x.fill_(float("nan"))
        _, ginfo = batch.solve(bs, outs, tol=TOL, precision=precision, graph=True)
        torch.cuda.synchronize()
        same = [bitwise_equal(x, r) for x, r in zip(outs, ref)]
        its = [(a.iters, b.iters) for a, b in zip(ginfo, rinfo)]
        counts.append(batch.graph_stats())
        print("replay round %d: bitwise equal %s, IT (graph, direct) %s, graphs (captured, launched) %s"
              % (rep, same, its, counts[-1]), flush=True)
        assert all(same)
        assert all(a.iters == b.iters and a.status == b.status for a, b in zip(ginfo, rinfo))
        # other GPU work and a direct-launch solve between the replays
        junk = torch.randn(1 << 20, device=dev).cumsum(0)
        _, dinfo = batch.solve(bs, [torch.empty_like(x) for x in ref], tol=TOL, precision=precision)
        torch.cuda.synchronize()
        del junk
    assert counts[0][0] >= 1 and counts[0][1] >= sum(i.iters for i in rinfo) // len(rinfo)
    assert all(c[0] == counts[0][0] for c in counts), "repeated calls captured new graphs"
    assert all(b[1] > a[1] for a, b in zip(counts, counts[1:]))
    batch.close()


def test_batched_workload_graph_mode(torch_dev):
    from paper_2410_03643_amd.fnls import Batch, Solver
    torch, dev = torch_dev
    cases = inputs.batched_cases(64)
    solvers = [Solver(p.alpha, p.rho, p.d, p.n, p.h, p.tau, device=dev) for p in cases]
    us = [torch.from_numpy(p.u).to(dev) for p in cases]
    batch = Batch(solvers)
    direct = [torch.empty_like(u) for u in us]
    graph = [torch.empty_like(u) for u in us]
    times = {}
    for name, outs, g in (("direct", direct, False), ("graph", graph, True), ("direct", direct, False),
                          ("graph", graph, True)):
        batch.step(us, us, outs, tol=TOL, precision="fp32_ir", graph=g)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            _, infos = batch.step(us, us, outs, tol=TOL, precision="fp32_ir", graph=g)
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / reps
        assert all(i.status == 0 and i.relres_true < TOL for i in infos)
    same = [bitwise_equal(a, b) for a, b in zip(direct, graph)]
    print("64 instances, one FP32-IR step of all: direct launches %.2f ms, graph replays %.2f ms; "
          "graphs (captured, launched) %s; bitwise equal %d / 64"
          % (1e3 * times["direct"], 1e3 * times["graph"], batch.graph_stats(), sum(same)), flush=True)
    assert all(same)
    batch.close()
