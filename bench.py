#!/usr/bin/env python3
"""Benchmark: preconditioned GMRES solves per second on one MI355X.

Workload (default): the d = 2, n = 1023 system (1,046,529 complex unknowns)
on [-10, 10]^2 with alpha = 1.5, rho = 2, dt = 0.01, u = sech(|x|) exp(i x_1)
plus 1e-3 complex noise (seed 0); right-preconditioned GMRES(30) with the
sine-transform TBAN preconditioner (omega = 1), tolerance 1e-10.
--workload d3: the d = 3, n = 255 system on [-8, 8]^3 (16,581,375 unknowns),
alpha = 1.6, rho = 1, dt = 0.01 (profiling of the HBM-resident case).
--workload batch64: 64 independent d = 2 instances (n drawn from 127, 255,
511, 1023; alpha, rho, soliton centre and phase drawn with seed 0), one
FP32-IR time step of all of them per step through the batched solver, with
direct launches and with hipGraph replays (profiling of the batched path).

One step = one time-step solve of the whole hot path through the C ABI:
preconditioner setup D = rho dt |u|^2, right-hand side b = (iI + T - D) u, and
the GMRES solve (FP64, or FP32 GMRES-IR with --precision fp32_ir; both are
timed and reported).  The operator tables are assembled once before timing
(they depend only on alpha, h, dt).  Inputs are resident in HBM.

Prints one JSON line (rank 0, N = 1).  "roofline" is for the dominant kernel
class of the headline precision: its minimal algorithmic bytes per launch
(each vector the method must move, charged once; the first Gram-Schmidt
sweep to the pass that forms w) over its average launch duration from HIP
events around each launch, in a separate instrumented run of the same
steps; "step_roofline" does the same for the whole step.  "cpu_baseline"
times the CPU oracle on a bounded sample of the same workload (all host
threads and one thread), and in that leg the oracle's FP64 solution gives
the GPU solutions' errors.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TOL = 1e-10
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 256 << 20
TRAFFIC_FILES = {"metric": os.path.join(ROOT, "profiles", "traffic_pass64_toep_next_wdots_d2_n1023.txt"),
                 "d3": os.path.join(ROOT, "profiles", "traffic_pass64_toep_next_wdots_d3_n255.txt")}
METRIC = "PGMRES solves/s at d=2 n=1023 (FP64 vs FP32-IR @1e-10); % HBM roofline"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def time_steps(torch, s, u, un, steps, precision):
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    info = None
    for _ in range(steps):
        _, info = s.step(u, u, out=un, tol=TOL, precision=precision)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ev0.elapsed_time(ev1) / 1e3, info


def kernel_profile(torch, s, u, un, steps, precision):
    """Per kernel class over `steps` instrumented steps: launches, average
    duration, minimal and multi-pass algorithmic bytes per launch."""
    s.timing(True)
    for _ in range(steps):
        s.step(u, u, out=un, tol=TOL, precision=precision)
    rep = s.timing_report()
    s.timing(False)
    for r in rep:
        r["avg_us"] = 1e3 * r["total_ms"] / r["launches"]
        r["bytes_per_launch"] = r["bytes_min"] / r["launches"]
        r["multipass_bytes_per_launch"] = r["bytes"] / r["launches"]
        r["gbs"] = r["bytes_per_launch"] / (r["avg_us"] * 1e-6) / 1e9
        r["multipass_gbs"] = r["multipass_bytes_per_launch"] / (r["avg_us"] * 1e-6) / 1e9
        r["ms_per_step"] = r["total_ms"] / steps
    rep.sort(key=lambda r: -r["total_ms"])
    return rep


def copy_bandwidth(torch, dev, nbytes=512 << 20, reps=10):
    """Device-to-device copy rate (bytes read + written per second, GB/s) of a
    plain torch copy of nbytes, best of `reps` event-timed copies."""
    src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        best = t if best is None else min(best, t)
    del src, dst
    return 2.0 * nbytes / best / 1e9


def source_hash():
    """SHA-256 over the HIP sources and headers the library is built from."""
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2410_03643_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(src, "*"))):
        if f.endswith((".hip", ".h", ".hpp")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def read_keyvals(path):
    out = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                out[k.strip()] = v.strip().strip("`")
    return out


def committed_traffic(workload, timing_name):
    """HBM bytes per launch of `timing_name` from the committed counter summary
    of the workload, or None when there is none or the kernels changed since
    it was taken."""
    path = TRAFFIC_FILES[workload]
    if not os.path.exists(path):
        return None
    kv = read_keyvals(path)
    if kv.get("timing_name") != timing_name or kv.get("source_sha256") != source_hash():
        return None
    return float(kv["hbm_bytes_per_launch"])


def summarize(dirs, timing_name, kernel_regex):
    """Markdown summary of rocprofv3 CSV output (kernel stats and/or counters)."""
    import re
    rx = re.compile(kernel_regex) if kernel_regex else None
    lines = []
    per = {}   # (counter, kernel) -> [values]
    for d in dirs:
        for f in sorted(glob.glob(os.path.join(d, "**", "*_kernel_stats.csv"), recursive=True)):
            lines.append("Kernel statistics (`%s`), durations in microseconds:" % os.path.basename(f))
            lines.append("")
            lines.append("| kernel | calls | avg us | min us | max us | total us | % |")
            lines.append("|---|---|---|---|---|---|---|")
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    lines.append("| `%s` | %s | %.2f | %.2f | %.2f | %.1f | %.2f |" % (
                        r["Name"], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                        float(r["MaxNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e3, float(r["Percentage"])))
            lines.append("")
        for f in sorted(glob.glob(os.path.join(d, "**", "*_counter_collection.csv"), recursive=True)):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    per.setdefault((r["Counter_Name"], r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    if per:
        lines.append("Counters, KiB per dispatch (mean over the dispatches that did work: a launch")
        lines.append("enqueued ahead of the solver's stop decision that the device then skipped moves")
        lines.append("almost nothing and is left out, as counted in the last column):")
        lines.append("")
        lines.append("| counter | kernel | dispatches | mean KiB | skipped |")
        lines.append("|---|---|---|---|---|")
        factors = {}
        for (cn, kn), vals in sorted(per.items()):
            skipped = 0
            if kn == COPY_KERNEL:
                # the calibration copies are the large dispatches of the copy kernel
                vals = [v for v in vals if v >= 0.5 * max(vals)]
                factors[cn] = (COPY_BYTES / 1024.0) / (sum(vals) / len(vals))
            elif max(vals) > 0:
                work = [v for v in vals if v >= 0.01 * max(vals)]
                skipped = len(vals) - len(work)
                vals = work
            per[(cn, kn)] = vals
            lines.append("| %s | `%s` | %d | %.1f | %d |" % (cn, kn, len(vals), sum(vals) / len(vals), skipped))
        lines.append("")
        for cn, fct in sorted(factors.items()):
            lines.append("- %s_copy_factor: %.4f" % (cn.lower(), fct))
        if rx:
            tot = 0.0
            for cn in ("FETCH_SIZE", "WRITE_SIZE"):
                vals = [v for (c, kn), vs in per.items() if c == cn and rx.search(kn) for v in vs]
                if not vals or cn not in factors:
                    tot = None
                    break
                b = sum(vals) / len(vals) * 1024.0 * factors[cn]
                lines.append("- %s_bytes_per_launch: %.0f" % (cn.lower(), b))
                tot += b
            if tot is not None:
                lines.append("- timing_name: %s" % timing_name)
                lines.append("- hbm_bytes_per_launch: %.0f" % tot)
                lines.append("- source_sha256: %s" % source_hash())
    print("\n".join(lines))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, seconds, x64, x32):
    """The oracle's own step (D, b, FP64 GMRES(30) to 1e-10, dense per-axis
    operators) timed on the host's cores, with all BLAS threads and with one,
    about `seconds` each; then the oracle's FP64 solution of the same system
    to 1e-13, against which the GPU's FP64 and FP32-IR solutions (copied to
    the host after the timed region) are measured."""
    import numpy as np
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    o = oracle.OracleSolver(p.alpha, p.rho, p.d, p.n, p.h, p.tau)

    def timed(limit):
        with threadpool_limits(limits=limit):
            t0 = time.perf_counter()
            count, iters = 0, None
            while True:
                _, info = o.step(p.u, p.u, tol=TOL)
                count += 1
                iters = info.iters
                if time.perf_counter() - t0 >= seconds:
                    break
            return count, iters, time.perf_counter() - t0

    n_all, it_all, t_all = timed(threads)
    n_one, it_one, t_one = timed(1)
    o.precond_setup(p.u)
    b = o.rhs(p.u)
    xo, _ = o.solve(b, tol=1e-13)
    nx = float(np.linalg.norm(xo))
    errs = {"fp64": float(np.linalg.norm(x64 - xo)) / nx, "fp32_ir": float(np.linalg.norm(x32 - xo)) / nx}
    base = {"value": n_all / t_all, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "value_1thread": n_one / t_one, "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "sample": "oracle time-step solves (D, b, FP64 GMRES(30) to 1e-10, %d iterations each) of the "
                      "same %s system: %d in %.1f s on %d BLAS threads, %d in %.1f s on 1 thread"
                      % (it_all, p.name, n_all, t_all, threads, n_one, t_one)}
    return base, errs


def batch_bench(args, torch, dev):
    """64 batched d = 2 instances, one FP32-IR time step of all per step:
    direct launches and hipGraph replays timed alike.  The whole-step
    roofline charges each instance the minimal-traffic bytes of its own
    step (the single-instance timing records of the same step, whose
    iteration counts the batch matches within one)."""
    from paper_2410_03643_amd import inputs
    from paper_2410_03643_amd.fnls import Batch, Solver
    cases = inputs.batched_cases(64)
    sizes = sorted(set(p.n for p in cases))
    counts = {n: sum(p.n == n for p in cases) for n in sizes}
    log("batch64: n counts %s, %d unknowns" % (counts, sum(p.N for p in cases)))
    solvers = [Solver(p.alpha, p.rho, p.d, p.n, p.h, p.tau, device=dev) for p in cases]
    us = [torch.from_numpy(p.u).to(dev) for p in cases]
    outs = [torch.empty_like(u) for u in us]
    batch = Batch(solvers)
    times, infos = {}, None
    for mode in ("direct", "graph"):
        g = mode == "graph"
        for _ in range(args.warmup):
            batch.step(us, us, outs, tol=TOL, precision="fp32_ir", graph=g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, infos = batch.step(us, us, outs, tol=TOL, precision="fp32_ir", graph=g)
        torch.cuda.synchronize()
        times[mode] = (time.perf_counter() - t0) / args.steps
        assert all(i.status == 0 and i.relres_true < TOL for i in infos), "a batched solve missed the tolerance"
        log("batch64 %s: %.3f ms per step of all 64" % (mode, 1e3 * times[mode]))
    # minimal-traffic bytes of each instance's step, from its own timed step
    alg, single_its = 0.0, []
    for s, u, o in zip(solvers, us, outs):
        s.timing(True)
        _, si = s.step(u, u, out=o, tol=TOL, precision="fp32_ir")
        rep = s.timing_report()
        s.timing(False)
        alg += sum(r["bytes_min"] for r in rep)
        single_its.append(si.iters)
    batch.close()
    its = [i.iters for i in infos]
    assert all(abs(a - b) <= 1 for a, b in zip(its, single_its))
    t = times["direct"]
    gbs = alg / t / 1e9
    out = {
        "metric": "batched PGMRES instance-steps/s: 64 d=2 instances, n in {127,255,511,1023}, FP32-IR @1e-10",
        "value": round(64 / t, 1), "unit": "instance-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * t, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "batch64: 64 independent d=2 instances on [-10,10]^2, dt=0.01, n counts %s, "
                               "alpha ~ U[1.1,1.9], rho ~ U[0.5,3], soliton with random centre and phase "
                               "(seed 0); one FP32-IR time step of all per step" % counts,
                   "instances": 64, "unknowns": sum(p.N for p in cases), "tol": TOL},
        "iters_min": min(its), "iters_max": max(its),
        "graph": {"value": round(64 / times["graph"], 1), "ms_per_step": round(1e3 * times["graph"], 4)},
        "step_roofline": {"alg_bytes": int(alg), "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                          "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=["metric", "d3", "batch64"], default="metric",
                    help="metric: d=2 n=1023 (the headline); d3: d=3 n=255; batch64: 64 batched d=2 "
                         "instances (both for profiling)")
    ap.add_argument("--precision", choices=["fp64", "fp32_ir"], default="fp64",
                    help="precision of the headline value (both are measured)")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run three plain 256 MiB device copies (reference for HBM byte counters)")
    ap.add_argument("--summarize", nargs="+", metavar="DIR",
                    help="print a markdown summary of rocprofv3 CSV output directories and exit (no GPU)")
    ap.add_argument("--kernel-regex", default=None,
                    help="with --summarize: the kernel whose counters give the traffic figure")
    ap.add_argument("--timing-name", default="pass64.toep_next_wdots.ax0",
                    help="with --summarize: that kernel's name in the per-launch timing report")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize, args.timing_name, args.kernel_regex)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_03643_amd import inputs
    from paper_2410_03643_amd.fnls import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    if args.workload == "batch64":
        batch_bench(args, torch, dev)
        return
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x %d MiB device-to-device copies" % (COPY_BYTES >> 20))
        del src, dst
    p = inputs.metric_case() if args.workload == "metric" else inputs.three_dim_case()
    log("workload %s: N=%d" % (p.name, p.N))
    s = Solver(p.alpha, p.rho, p.d, p.n, p.h, p.tau, device=dev, restart=30)
    u = torch.from_numpy(p.u).to(dev)
    un = torch.empty_like(u)

    results = {}
    for prec in ("fp64", "fp32_ir"):
        log("%s: warmup %d" % (prec, args.warmup))
        for _ in range(args.warmup):
            s.step(u, u, out=un, tol=TOL, precision=prec)
        torch.cuda.synchronize()
        log("%s: timing %d steps" % (prec, args.steps))
        wall, gpu, info = time_steps(torch, s, u, un, args.steps, prec)
        log("%s: %.3f ms/step wall, %.3f ms/step events, IT=%d outer=%d relres=%.2e"
            % (prec, 1e3 * wall / args.steps, 1e3 * gpu / args.steps, info.iters,
               info.outer_iters, info.relres_true))
        assert info.status == 0 and info.relres_true < TOL, "solve did not reach the tolerance"
        x_host = un.cpu().numpy()          # after the timed region
        log("%s: kernel profile over %d steps" % (prec, args.profile_steps))
        prof = kernel_profile(torch, s, u, un, args.profile_steps, prec)
        results[prec] = dict(wall=wall, gpu=gpu, info=info, prof=prof, x=x_host)
    copy_gbs = copy_bandwidth(torch, dev)
    log("device copy: %.0f GB/s (read + write)" % copy_gbs)

    head = results[args.precision]
    other = "fp32_ir" if args.precision == "fp64" else "fp64"
    steps = args.steps
    dom = head["prof"][0]
    traffic = committed_traffic(args.workload, dom["name"])
    roofline = {"bound": "hbm", "kernel": dom["name"], "achieved": round(dom["gbs"], 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(dom["gbs"] / PEAK_HBM_GBS, 4),
                "traffic": None if traffic is None else int(traffic), "avg_us": round(dom["avg_us"], 2),
                "bytes_per_launch": int(dom["bytes_per_launch"]),
                "multipass_bytes_per_launch": int(dom["multipass_bytes_per_launch"]),
                "multipass_achieved": round(dom["multipass_gbs"], 1),
                "multipass_frac": round(dom["multipass_gbs"] / PEAK_HBM_GBS, 4),
                "measured_copy_gbs": round(copy_gbs, 1),
                "frac_of_measured_copy": round(dom["gbs"] / copy_gbs, 4)}
    step_ms = 1e3 * head["wall"] / steps
    alg_step = sum(r["bytes_min"] for r in head["prof"]) / args.profile_steps
    multi_step = sum(r["bytes"] for r in head["prof"]) / args.profile_steps
    step_gbs = alg_step / (step_ms * 1e-3) / 1e9
    step_roofline = {"alg_bytes": int(alg_step), "alg_bytes_per_unknown": round(alg_step / p.N, 1),
                     "achieved": round(step_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(step_gbs / PEAK_HBM_GBS, 4),
                     "ceiling_steps_per_s": round(PEAK_HBM_GBS * 1e9 / alg_step, 1),
                     "multipass_bytes": int(multi_step)}
    ws = "d=2 n=1023 [-10,10]^2 rho=2 dt=0.01" if args.workload == "metric" else "d=3 n=255 [-8,8]^3 rho=1 dt=0.01"
    out = {
        "metric": METRIC if args.workload == "metric" else "PGMRES solves/s at d=3 n=255 (FP64 vs FP32-IR @1e-10)",
        "value": round(steps / head["wall"], 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": p.name + ": " + ws + ", sech soliton + 1e-3 noise (seed 0), one time-step "
                   "solve (setup + rhs + GMRES(30), tol 1e-10)",
                   "d": p.d, "n": p.n, "unknowns": p.N, "restart": 30, "tol": TOL,
                   "precision": args.precision},
        "iters": head["info"].iters,
        "outer_iters": head["info"].outer_iters,
        "relres_true": head["info"].relres_true,
        "gpu_ms_per_step": round(1e3 * head["gpu"] / steps, 4),
        "roofline": roofline,
        "step_roofline": step_roofline,
        other: {"value": round(steps / results[other]["wall"], 2),
                "ms_per_step": round(1e3 * results[other]["wall"] / steps, 4),
                "iters": results[other]["info"].iters,
                "outer_iters": results[other]["info"].outer_iters,
                "relres_true": results[other]["info"].relres_true,
                "dominant_kernel": results[other]["prof"][0]["name"],
                "dominant_gbs": round(results[other]["prof"][0]["gbs"], 1),
                "err_vs_fp64_oracle": None},
        "kernels": [{k: (round(v, 3) if isinstance(v, float) else v)
                     for k, v in r.items() if k in ("name", "launches", "avg_us", "gbs", "multipass_gbs",
                                                    "ms_per_step")}
                    for r in head["prof"][:10]],
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle), ~%.0f s on all threads and ~%.0f s on one" % (args.cpu_seconds, args.cpu_seconds))
        base, errs = cpu_baseline(p, args.cpu_seconds, results["fp64"]["x"], results["fp32_ir"]["x"])
        out["cpu_baseline"] = base
        out["err_vs_fp64_oracle"] = errs[args.precision]
        out[other]["err_vs_fp64_oracle"] = errs[other]
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
