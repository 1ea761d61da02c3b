"""Python binding of libfnls (the C ABI in include/fnls.h), via ctypes.

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory (the workspace is a torch uint8 tensor) and the
stream (the current torch stream of the device at construction time).  The
library must have been built (``python -m paper_2410_03643_amd.build``);
nothing here falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfnls.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fnls.h")

OK = 0
NOT_CONVERGED = 1
ERR_INVALID_ARG = -1
ERR_STATE = -2
ERR_WORKSPACE = -3
ERR_NONFINITE = -4
ERR_HIP = -5
ERR_NO_DEVICE = -6
FP64 = 0
FP32_IR = 1


class FnlsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("fnls error %d: %s" % (code, msg))
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
                ("precision", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("fixed_iters", ctypes.c_int),
                ("lookahead", ctypes.c_int), ("graph", ctypes.c_int), ("poll_delay_us", ctypes.c_int),
                ("reserved", ctypes.c_int * 2)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("status", ctypes.c_int),
                ("breakdown", ctypes.c_int), ("relres_true", ctypes.c_double),
                ("relres_hist", ctypes.c_double * 64)]


class HostStats(ctypes.Structure):
    _fields_ = [("solves", ctypes.c_longlong), ("cycles", ctypes.c_longlong),
                ("iterations", ctypes.c_longlong), ("stop_predictions", ctypes.c_longlong),
                ("ends_ahead", ctypes.c_longlong), ("late_reads", ctypes.c_longlong),
                ("cycles_ahead", ctypes.c_longlong), ("early_stops", ctypes.c_longlong)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("launches", ctypes.c_int),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double), ("bytes_min", ctypes.c_double)]


@dataclass
class SolveInfo:
    iters: int
    outer_iters: int
    status: int
    breakdown: int
    relres_true: float
    relres_hist: list = field(default_factory=list)


_lib = None


def lib() -> ctypes.CDLL:
    """Load libfnls.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfnls.so is not built: run python -m paper_2410_03643_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, ci, cd, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    L.fnls_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.fnls_default_opts.restype = None
    L.fnls_create.argtypes = [ctypes.POINTER(vp), ci, vp]
    L.fnls_create.restype = ci
    L.fnls_destroy.argtypes = [vp]
    L.fnls_destroy.restype = None
    L.fnls_workspace_bytes.argtypes = [ci, ci, ci]
    L.fnls_workspace_bytes.restype = sz
    L.fnls_assemble.argtypes = [vp, cd, cd, ci, ci, cd, cd, vp, sz]
    L.fnls_assemble.restype = ci
    L.fnls_precond_setup.argtypes = [vp, vp, vp, cd]
    L.fnls_precond_setup.restype = ci
    L.fnls_check_assemble.argtypes = [cd, cd, ci, ci, cd, cd, vp, sz, ctypes.c_char_p, sz]
    L.fnls_check_assemble.restype = ci
    L.fnls_get_host_stats.argtypes = [vp, ctypes.POINTER(HostStats), ci]
    L.fnls_get_host_stats.restype = ci
    L.fnls_status_report_accepted.argtypes = [ctypes.c_uint, ctypes.c_uint, ctypes.c_uint, ci, ci, ci]
    L.fnls_status_report_accepted.restype = ci
    L.fnls_pass_geometry.argtypes = [ci, ci, ci, ci, ci, ci, sz, ctypes.POINTER(ctypes.c_longlong)]
    L.fnls_pass_geometry.restype = ci
    for name in ("fnls_apply_A", "fnls_apply_precond", "fnls_rhs", "fnls_apply_A_c64", "fnls_apply_precond_c64"):
        getattr(L, name).argtypes = [vp, vp, vp]
        getattr(L, name).restype = ci
    L.fnls_solve.argtypes = [vp, vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    L.fnls_solve.restype = ci
    L.fnls_solve_noalloc.argtypes = [vp, vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    L.fnls_solve_noalloc.restype = ci
    L.fnls_step.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    L.fnls_step.restype = ci
    L.fnls_first_step.argtypes = [vp, vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    L.fnls_first_step.restype = ci
    L.fnls_last_error.argtypes = [vp]
    L.fnls_last_error.restype = ctypes.c_char_p
    L.fnls_status_string.argtypes = [ci]
    L.fnls_status_string.restype = ctypes.c_char_p
    L.fnls_set_pass_config.argtypes = [vp, ci, ci, ci, ci]
    L.fnls_set_pass_config.restype = ci
    L.fnls_timing.argtypes = [vp, ci]
    L.fnls_timing.restype = ci
    L.fnls_timing_report.argtypes = [vp, ctypes.POINTER(KernelStat), ci]
    L.fnls_timing_report.restype = ci
    L.fnls_set_potential.argtypes = [vp, vp]
    L.fnls_set_potential.restype = ci
    L.fnls_step_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    L.fnls_step_backward.restype = ci
    L.fnls_first_step_backward.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    L.fnls_first_step_backward.restype = ci
    L.fnls_autotune.argtypes = [vp, vp, ci, ci, ctypes.POINTER(ci), ctypes.POINTER(cd)]
    L.fnls_autotune.restype = ci
    L.fnls_batch_workspace_bytes.argtypes = [ci]
    L.fnls_batch_workspace_bytes.restype = sz
    L.fnls_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ci, vp, sz]
    L.fnls_batch_create.restype = ci
    L.fnls_batch_destroy.argtypes = [vp]
    L.fnls_batch_destroy.restype = None
    L.fnls_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(Opts),
                                   ctypes.POINTER(Info)]
    L.fnls_batch_solve.restype = ci
    L.fnls_batch_step.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    L.fnls_batch_step.restype = ci
    L.fnls_batch_autotune.argtypes = [vp, ctypes.POINTER(vp), ci, ci, ctypes.POINTER(ci)]
    L.fnls_batch_autotune.restype = ci
    L.fnls_batch_schedule.argtypes = [vp, ci, ci, ci, ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.fnls_batch_schedule.restype = ci
    L.fnls_batch_last_error.argtypes = [vp]
    L.fnls_batch_last_error.restype = ctypes.c_char_p
    L.fnls_batch_graph_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
    L.fnls_batch_graph_stats.restype = ci
    _lib = L
    return L


def declared_symbols() -> list[str]:
    """Function names declared in include/fnls.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)   # drop comments
    return sorted(set(re.findall(r"\b(fnls_[a-zA-Z0-9_]+)\s*\(", txt)))


def workspace_bytes(d: int, n: int, restart: int = 30) -> int:
    return int(lib().fnls_workspace_bytes(d, n, restart))


def default_opts() -> Opts:
    o = Opts()
    lib().fnls_default_opts(ctypes.byref(o))
    return o


class Solver:
    """One assembled operator (alpha, rho, d, n, h, tau) on one GPU.

    Vectors are torch.complex128 tensors of shape (n,)*d on the solver's
    device (C order, last axis = x_1)."""

    def __init__(self, alpha: float, rho: float, d: int, n: int, h: float, tau: float,
                 device=None, restart: int = 30):
        import torch
        self.torch = torch
        if device is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.alpha, self.rho, self.d, self.n, self.h, self.tau = alpha, rho, d, n, h, tau
        self.shape = (n,) * d
        L = lib()
        self._ctx = ctypes.c_void_p()
        rc = L.fnls_create(ctypes.byref(self._ctx), self.device.index or 0,
                           ctypes.c_void_p(self.stream.cuda_stream))
        if rc != OK:
            raise FnlsError(rc, L.fnls_status_string(rc).decode())
        nbytes = L.fnls_workspace_bytes(d, n, restart)
        if nbytes == 0:
            L.fnls_destroy(self._ctx)
            self._ctx = None
            raise FnlsError(ERR_INVALID_ARG, "unsupported size d=%d n=%d restart=%d" % (d, n, restart))
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._check(L.fnls_assemble(self._ctx, alpha, rho, d, n, h, tau,
                                    ctypes.c_void_p(self._ws_ptr), nbytes))

    # -- helpers -----------------------------------------------------------
    def _check(self, rc: int) -> int:
        if rc < 0:
            raise FnlsError(rc, lib().fnls_last_error(self._ctx).decode())
        return rc

    def _vec(self, t, name):
        torch = self.torch
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.dtype != torch.complex128 or tuple(t.shape) != self.shape or not t.is_contiguous() \
                or t.device != self.device:
            raise ValueError("%s must be a contiguous complex128 tensor of shape %s on %s"
                             % (name, self.shape, self.device))
        return ctypes.c_void_p(t.data_ptr())

    def _out(self):
        return self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)

    @staticmethod
    def _opts(tol, restart, maxit, precision, inner_tol, max_outer, fixed_iters, lookahead, poll_delay_us=0):
        o = default_opts()
        o.tol = tol
        o.restart = restart
        o.maxit = maxit
        o.precision = {"fp64": FP64, "fp32_ir": FP32_IR}[precision] if isinstance(precision, str) \
            else int(precision)
        o.inner_tol = inner_tol
        o.max_outer = max_outer
        o.fixed_iters = fixed_iters
        o.lookahead = lookahead
        o.poll_delay_us = poll_delay_us
        return o

    @staticmethod
    def _info(i: Info) -> SolveInfo:
        return SolveInfo(i.iters, i.outer_iters, i.status, i.breakdown, i.relres_true,
                         [i.relres_hist[k] for k in range(min(64, i.iters))])

    # -- C ABI calls -------------------------------------------------------
    def precond_setup(self, u_cur, V=None, omega: float = 1.0):
        vp = None
        if V is not None:
            if V.dtype != self.torch.float64 or tuple(V.shape) != self.shape or not V.is_contiguous():
                raise ValueError("V must be a contiguous float64 tensor of shape %s" % (self.shape,))
            vp = ctypes.c_void_p(V.data_ptr())
        self._check(lib().fnls_precond_setup(self._ctx, self._vec(u_cur, "u_cur"), vp, omega))

    def apply_A(self, x, out=None):
        y = self._out() if out is None else out
        self._check(lib().fnls_apply_A(self._ctx, self._vec(x, "x"), self._vec(y, "y")))
        return y

    def apply_precond(self, r, out=None):
        z = self._out() if out is None else out
        self._check(lib().fnls_apply_precond(self._ctx, self._vec(r, "r"), self._vec(z, "z")))
        return z

    def _vec64(self, t, name):
        torch = self.torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex64 or tuple(t.shape) != self.shape \
                or not t.is_contiguous() or t.device != self.device:
            raise ValueError("%s must be a contiguous complex64 tensor of shape %s on %s"
                             % (name, self.shape, self.device))
        return ctypes.c_void_p(t.data_ptr())

    def apply_A_c64(self, x, out=None):
        """y = A x on complex64 vectors (the GMRES-IR inner kernels)."""
        y = self.torch.empty(self.shape, dtype=self.torch.complex64, device=self.device) if out is None else out
        self._check(lib().fnls_apply_A_c64(self._ctx, self._vec64(x, "x"), self._vec64(y, "y")))
        return y

    def apply_precond_c64(self, r, out=None):
        """z = Ptilde^{-1} r on complex64 vectors (the GMRES-IR inner kernels)."""
        z = self.torch.empty(self.shape, dtype=self.torch.complex64, device=self.device) if out is None else out
        self._check(lib().fnls_apply_precond_c64(self._ctx, self._vec64(r, "r"), self._vec64(z, "z")))
        return z

    def host_stats(self, reset: bool = False) -> dict:
        """Counters of the host's GMRES sequencing (fnls_get_host_stats)."""
        st = HostStats()
        self._check(lib().fnls_get_host_stats(self._ctx, ctypes.byref(st), 1 if reset else 0))
        return {name: getattr(st, name) for name, _ in HostStats._fields_}

    def rhs(self, u_prev, out=None):
        b = self._out() if out is None else out
        self._check(lib().fnls_rhs(self._ctx, self._vec(u_prev, "u_prev"), self._vec(b, "b")))
        return b

    def solve(self, b, out=None, *, tol=1e-10, restart=30, maxit=2000, precision="fp64",
              inner_tol=1e-5, max_outer=20, fixed_iters=0, lookahead=1, poll_delay_us=0):
        x = self._out() if out is None else out
        o = self._opts(tol, restart, maxit, precision, inner_tol, max_outer, fixed_iters, lookahead,
                       poll_delay_us)
        info = Info()
        self._check(lib().fnls_solve(self._ctx, self._vec(b, "b"), self._vec(x, "x"),
                                     ctypes.byref(o), ctypes.byref(info)))
        return x, self._info(info)

    def solve_noalloc(self, b, out, *, tol=1e-10, restart=30, maxit=2000, precision="fp64",
                      inner_tol=1e-5, max_outer=20, fixed_iters=0, lookahead=1):
        """fnls_solve_noalloc: the solve with the library's static scratch
        (the output tensor is the caller's)."""
        o = self._opts(tol, restart, maxit, precision, inner_tol, max_outer, fixed_iters, lookahead)
        info = Info()
        self._check(lib().fnls_solve_noalloc(self._ctx, self._vec(b, "b"), self._vec(out, "x"),
                                             ctypes.byref(o), ctypes.byref(info)))
        return out, self._info(info)

    def step(self, u_prev, u_cur, out=None, *, tol=1e-10, restart=30, maxit=2000,
             precision="fp64", inner_tol=1e-5, max_outer=20, lookahead=1):
        un = self._out() if out is None else out
        o = self._opts(tol, restart, maxit, precision, inner_tol, max_outer, 0, lookahead)
        info = Info()
        self._check(lib().fnls_step(self._ctx, self._vec(u_prev, "u_prev"), self._vec(u_cur, "u_cur"),
                                    self._vec(un, "u_next"), ctypes.byref(o), ctypes.byref(info)))
        return un, self._info(info)

    def first_step(self, u0, out=None, *, tol=1e-10, restart=30, maxit=2000,
                   precision="fp64", inner_tol=1e-5, max_outer=20, lookahead=1):
        u1 = self._out() if out is None else out
        o = self._opts(tol, restart, maxit, precision, inner_tol, max_outer, 0, lookahead)
        info = Info()
        self._check(lib().fnls_first_step(self._ctx, self._vec(u0, "u0"), self._vec(u1, "u1"),
                                          ctypes.byref(o), ctypes.byref(info)))
        return u1, self._info(info)

    def _real(self, V, name):
        if V is None:
            return None
        if not isinstance(V, self.torch.Tensor) or V.dtype != self.torch.float64 \
                or tuple(V.shape) != self.shape or not V.is_contiguous() or V.device != self.device:
            raise ValueError("%s must be a contiguous float64 tensor of shape %s on %s"
                             % (name, self.shape, self.device))
        return ctypes.c_void_p(V.data_ptr())

    def set_potential(self, V):
        """Real potential added to D by step / first_step and their reverse
        modes (None removes it).  The tensor must stay alive while in use."""
        self._potential = V          # keep the storage alive
        self._check(lib().fnls_set_potential(self._ctx, self._real(V, "V")))

    def step_backward(self, u_prev, u_cur, u_next, g_next, g_prev, g_cur, g_V=None, *, tol=1e-10,
                      restart=30, maxit=2000, lookahead=1):
        """Accumulate the reverse mode of step(u_prev, u_cur) -> u_next into
        g_prev, g_cur (complex) and g_V (real, optional)."""
        o = self._opts(tol, restart, maxit, "fp64", 1e-5, 20, 0, lookahead)
        info = Info()
        self._check(lib().fnls_step_backward(
            self._ctx, self._vec(u_prev, "u_prev"), self._vec(u_cur, "u_cur"), self._vec(u_next, "u_next"),
            self._vec(g_next, "g_next"), self._vec(g_prev, "g_prev"), self._vec(g_cur, "g_cur"),
            self._real(g_V, "g_V"), ctypes.byref(o), ctypes.byref(info)))
        return self._info(info)

    def first_step_backward(self, u0, u1, g1, g0, g_V=None, *, tol=1e-10, restart=30, maxit=2000,
                            lookahead=1):
        """Accumulate the reverse mode of first_step(u0) -> u1 into g0 and g_V."""
        o = self._opts(tol, restart, maxit, "fp64", 1e-5, 20, 0, lookahead)
        info = Info()
        self._check(lib().fnls_first_step_backward(
            self._ctx, self._vec(u0, "u0"), self._vec(u1, "u1"), self._vec(g1, "g1"), self._vec(g0, "g0"),
            self._real(g_V, "g_V"), ctypes.byref(o), ctypes.byref(info)))
        return self._info(info)

    def autotune(self, b, precision="fp64", reps: int = 5):
        """Time solves of b over the transform-pass schedules and keep the
        fastest; returns ({axis kind: (rmax, lines)}, ms per solve)."""
        p = {"fp64": FP64, "fp32_ir": FP32_IR}[precision] if isinstance(precision, str) else precision
        best = (ctypes.c_int * 4)()
        ms = ctypes.c_double()
        self._check(lib().fnls_autotune(self._ctx, self._vec(b, "b"), p, reps, best, ctypes.byref(ms)))
        return {"contiguous": (best[0], best[1]), "strided": (best[2], best[3])}, ms.value

    def set_pass_config(self, precision, strided: bool, rmax: int, lines: int):
        """Transform-pass tuning: largest radix and lines per workgroup."""
        p = {"fp64": FP64, "fp32_ir": FP32_IR}[precision] if isinstance(precision, str) else precision
        self._check(lib().fnls_set_pass_config(self._ctx, p, 1 if strided else 0, rmax, lines))

    def timing(self, enable: bool):
        """Start (clearing earlier records) or stop per-launch event timing."""
        self._check(lib().fnls_timing(self._ctx, 1 if enable else 0))

    def timing_report(self):
        """Per kernel class: launches, summed event milliseconds, algorithmic bytes."""
        arr = (KernelStat * 256)()
        k = self._check(lib().fnls_timing_report(self._ctx, arr, 256))
        return [dict(name=arr[i].name.decode(), launches=arr[i].launches,
                     total_ms=arr[i].total_ms, bytes=arr[i].bytes, bytes_min=arr[i].bytes_min)
                for i in range(k)]

    def close(self):
        if getattr(self, "_ctx", None):
            lib().fnls_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many Solver instances (uneven sizes, same d, device and stream)
    advanced together: one kernel launch per pass / update / decision for all
    of them.  The solvers must outlive the batch."""

    def __init__(self, solvers):
        import torch
        self.torch = torch
        self.solvers = list(solvers)
        if not self.solvers:
            raise ValueError("empty batch")
        L = lib()
        n = len(self.solvers)
        ctxs = (ctypes.c_void_p * n)(*[s._ctx for s in self.solvers])
        nbytes = L.fnls_batch_workspace_bytes(n)
        if nbytes == 0:
            raise FnlsError(ERR_INVALID_ARG, "unsupported batch size %d" % n)
        dev = self.solvers[0].device
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        ptr = (self._ws.data_ptr() + 255) // 256 * 256
        self._b = ctypes.c_void_p()
        rc = L.fnls_batch_create(ctypes.byref(self._b), ctxs, n, ctypes.c_void_p(ptr), nbytes)
        if rc != OK:
            raise FnlsError(rc, L.fnls_status_string(rc).decode())

    def _check(self, rc):
        if rc < 0:
            raise FnlsError(rc, lib().fnls_batch_last_error(self._b).decode())
        return rc

    def _ptrs(self, ts, name):
        n = len(self.solvers)
        if len(ts) != n:
            raise ValueError("%s: expected %d tensors" % (name, n))
        return (ctypes.c_void_p * n)(*[s._vec(t, name) for s, t in zip(self.solvers, ts)])

    def autotune(self, bs, precision="fp64", reps: int = 3) -> int:
        """fnls_batch_autotune: time batched solves of bs over the schedules of
        each line-length class; returns the number of classes tuned."""
        p = {"fp64": FP64, "fp32_ir": FP32_IR}[precision] if isinstance(precision, str) else precision
        n = ctypes.c_int()
        self._check(lib().fnls_batch_autotune(self._b, self._ptrs(bs, "b"), p, reps, ctypes.byref(n)))
        return n.value

    def schedule(self, n: int, precision="fp64", strided: bool = True):
        """(rmax, lines) the batch's autotuner chose for line length n + 1, or
        (0, 0) for the default shape."""
        p = {"fp64": FP64, "fp32_ir": FP32_IR}[precision] if isinstance(precision, str) else precision
        rm, li = ctypes.c_int(), ctypes.c_int()
        self._check(lib().fnls_batch_schedule(self._b, n, p, 1 if strided else 0, ctypes.byref(rm), ctypes.byref(li)))
        return rm.value, li.value

    def solve(self, bs, outs=None, *, tol=1e-10, restart=30, maxit=2000, precision="fp64", inner_tol=1e-5,
              max_outer=20, lookahead=1, graph=False):
        xs = [s._out() for s in self.solvers] if outs is None else outs
        o = Solver._opts(tol, restart, maxit, precision, inner_tol, max_outer, 0, lookahead)
        o.graph = 1 if graph else 0
        infos = (Info * len(self.solvers))()
        self._check(lib().fnls_batch_solve(self._b, self._ptrs(bs, "b"), self._ptrs(xs, "x"), ctypes.byref(o),
                                           infos))
        return xs, [Solver._info(i) for i in infos]

    def step(self, u_prev, u_cur, outs=None, *, tol=1e-10, restart=30, maxit=2000, precision="fp64",
             inner_tol=1e-5, max_outer=20, lookahead=1, graph=False):
        un = [s._out() for s in self.solvers] if outs is None else outs
        o = Solver._opts(tol, restart, maxit, precision, inner_tol, max_outer, 0, lookahead)
        o.graph = 1 if graph else 0
        infos = (Info * len(self.solvers))()
        self._check(lib().fnls_batch_step(self._b, self._ptrs(u_prev, "u_prev"), self._ptrs(u_cur, "u_cur"),
                                          self._ptrs(un, "u_next"), ctypes.byref(o), infos))
        return un, [Solver._info(i) for i in infos]

    def graph_stats(self):
        """(graphs captured, graph launches) since the batch was created."""
        cap, rep = ctypes.c_longlong(), ctypes.c_longlong()
        self._check(lib().fnls_batch_graph_stats(self._b, ctypes.byref(cap), ctypes.byref(rep)))
        return cap.value, rep.value

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            lib().fnls_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
