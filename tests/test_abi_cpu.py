"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/fnls.h, sizes workspaces, and rejects bad calls on the
host (no device is touched)."""
import ctypes

import pytest

from paper_2410_03643_amd import fnls


@pytest.fixture(scope="module")
def L():
    return fnls.lib()


def test_exports_every_declared_symbol(L):
    names = fnls.declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


def test_library_carries_the_host_trace_ranges(L):
    """The solve-level calls open roctx ranges: the library needs the ROCm
    profiler SDK's roctx library and imports its push and pop."""
    import shutil
    import subprocess
    if not shutil.which("readelf"):
        pytest.skip("readelf not available")
    dyn = subprocess.run(["readelf", "-d", fnls.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert "librocprofiler-sdk-roctx.so" in dyn
    syms = subprocess.run(["readelf", "--dyn-syms", "-W", fnls.LIB_PATH], capture_output=True, text=True,
                          check=True).stdout
    undef = {ln.split()[-1].split("@")[0] for ln in syms.splitlines() if " UND " in ln}
    assert {"roctxRangePushA", "roctxRangePop"} <= undef


def test_default_opts(L):
    o = fnls.default_opts()
    assert o.tol == 1e-10 and o.restart == 30 and o.maxit == 2000
    assert o.precision == fnls.FP64 and o.fixed_iters == 0 and o.lookahead == 1
    assert o.inner_tol == 1e-5 and o.max_outer == 20


def test_struct_sizes_match_header():
    # double + 3 int + pad + double + 5 int (max_outer .. poll_delay_us) + int[2] -> 64 bytes; info 24 + 512
    assert ctypes.sizeof(fnls.Opts) == 64
    assert ctypes.sizeof(fnls.Info) == 24 + 64 * 8


@pytest.mark.parametrize("d,n", [(1, 1), (1, 1023), (2, 7), (2, 1023), (3, 255)])
def test_workspace_bytes_valid(L, d, n):
    b30 = fnls.workspace_bytes(d, n, 30)
    b1 = fnls.workspace_bytes(d, n, 1)
    N = n ** d
    assert b30 >= (30 + 6) * 16 * N
    assert b30 - b1 >= 29 * 16 * N - 256   # one basis vector per extra restart slot


@pytest.mark.parametrize("d,n,r", [(0, 7, 30), (4, 7, 30), (2, 0, 30), (2, 6, 30), (2, 1024, 30),
                                   (2, 2047, 30), (2, 7, 0), (2, 7, 65)])
def test_workspace_bytes_invalid(L, d, n, r):
    assert fnls.workspace_bytes(d, n, r) == 0


def test_status_strings(L):
    for code, word in [(0, "ok"), (1, "not converged"), (-1, "invalid"), (-3, "workspace"),
                       (-4, "non-finite"), (-6, "GPU")]:
        assert word in L.fnls_status_string(code).decode()


def test_null_context_is_rejected(L):
    assert L.fnls_assemble(None, 1.5, 2.0, 2, 7, 0.1, 0.01, None, 0) == fnls.ERR_INVALID_ARG
    assert L.fnls_precond_setup(None, None, None, 1.0) == fnls.ERR_INVALID_ARG
    assert L.fnls_apply_A(None, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_apply_precond(None, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_rhs(None, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_solve(None, None, None, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_step(None, None, None, None, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_first_step(None, None, None, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_create(None, 0, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_set_pass_config(None, 0, 0, 4, 1) == fnls.ERR_INVALID_ARG
    assert L.fnls_timing(None, 1) == fnls.ERR_INVALID_ARG
    assert L.fnls_timing_report(None, None, 0) == fnls.ERR_INVALID_ARG
    assert L.fnls_set_potential(None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_step_backward(None, None, None, None, None, None, None, None, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_first_step_backward(None, None, None, None, None, None, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_autotune(None, None, 0, 1, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_batch_create(None, None, 0, None, 0) == fnls.ERR_INVALID_ARG
    assert L.fnls_batch_solve(None, None, None, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_batch_step(None, None, None, None, None, None) == fnls.ERR_INVALID_ARG
    assert L.fnls_batch_last_error(None) == b"null batch"
    assert L.fnls_batch_autotune(None, None, 0, 1, None) == fnls.ERR_INVALID_ARG
    rm, li = ctypes.c_int(-1), ctypes.c_int(-1)
    assert L.fnls_batch_schedule(None, 1023, 0, 1, ctypes.byref(rm), ctypes.byref(li)) == fnls.ERR_INVALID_ARG
    assert L.fnls_batch_workspace_bytes(0) == 0 and L.fnls_batch_workspace_bytes(4097) == 0
    assert L.fnls_batch_workspace_bytes(64) >= 16 << 20
    # the workspace grows with the count (argument tables of the cached graphs)
    assert L.fnls_batch_workspace_bytes(4096) > L.fnls_batch_workspace_bytes(64)
    cap, rep = ctypes.c_longlong(-1), ctypes.c_longlong(-1)
    assert L.fnls_batch_graph_stats(None, ctypes.byref(cap), ctypes.byref(rep)) == fnls.ERR_INVALID_ARG
    assert cap.value == -1 and rep.value == -1
    L.fnls_batch_destroy(None)
    L.fnls_destroy(None)
    assert L.fnls_last_error(None) == b"null context"


def test_create_without_device_reports_no_device(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    assert L.fnls_create(ctypes.byref(ctx), 0, None) == fnls.ERR_NO_DEVICE
    assert not ctx.value


# ---------------------------------------------------------------------------
# fnls_assemble's argument checks, reached without a device through the
# context-free checker that fnls_assemble itself calls first
# ---------------------------------------------------------------------------
ALIGNED = 1 << 20          # a 256-byte aligned address (never dereferenced)


def check_assemble(L, alpha=1.5, rho=2.0, d=2, n=63, h=0.3, tau=0.01, ws=ALIGNED, nbytes=None):
    if nbytes is None:
        nbytes = fnls.workspace_bytes(d if 1 <= d <= 3 else 2, n if n in (1, 3, 7, 63) else 63, 1)
    msg = ctypes.create_string_buffer(256)
    rc = L.fnls_check_assemble(alpha, rho, d, n, h, tau, ctypes.c_void_p(ws) if ws else None, nbytes, msg, 256)
    return rc, msg.value.decode()


def test_check_assemble_accepts_valid_arguments(L):
    for d, n in ((1, 1), (1, 1023), (2, 63), (3, 7)):
        assert check_assemble(L, d=d, n=n, nbytes=fnls.workspace_bytes(d, n, 1)) == (fnls.OK, "")
    assert check_assemble(L, alpha=2.0, rho=0.0)[0] == fnls.OK      # alpha = 2 and the linear limit


@pytest.mark.parametrize("kw,code,word", [
    (dict(alpha=1.0), fnls.ERR_INVALID_ARG, "alpha"),
    (dict(alpha=2.0000001), fnls.ERR_INVALID_ARG, "alpha"),
    (dict(alpha=float("nan")), fnls.ERR_INVALID_ARG, "alpha"),
    (dict(rho=-1e-12), fnls.ERR_INVALID_ARG, "rho"),
    (dict(rho=float("inf")), fnls.ERR_INVALID_ARG, "rho"),
    (dict(rho=float("nan")), fnls.ERR_INVALID_ARG, "rho"),
    (dict(d=0), fnls.ERR_INVALID_ARG, "d must"),
    (dict(d=4), fnls.ERR_INVALID_ARG, "d must"),
    (dict(n=0), fnls.ERR_INVALID_ARG, "power of two"),
    (dict(n=62), fnls.ERR_INVALID_ARG, "power of two"),
    (dict(n=2047), fnls.ERR_INVALID_ARG, "power of two"),
    (dict(h=0.0), fnls.ERR_INVALID_ARG, "h must"),
    (dict(h=-0.1), fnls.ERR_INVALID_ARG, "h must"),
    (dict(h=float("inf")), fnls.ERR_INVALID_ARG, "h must"),
    (dict(tau=0.0), fnls.ERR_INVALID_ARG, "tau must"),
    (dict(tau=float("nan")), fnls.ERR_INVALID_ARG, "tau must"),
    (dict(ws=0), fnls.ERR_WORKSPACE, "NULL"),
    (dict(ws=ALIGNED + 128), fnls.ERR_WORKSPACE, "aligned"),
    (dict(nbytes=0), fnls.ERR_WORKSPACE, "too small"),
])
def test_check_assemble_rejections(L, kw, code, word):
    rc, msg = check_assemble(L, **kw)
    assert rc == code and word in msg, (rc, msg)


def test_check_assemble_workspace_boundary(L):
    need = fnls.workspace_bytes(2, 63, 1)
    assert check_assemble(L, nbytes=need)[0] == fnls.OK
    assert check_assemble(L, nbytes=need - 1)[0] == fnls.ERR_WORKSPACE
    # no message buffer: the status alone
    assert L.fnls_check_assemble(1.5, 2.0, 2, 63, 0.3, 0.01, None, need, None, 0) == fnls.ERR_WORKSPACE


def test_host_stats_null_context(L):
    assert L.fnls_get_host_stats(None, None, 0) == fnls.ERR_INVALID_ARG


# ---------------------------------------------------------------------------
# host status protocol: the library's own acceptance rule for a report
# ---------------------------------------------------------------------------
SEQ_STRIDE = 1 << 24    # window of one solve's status sequence


def accepted(L, base, s1, s2=None, total=5, done=0, target=5):
    s2 = s1 if s2 is None else s2
    return L.fnls_status_report_accepted(base & 0xFFFFFFFF, s1 & 0xFFFFFFFF, s2 & 0xFFFFFFFF, total, done,
                                         target) == 1


@pytest.mark.parametrize("solve", [1, 2, 255, 256, 257, 1000])
def test_status_sequence_window(L, solve):
    """Each solve advances the base by 2^24 (mod 2^32); a report adds 2 and is
    odd while being written.  The host takes only complete reports of the
    current solve: not the configuration value itself, not a half-written
    report, not any report of the previous solve (also across the wrap of the
    32-bit counter), and every report up to 2 (2^21 + 64) of this solve (the
    maxit bound keeps a solve's reports inside the window)."""
    base = solve * SEQ_STRIDE
    prev = (solve - 1) * SEQ_STRIDE
    assert not accepted(L, base, base)
    max_reports = (1 << 21) + 64
    for k in (1, 2, 3, 1000, max_reports):
        assert accepted(L, base, base + 2 * k)
        assert not accepted(L, base, base + 2 * k - 1)
        assert not accepted(L, base, prev + 2 * k)
    assert not accepted(L, base, base + SEQ_STRIDE)
    assert 2 * max_reports < SEQ_STRIDE


def test_status_report_needs_a_stable_copy_and_the_awaited_total(L):
    base = 7 * SEQ_STRIDE
    s = base + 10
    assert accepted(L, base, s, s, total=5, target=5)
    assert accepted(L, base, s, s, total=9, target=5)          # a later report covers it
    assert not accepted(L, base, s, s + 2, total=5, target=5)  # a report landed during the copy
    assert not accepted(L, base, s, s + 1, total=5, target=5)
    assert not accepted(L, base, s, s, total=4, target=5)      # not there yet
    assert accepted(L, base, s, s, total=0, done=1, target=5)  # the solve ended (b = 0, stop)
