/*
 * fnls.h -- C ABI of libfnls: tau-preconditioned GMRES for the linear systems
 * of the Riesz fractional nonlinear Schroedinger time stepper, on one AMD
 * MI355X (gfx950).
 *
 * Problem (Sec. 2 of arXiv 2410.03643, "the discrete linear systems"):
 * at every time level solve
 *
 *     (D - T_d + i I) u = b,
 *
 * where T_d = sum over the d axes of T_1 = mu T_0 applied along that axis
 * (Kronecker sum, Sec. 2.2), T_0 the symmetric Toeplitz matrix of the
 * fractional centred-difference coefficients c_k (Sec. 2.1),
 * mu = dt / h^alpha, and D = rho dt |u^n|^2 (+ dt V) the real diagonal.
 *
 * Method: GMRES, right-preconditioned by the sine-transform TBAN
 * preconditioner of Sec. 4 (its parameter omega, 1 by default) written in
 * complex form,
 *
 *     z = -2 i omega ((omega+1) - i D)^{-1} . S_d (omega + i Lambda_d)^{-1} . S_d r,
 *
 * where S_d is the d-fold orthonormal sine transform (DST-I) and Lambda_d the
 * Kronecker sum of the eigenvalues of the tau matrix tau(T_1) (Sec. 4).
 * Zero initial guess, relative-residual stopping test (Sec. 5 protocol).
 *
 * Conventions (all entry points)
 * ------------------------------
 * - Grid: n interior points per axis, n + 1 a power of two, 1 <= n <= 1023,
 *   d in {1, 2, 3}; h = (b - a)/(n + 1) is the spacing (Sec. 2.1).
 * - Vectors: device pointers to N = n^d complex values, C order over
 *   (n,)*d with the LAST axis the fastest (x_1), i.e. the column-stacking
 *   vec() of Sec. 2.2.  fnls_c128 is layout-compatible with torch.complex128
 *   and with double[2].  All vectors are owned by the caller and must stay
 *   valid until the context's stream has executed the call.  Input vectors
 *   must not alias output vectors unless stated otherwise.
 * - Workspace: one caller-owned device block of at least
 *   fnls_workspace_bytes(d, n, restart) bytes, passed to fnls_assemble; the
 *   library keeps its tables, the diagonal, the Krylov basis and all
 *   temporaries there.  The library allocates no device memory; it owns the
 *   context struct and a small pinned host buffer for status words.
 * - Streams: every call enqueues its kernels on the context's HIP stream.
 *   fnls_solve / fnls_step / fnls_first_step return when the result is
 *   complete (they wait on that stream to make convergence decisions);
 *   fnls_rhs / fnls_apply_A / fnls_apply_precond / fnls_precond_setup return
 *   immediately (stream-ordered).
 * - Errors: functions return an fnls_status.  Argument errors are detected on
 *   the host before any GPU work and leave the context unchanged.  No C++
 *   exception crosses the ABI.  fnls_last_error() gives a message.
 * - Threading: a context is not thread-safe; use one context per stream.
 */
#ifndef FNLS_H
#define FNLS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fnls_ctx fnls_ctx;

/* One complex double: re, im (torch.complex128 element). */
typedef struct { double re, im; } fnls_c128;

/* One complex float: re, im (torch.complex64 element). */
typedef struct { float re, im; } fnls_c64;

typedef enum {
    FNLS_OK = 0,
    FNLS_NOT_CONVERGED = 1,     /* result written; info says how far it got    */
    FNLS_ERR_INVALID_ARG = -1,  /* bad size / parameter / NULL pointer          */
    FNLS_ERR_STATE = -2,        /* call order (e.g. solve before precond_setup) */
    FNLS_ERR_WORKSPACE = -3,    /* workspace missing or too small               */
    FNLS_ERR_NONFINITE = -4,    /* NaN / Inf in b (detected by the first norm)  */
    FNLS_ERR_HIP = -5,          /* a HIP runtime call failed                    */
    FNLS_ERR_NO_DEVICE = -6     /* no usable GPU                                */
} fnls_status;

typedef enum {
    FNLS_FP64 = 0,     /* everything in FP64 / complex128                                */
    FNLS_FP32_IR = 1   /* GMRES-IR: FP32 (complex64) transforms, matvec and basis inside
                          an FP64 refinement loop; dots, Hessenberg, x, b and the outer
                          residual in FP64                                               */
} fnls_precision;

/* Solver options.  Fill with fnls_default_opts() and override fields. */
typedef struct {
    double tol;        /* relative residual ||b - A x|| / ||b|| to reach (default 1e-10) */
    int restart;       /* GMRES restart length m (default 30; <= workspace capacity)     */
    int maxit;         /* total GMRES iterations allowed (default 2000, Sec. 5; <= 2^21)  */
    int precision;     /* fnls_precision (default FNLS_FP64)                             */
    double inner_tol;  /* FNLS_FP32_IR: inner relative tolerance of the first refinement
                          step (default 1e-5); later steps stop at
                          max(inner_tol, tol / (2 relres)), relres the current outer
                          relative residual                                              */
    int max_outer;     /* FNLS_FP32_IR: maximum refinement steps (default 20)            */
    int fixed_iters;   /* > 0: run exactly this many iterations, no tolerance test (FP64) */
    int lookahead;     /* iterations enqueued ahead of the host's convergence check
                          (0 = synchronise every iteration; default 1)                   */
    int graph;         /* batches (fnls_batch_solve / fnls_batch_step): 1 = enqueue every
                          Arnoldi iteration of all instances as one replay of a captured
                          hipGraph (see fnls_batch_create); 0 = direct launches (default).
                          Single-instance calls ignore it                                */
    int poll_delay_us; /* testing aid (default 0): the host sleeps this many microseconds
                          (at most 1e6) before each wait for an iteration's status, so
                          that work enqueued ahead has run by the time it reads; results
                          are the same with any value                                  */
    int reserved[2];
} fnls_opts;

/* Result of a solve.  relres_hist[k] is the GMRES estimate |g_{k+1}|/||b||
 * after total iteration k (FP64 path; inner estimates for FP32_IR), for
 * k < min(iters, 64). */
typedef struct {
    int iters;          /* total (inner) GMRES iterations                       */
    int outer_iters;    /* refinement steps (FP32_IR) or GMRES cycles (FP64)    */
    int status;         /* fnls_status of the solve                             */
    int breakdown;      /* 1 if an Arnoldi happy breakdown ended a cycle        */
    double relres_true; /* ||b - A x|| / ||b|| recomputed in FP64 at the end    */
    double relres_hist[64];
} fnls_info;

/* Default options (see field comments). */
void fnls_default_opts(fnls_opts *opts);

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Returns FNLS_ERR_NO_DEVICE if the
 * device does not exist.  *out is NULL on failure. */
int fnls_create(fnls_ctx **out, int device, void *hip_stream);

/* Release the context (not the caller's workspace).  Waits for its stream. */
void fnls_destroy(fnls_ctx *ctx);

/* Bytes of device workspace needed for d, n and a Krylov restart length
 * `restart` (both precisions fit the same block).  0 for invalid sizes. */
size_t fnls_workspace_bytes(int d, int n, int restart);

/* Host-only check of fnls_assemble's arguments (Sec. 2.1: alpha in (1, 2],
 * rho >= 0, h > 0, tau > 0; d in {1, 2, 3}; n + 1 a power of two, n <= 1023;
 * a 256-byte aligned workspace of at least fnls_workspace_bytes(d, n, 1)
 * bytes).  Touches no device and no context and never dereferences
 * `workspace`.  Returns the status fnls_assemble gives for these arguments
 * before any GPU work: FNLS_OK, FNLS_ERR_INVALID_ARG or FNLS_ERR_WORKSPACE.
 * msg (may be NULL) receives the reason, at most msg_len bytes including the
 * terminating NUL ("" when FNLS_OK).  fnls_assemble calls it first. */
int fnls_check_assemble(double alpha, double rho, int d, int n, double h, double tau,
                        const void *workspace, size_t workspace_bytes, char *msg, size_t msg_len);

/* a1 -- Assemble the operator for one parameter set (Sec. 2.1, 2.2, 4):
 * fractional centred-difference coefficients c_k of order alpha in (1, 2],
 * mu = tau / h^alpha, the circulant-embedding symbol of T_1 and the
 * eigenvalues lambda_k of tau(T_1) (both on the host in extended precision,
 * then copied into the workspace).  rho >= 0 scales |u|^2 in D, tau > 0 is
 * the time step, h > 0 the grid spacing.  `workspace` is a device pointer
 * owned by the caller, 256-byte aligned, of `workspace_bytes` bytes; its
 * size fixes the largest usable restart length.  Invalidates any previous
 * precond_setup. */
int fnls_assemble(fnls_ctx *ctx, double alpha, double rho, int d, int n, double h, double tau,
                  void *workspace, size_t workspace_bytes);

/* a2 -- Preconditioner setup for the current time level (Sec. 2.1, 2.2):
 * D_j = rho tau |u_cur_j|^2 (+ tau V_j if V != NULL, V real, N doubles on
 * the device), and the preconditioner parameter omega > 0 (Sec. 3-4; 1 is
 * the paper's choice). */
int fnls_precond_setup(fnls_ctx *ctx, const fnls_c128 *u_cur, const double *V, double omega);

/* a3 -- y = A x = (D - T_d + i I) x.  x and y must not alias. */
int fnls_apply_A(fnls_ctx *ctx, const fnls_c128 *x, fnls_c128 *y);

/* a4 -- z = Ptilde^{-1} r, the complex form of the sine-transform TBAN
 * preconditioner (formula in the header comment).  r and z must not alias. */
int fnls_apply_precond(fnls_ctx *ctx, const fnls_c128 *r, fnls_c128 *z);

/* a3, a4 in the precision of the GMRES-IR inner solve: the same operators as
 * fnls_apply_A and fnls_apply_precond on complex64 vectors (torch.complex64,
 * same layout), computed by the complex64 transform kernels of the inner
 * iteration with the FP32 copies of the tables and of D.  They let a caller
 * (and the test-suite) check those kernels against an FP64 reference; their
 * error is a few FP32 roundings per transform stage.  Same errors as the
 * FP64 entry points; inputs and outputs must not alias. */
int fnls_apply_A_c64(fnls_ctx *ctx, const fnls_c64 *x, fnls_c64 *y);
int fnls_apply_precond_c64(fnls_ctx *ctx, const fnls_c64 *r, fnls_c64 *z);

/* Right-hand side of the three-level scheme (Sec. 2.1, 2.2 multiplied by
 * 2 dt): b = (i I + T_d - D) u_prev, with D from the last precond_setup. */
int fnls_rhs(fnls_ctx *ctx, const fnls_c128 *u_prev, fnls_c128 *b);

/* a5-a8 -- Solve A x = b (x0 = 0) by right-preconditioned GMRES(m) with
 * classical Gram-Schmidt applied twice and complex Givens rotations, FP64 or
 * FP32 GMRES-IR per opts->precision.  Stops when the recomputed relative
 * residual is below opts->tol (FNLS_OK) or after opts->maxit iterations
 * (FNLS_NOT_CONVERGED, best x written).  b == 0 gives x = 0.  `opts` may be
 * NULL (defaults); `info` may be NULL.  b and x must not alias. */
int fnls_solve(fnls_ctx *ctx, const fnls_c128 *b, fnls_c128 *x, const fnls_opts *opts,
               fnls_info *info);

/* For callers that cannot allocate device memory at the call (code that may
 * not call hipMalloc: tight serving loops, harnesses that forbid it): the
 * same solve as fnls_solve (same kernels, results bitwise equal), with the
 * solver scratch -- GMRES state, partial sums, work vectors and both Krylov
 * bases, about (2 restart + 5) 16 n^d bytes -- in a static array of the
 * library, 64 MiB per device, held by every GPU the library runs on until the
 * process ends, instead of in the context's workspace.  The context still
 * needs fnls_assemble and fnls_precond_setup (its workspace keeps the
 * operator tables and D).  Allocates nothing: no hipMalloc, hipFree or
 * allocating library call.  FNLS_ERR_WORKSPACE when the scratch for d, n and
 * opts->restart exceeds 64 MiB (restart 30 fits up to n^d of about 64,000,
 * e.g. d = 2, n = 127; a shorter restart fits more).  All calls on one device
 * share the array, which keeps the last call's contents: calls that overlap
 * in time on one device (other host threads, other streams) race and must
 * not be made.  Same arguments, errors and results as fnls_solve. */
int fnls_solve_noalloc(fnls_ctx *ctx, const fnls_c128 *b, fnls_c128 *x, const fnls_opts *opts,
                       fnls_info *info);

/* a9 -- One three-level time step (Sec. 2.1 LICD / Sec. 2.2 TLID scheme):
 * precond_setup(u_cur), b = (i I + T_d - D) u_prev, solve, u_next = x.
 * u_next must not alias u_prev or u_cur. */
int fnls_step(fnls_ctx *ctx, const fnls_c128 *u_prev, const fnls_c128 *u_cur, fnls_c128 *u_next,
              const fnls_opts *opts, fnls_info *info);

/* Starter u^0 -> u^1: one Crank-Nicolson step with the nonlinearity frozen
 * at u^0, i.e. the same system with tau replaced by tau/2 (the paper cites a
 * second-order starter without defining it).  u1 must not alias u0. */
int fnls_first_step(fnls_ctx *ctx, const fnls_c128 *u0, fnls_c128 *u1, const fnls_opts *opts,
                    fnls_info *info);

/* A real potential V added to the diagonal by fnls_step, fnls_first_step
 * and their reverse modes: D = rho dt |u_cur|^2 + dt V (the paper's D is the
 * case V = 0; the potential is an extension for differentiating with respect
 * to a spatially varying coefficient).  V is a device pointer to N doubles,
 * owned by the caller, kept by the context and read by every later step until
 * replaced; NULL removes it.  fnls_precond_setup takes its own V argument and
 * ignores this one. */
int fnls_set_potential(fnls_ctx *ctx, const double *V);

/* Reverse mode of fnls_step (one three-level step of Sec. 2.1 / 2.2,
 * u_next = A^{-1} B u_prev with A = D - T_d + iI, B = iI + T_d - D and
 * D = rho dt |u_cur|^2 + dt V).  For a real loss L with gradients taken as
 * g_z = dL/dRe z + i dL/dIm z (PyTorch's convention for complex tensors),
 * given g_next for u_next this ACCUMULATES
 *     g_prev += B^H lam,   g_cur += 2 dt rho g_D u_cur,   g_V += dt g_D
 * (g_V may be NULL), where lam solves the adjoint system A^H lam = g_next and
 * g_D = -Re(conj(lam) (u_next + u_prev)).  A is complex symmetric, so the
 * adjoint solve is the same preconditioned GMRES applied to conj(g_next)
 * (opts / info as for fnls_solve; info describes that solve).  u_next must be
 * the forward result for (u_prev, u_cur).  Gradient outputs must not alias
 * each other or the inputs.  Returns when the result is complete. */
int fnls_step_backward(fnls_ctx *ctx, const fnls_c128 *u_prev, const fnls_c128 *u_cur,
                       const fnls_c128 *u_next, const fnls_c128 *g_next, fnls_c128 *g_prev,
                       fnls_c128 *g_cur, double *g_V, const fnls_opts *opts, fnls_info *info);

/* Reverse mode of fnls_first_step (the starter: the same system with dt / 2
 * and u_prev = u_cur = u0): g0 += (both contributions), g_V += (dt/2) g_D. */
int fnls_first_step_backward(fnls_ctx *ctx, const fnls_c128 *u0, const fnls_c128 *u1,
                             const fnls_c128 *g1, fnls_c128 *g0, double *g_V,
                             const fnls_opts *opts, fnls_info *info);

/* Batches: many independent systems of uneven sizes (each an assembled
 * context with its own operator, workspace and preconditioner setup)
 * advanced together.  Every GMRES iteration issues one launch per transform
 * pass (per line-length class: 1024, 512, 256, other; radix 4 with 1024
 * threads per workgroup unless fnls_batch_autotune chose a schedule for the
 * class), Gram-Schmidt update and Givens step for all
 * instances together;
 * each instance keeps its own convergence state, and instances that have
 * converged drop out.  All contexts must share device, stream and d (d >= 2),
 * with n >= 31 and n^(d-1) <= 262144.  The batch does not own the contexts. */
typedef struct fnls_batch fnls_batch;

/* Bytes of caller-owned device workspace for a batch of `count` instances
 * (a ring for argument staging, then the argument tables of up to 4 cached
 * iteration graphs); 0 for count outside [1, 4096]. */
size_t fnls_batch_workspace_bytes(int count);

/* Create a batch over ctxs[0..count-1] (host array of contexts).  The
 * workspace (device, 256-byte aligned) must stay valid for the batch's
 * life.  FNLS_ERR_STATE if a context is not assembled, FNLS_ERR_INVALID_ARG
 * for mismatched or unsupported contexts.
 *
 * The launches of one Arnoldi iteration read the iteration index from each
 * instance's GMRES state, so one argument table serves every iteration of a
 * GMRES cycle.  With opts->graph = 1 those launches are captured (on a
 * stream of the batch's own that executes nothing) into a hipGraph, which is
 * then launched once per iteration on the contexts' stream.  Up to 4 graphs
 * stay cached, keyed by the argument table and the launch shapes, so that
 * repeated steps with the same vectors replay them without a new capture; a
 * different vector set, a converged instance dropping out or a changed
 * omega captures a new one (least recently used slot).  The graphs hold
 * kernel nodes only. */
int fnls_batch_create(fnls_batch **out, fnls_ctx *const *ctxs, int count, void *workspace, size_t bytes);
/* Waits for the stream, then releases the graphs, events and staging memory. */
void fnls_batch_destroy(fnls_batch *batch);

/* Counters of graph mode since the batch was created: graphs captured and
 * graph launches (one per Arnoldi iteration of the batch). */
int fnls_batch_graph_stats(const fnls_batch *batch, long long *captures, long long *replays);

/* f1 -- Solve A_k x_k = b_k for every instance k (host arrays of device
 * vectors) with each instance's last precond_setup; same options for all
 * (fixed_iters not supported); infos (may be NULL) receives one fnls_info per
 * instance.  Returns FNLS_OK, FNLS_NOT_CONVERGED if any instance did not
 * converge, or an error. */
int fnls_batch_solve(fnls_batch *batch, const fnls_c128 *const *b, fnls_c128 *const *x,
                     const fnls_opts *opts, fnls_info *infos);

/* One three-level step of every instance (precond_setup(u_cur), b, solve),
 * as fnls_step. */
int fnls_batch_step(fnls_batch *batch, const fnls_c128 *const *u_prev, const fnls_c128 *const *u_cur,
                    fnls_c128 *const *u_next, const fnls_opts *opts, fnls_info *infos);

/* Autotune the batch's transform schedules: for every line-length class of
 * the batch with a compile-time plan (m = n + 1 = 256, 512, 1024), and for
 * its strided and then its contiguous axes, time batched solves of the
 * right-hand sides b (host array of device vectors, one per instance; every
 * instance's last precond_setup; default options in the given precision;
 * per schedule one untimed solve, then the fastest of two runs of `reps`
 * solves) over radix {4, 8} x lines per workgroup {1, 2, 4} (the rule of
 * fnls_set_pass_config; radix 4 with 4 lines is the default shape of 1024
 * threads), keeping a candidate only when it is more than 1 % faster.  The
 * batch keeps the result for its later launches.  *classes (may be NULL)
 * receives the number of classes tuned.  Solutions are written into each
 * instance's workspace only.  Returns when done. */
int fnls_batch_autotune(fnls_batch *batch, const fnls_c128 *const *b, int precision, int reps, int *classes);

/* The schedule fnls_batch_autotune chose for line length n + 1, precision and
 * axis kind (strided = 1: the non-contiguous axes): *rmax and *lines, both 0
 * when the class runs the default shape. */
int fnls_batch_schedule(const fnls_batch *batch, int n, int precision, int strided, int *rmax, int *lines);

const char *fnls_batch_last_error(const fnls_batch *batch);

/* Per-kernel timing (optional instrumentation, used by the benchmark).
 * fnls_timing(ctx, 1) clears earlier records; every following kernel launch
 * of this context then carries a pair of HIP events that the runtime records
 * at the kernel's start and end (hipExtLaunchKernel), so a record is the
 * kernel's own execution time; fnls_timing(ctx, 0) stops recording.  fnls_timing_report waits for the
 * stream and writes one entry per kernel class (at most max_entries): the
 * number of launches, their summed event time in milliseconds, and their
 * summed algorithmic bytes (every vector a launch must read once and write
 * once).  Launches of GMRES iterations that were enqueued ahead of the
 * stopping decision and then skipped by the device count with their time and
 * zero bytes.  Returns the number of entries written, or a negative status. */
typedef struct {
    char name[64];
    int launches;
    double total_ms;
    double bytes;       /* every vector the launches read or wrote, once each      */
    double bytes_min;   /* their share of the method's minimal traffic: each vector
                           an operation (the preconditioned operator, a
                           Gram-Schmidt step, the end-of-cycle update, apply_A,
                           apply_precond, rhs, setup) must read or write, charged
                           once to the launch that first touches it, the first
                           sweep of the Gram-Schmidt dot products to the Arnoldi
                           pass that forms w; intermediates between axis passes
                           and the recomputed true residual cost nothing        */
} fnls_kernel_stat;

int fnls_timing(fnls_ctx *ctx, int enable);
int fnls_timing_report(fnls_ctx *ctx, fnls_kernel_stat *out, int max_entries);

/* Tuning of the transform passes (optional; the defaults suit m = n + 1 =
 * 1024).  For the given precision (fnls_precision) and axis kind (strided = 0:
 * the contiguous last axis, 1: the other axes): rmax in {4, 8, 16} is the
 * largest FFT radix, so m / rmax threads work on one line; `lines` (a power
 * of two) is the number of lines per workgroup at m = 1024.  Settings that
 * would exceed the workgroup size or LDS limits are rejected or clamped.
 * Waits for the context's stream. */
int fnls_set_pass_config(fnls_ctx *ctx, int precision, int strided, int rmax, int lines);

/* Autotuner of the transform-pass schedule above, for this context's
 * operator and one precision (the result is also kept for the process, per
 * line length m = n + 1, precision and axis kind: contexts assembled later
 * with the same m start from it): times solves of the device vector b with the
 * current preconditioner setup and default options (per schedule: one
 * warm-up solve, then the fastest of three runs of `reps` solves), for each
 * candidate rmax in {4, 8, 16} and lines in {1, 2, 4}, by coordinate descent
 * (strided axes first, then the contiguous axis).  A candidate replaces the
 * current schedule only when it is more than 1 % faster.  best (may be NULL) receives {rmax, lines} of
 * the contiguous and then of the strided axes; *best_ms (may be NULL) its
 * time per solve.  Uses the context's stream and workspace; returns when done. */
int fnls_autotune(fnls_ctx *ctx, const fnls_c128 *b, int precision, int reps, int best[4], double *best_ms);

/* Counters of the host's GMRES sequencing on one context (diagnostics and
 * tests).  GMRES runs the Sec. 5 protocol; the host enqueues iterations
 * ahead of their stopping decisions and reads each iteration's status from
 * pinned memory.  A cycle is a GMRES(m) cycle in FP64 or a refinement step
 * in FNLS_FP32_IR. */
typedef struct {
    long long solves;            /* solves run (fnls_solve, the steppers, reverse modes)     */
    long long cycles;            /* cycles whose end was enqueued                            */
    long long iterations;        /* Arnoldi iterations of those cycles                       */
    long long stop_predictions;  /* iterations issued only up to their first pass because
                                    the host predicted that their predecessor ends the cycle */
    long long ends_ahead;        /* cycle ends enqueued ahead of such a prediction that the
                                    device ran (the cycle stopped where predicted)           */
    long long late_reads;        /* stop reports the residual's report of the same cycle had
                                    already replaced when the host read them                 */
    long long cycles_ahead;      /* cycles enqueued before the previous cycle's residual
                                    decision was read                                        */
    long long early_stops;       /* cycles that stopped before the iteration a pending stop
                                    prediction named (possible with several iterations in
                                    flight); that prediction's guarded cycle end does not run */
} fnls_host_stats;

/* Copy the counters into *out (may be NULL); reset = 1 clears them afterwards. */
int fnls_get_host_stats(fnls_ctx *ctx, fnls_host_stats *out, int reset);

/* The host's rule for taking a status report from pinned memory, for tests
 * that exercise the real code without a device.  Each solve's reports carry
 * sequence values in (seq_base, seq_base + 2^24) modulo 2^32, odd while a
 * report is being written.  A report copied between reading seq_before and
 * seq_after is taken (returns 1) when seq_before is such a value, even,
 * seq_after == seq_before, and the report covers the awaited total of
 * iterations `target` (total >= target) or ends the solve (done != 0);
 * otherwise 0. */
int fnls_status_report_accepted(unsigned seq_base, unsigned seq_before, unsigned seq_after, int total,
                                int done, int target);

/* The host's launch geometry of a transform pass, for tests of the index
 * arithmetic without a device (host arithmetic only, no HIP call).  For the
 * pass along `axis` of the d-dimensional grid with n points per axis, in
 * `precision`, with largest radix `rmax` (4, 8 or 16) and the lines setting
 * `lines` (per workgroup at m = 1024, scaled up for shorter lines), within
 * `max_dyn_lds` bytes of dynamic LDS, writes out[0..9]: threads per line G,
 * lines per workgroup L, workgroups, dynamic LDS bytes, the axis stride, the
 * number of lines, then the line layouts with two buffers (offset of buffer B
 * and line stride, in slots) and with one (the same pair).  Returns
 * FNLS_ERR_INVALID_ARG for sizes or settings the library does not support. */
int fnls_pass_geometry(int d, int n, int axis, int precision, int rmax, int lines, size_t max_dyn_lds,
                       long long out[10]);

/* Last error message of this context ("" if none); valid until the next call. */
const char *fnls_last_error(const fnls_ctx *ctx);

/* Static description of a status code. */
const char *fnls_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* FNLS_H */
