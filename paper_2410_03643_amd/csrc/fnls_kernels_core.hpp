// Device helpers shared by the kernels of libfnls (gfx950): the status
// seqlock, the launch guards, the Arnoldi / residual decisions, fixed-order
// reductions, the XCD-aware block order, and the host-side launch helper.
// Included by every kernel translation unit (the pass kernels are compiled
// per precision in fnls_pass64.hip / fnls_pass32.hip, the rest in
// fnls_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "fnls_common.h"
#include "fnls_device.hpp"
#include "fnls_launch.h"

namespace fnls {

enum OpBits { OP_DST1 = 1, OP_DIV = 2, OP_DST2 = 4, OP_SCALE = 8, OP_TOEP = 16 };
constexpr int kMaxWaves = kStreamThreads / 64;   // wavefronts of the streaming and finish kernels

// ---------------------------------------------------------------------------
// status reporting
// ---------------------------------------------------------------------------
// The host polls hs->seq instead of waiting on events, so the status block
// is published as a seqlock: seq is odd while the fields change and equals
// st->seq (even) once they are complete.  Both seq stores are system-scope
// atomics and the system-scope release orders the field stores between them,
// so a host that reads the same even seq before and after copying the
// fields holds one report, complete.
static __device__ void report(GmresState* st, HostStatus* hs, int stopped) {
    st->seq += 2;
    if (hs) {
        const unsigned s = st->seq;
        __hip_atomic_store(&hs->seq, s - 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __threadfence_system();
        hs->total = st->total;
        hs->stopped = stopped;
        hs->done = st->done;
        hs->breakdown = st->breakdown;
        hs->nonfinite = st->nonfinite;
        hs->outer = st->outer;
        hs->est = st->est;
        hs->tol = st->tol;
        hs->relres = st->relres;
        hs->bnorm = st->bnorm;
        if (st->total >= 1 && st->total <= 64) hs->hist[st->total - 1] = st->hist[st->total - 1];
        __hip_atomic_store(&hs->seq, s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// check_active of a launch: 1 = it belongs to the running cycle (returns at
// once after the cycle stopped); 2 = it closes a cycle of guard_k basis
// vectors and was enqueued before the stop was known (returns at once unless
// the cycle has stopped with exactly guard_k vectors: with several
// iterations in flight an earlier one may have stopped it, and then the host
// enqueues the end of that cycle itself).  Every workgroup reads st->active
// and st->k before any write to them in the same launch.
__device__ __forceinline__ bool launch_skipped(int check_active, int guard_k, const GmresState* st) {
    return check_active == 1 ? st->active == 0
                             : (check_active == 2 ? (st->active != 0 || st->k != guard_k) : false);
}

__device__ __forceinline__ double2 dmk(double a, double b) { double2 r; r.x = a; r.y = b; return r; }
__device__ __forceinline__ double2 ddiv(double2 a, double2 b) {
    const double den = b.x * b.x + b.y * b.y;
    return dmk((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
__device__ __forceinline__ double dabs(double2 a) { return hypot(a.x, a.y); }

// Where the Arnoldi finish reads the earlier columns of R, the right-hand
// side g and the basis scales sigma, and keeps y while it back-substitutes:
// the GMRES state itself (all null), or copies the whole workgroup staged in
// LDS beforehand (then the one thread that finishes has no global round trip
// in its serial chain).  Rt packs column l, rows 0..l at l (l + 1) / 2.
struct FinishStage {
    double2* Rt;
    double2* g;
    const double* sigma;
    double2* y;
};

// Stage columns 0..j-1 of R, g_0..g_j and sigma_0..sigma_j in LDS with every
// thread of the workgroup (a barrier follows before the finish reads them).
static __device__ void stage_finish(const GmresState* st, int j, FinishStage f, double* sigma) {
    for (int t = threadIdx.x; t < j * kMaxRestart; t += blockDim.x) {
        const int l = t / kMaxRestart, i = t - l * kMaxRestart;
        if (i <= l) f.Rt[l * (l + 1) / 2 + i] = st->R[l][i];
    }
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        f.g[i] = st->g[i];
        sigma[i] = st->sigma[i];
    }
}

// Arnoldi step finish (after the second Gram-Schmidt round): new Hessenberg
// column, Givens rotation, residual estimate, stopping decision, and -- when
// the cycle stops -- the least-squares solution y and combination
// coefficients y_i sigma_i.  Rotation convention: c = |a|/r,
// s = (a/|a|) conj(b)/r, (x, y) -> (c x + s y, -conj(s) x + c y).
// s_col holds the new Hessenberg column (rows 0..j), s_cs / s_sn the earlier
// rotations, all staged in LDS by the whole workgroup; fs the rest (or
// nothing: then they are read from the state); one thread runs this.  The
// arithmetic and its order are the same either way.
static __device__ void arnoldi_finish(GmresState* st, HostStatus* hs, double hn2, int j, double2* s_col,
                               const double* s_cs, const double2* s_sn, FinishStage fs = FinishStage{}) {
    const bool staged = fs.Rt != nullptr;
    auto R_at = [&](int l, int i) -> double2 { return staged ? fs.Rt[l * (l + 1) / 2 + i] : st->R[l][i]; };
    double2* gv = staged ? fs.g : st->g;
    const double* sgv = staged ? fs.sigma : st->sigma;
    double2* yv = staged ? fs.y : st->y;
    const double hn = sqrt(hn2);
    double2* col = s_col;
    for (int i = 0; i < j; ++i) {
        const double c = s_cs[i];
        const double2 s = s_sn[i];
        const double2 a = col[i];
        const double2 b = col[i + 1];
        // t = c a + s b ; b' = -conj(s) a + c b
        const double2 t = dmk(c * a.x + s.x * b.x - s.y * b.y, c * a.y + s.x * b.y + s.y * b.x);
        const double2 b2 = dmk(-(s.x * a.x + s.y * a.y) + c * b.x, -(s.x * a.y - s.y * a.x) + c * b.y);
        col[i] = t;
        col[i + 1] = b2;
    }
    const double2 a = col[j];
    const double aa = dabs(a);
    double c;
    double2 s;
    if (aa == 0.0) {
        c = 0.0;
        s = dmk(1.0, 0.0);
    } else {
        const double r = hypot(aa, hn);
        c = aa / r;
        s = dmk(a.x / aa * hn / r, a.y / aa * hn / r);
    }
    st->cs[j] = c;
    st->sn[j] = s;
    col[j] = dmk(c * a.x + s.x * hn, c * a.y + s.y * hn);
    for (int i = 0; i <= j; ++i) st->R[j][i] = col[i];
    const double2 gj = gv[j];
    const double2 gj1 = dmk(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
    const double2 gjn = dmk(c * gj.x, c * gj.y);
    st->g[j + 1] = gj1;
    st->g[j] = gjn;
    gv[j + 1] = gj1;
    gv[j] = gjn;
    st->total += 1;
    const double est = dabs(gj1) / st->refnorm;
    st->est = est;
    if (st->total <= 64) st->hist[st->total - 1] = est;
    const int brk = (hn <= 1e-14 * st->wnorm0) ? 1 : 0;
    const int nonfinite = (!isfinite(hn) || !isfinite(est)) ? 1 : 0;
    int stop;
    if (st->fixed_iters > 0)
        stop = st->total >= st->fixed_iters;
    else
        stop = est < st->tol;
    stop = stop || brk || nonfinite || st->total >= st->maxit || (j + 1 >= st->restart);
    if (brk) st->breakdown = 1;
    if (nonfinite) st->nonfinite = 1;
    if (stop) {
        const int k = j + 1;
        st->k = k;
        // column j of R is the new one (col); earlier ones come from R
        auto Rc = [&](int l, int i) -> double2 { return l == j ? col[i] : R_at(l, i); };
        for (int i = k - 1; i >= 0; --i) {
            double2 acc = gv[i];
            for (int l = i + 1; l < k; ++l) {
                const double2 rl = Rc(l, i);
                const double2 yl = yv[l];
                acc.x -= rl.x * yl.x - rl.y * yl.y;
                acc.y -= rl.x * yl.y + rl.y * yl.x;
            }
            yv[i] = ddiv(acc, Rc(i, i));
        }
        for (int i = 0; i < k; ++i) {
            if (staged) st->y[i] = yv[i];
            st->coef[i] = dmk(yv[i].x * sgv[i], yv[i].y * sgv[i]);
        }
        st->active = 0;
    } else {
        st->sigma[j + 1] = 1.0 / hn;
        st->j = j + 1;
    }
    report(st, hs, stop);
}

// Decision after the recomputed residual r = b - A x (end of a GMRES cycle
// in FP64 mode, end of a refinement step in FP32-IR mode).
static __device__ void residual_finish(GmresState* st, HostStatus* hs, double rn2, int ir) {
    const double rn = sqrt(rn2);
    st->relres = rn / st->bnorm;
    st->outer += 1;
    int done;
    if (!isfinite(rn)) {
        st->nonfinite = 1;
        done = 1;
    } else if (ir) {
        done = st->relres < st->outer_tol || st->outer >= st->max_outer || st->total >= st->maxit;
    } else if (st->fixed_iters > 0) {
        done = st->total >= st->fixed_iters || st->breakdown;
    } else {
        done = st->relres < st->outer_tol || st->total >= st->maxit;
    }
    st->done = done;
    if (!done) {
        // FP32-IR: the next inner solve only has to bring this residual down
        // to the outer tolerance (with a factor 2 to spare); never below the
        // requested inner tolerance
        if (ir) st->tol = fmax(st->inner_tol0, 0.5 * st->outer_tol / st->relres);
        st->refnorm = ir ? rn : st->bnorm;
        st->g[0] = dmk(rn, 0.0);
        st->sigma[0] = 1.0 / rn;
        st->j = 0;
        st->active = 1;
        st->breakdown = 0;
    } else {
        st->active = 0;
    }
    report(st, hs, 0);
}

// Sum nv per-workgroup partials (layout [i][ps], nb producer workgroups) into
// tot[i] (LDS) with every thread of the workgroup taking part.  The order is
// fixed, so every consumer workgroup obtains bit-identical totals.
static __device__ void reduce_partials(const double2* __restrict__ p, int ps, int nb, int nv, double2* tot,
                                double2* red) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nv; ++i) {
        double sx = 0.0, sy = 0.0;
        const double2* pi = p + (size_t)i * ps;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            const double2 v = pi[b];
            sx += v.x;
            sy += v.y;
        }
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        if (lane == 0) red[i * nw + wave] = dmk(sx, sy);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        double sx = 0.0, sy = 0.0;
        for (int w = 0; w < nw; ++w) {
            sx += red[i * nw + w].x;
            sy += red[i * nw + w].y;
        }
        tot[i] = dmk(sx, sy);
    }
    __syncthreads();
}

// Complex update w -= c v and accumulation of conj(v) w as explicit fused
// multiply-adds: the rounding is fixed by the source, not by the contraction
// the compiler picks in each kernel, so every kernel that applies them (one
// instance or a batch, register-held or streamed basis) rounds alike.
__device__ __forceinline__ void cmsub(double& wx, double& wy, double2 c, double vx, double vy) {
    wx = fma(-c.x, vx, wx);
    wx = fma(c.y, vy, wx);
    wy = fma(-c.x, vy, wy);
    wy = fma(-c.y, vx, wy);
}
__device__ __forceinline__ void cdot_acc(double& sx, double& sy, double vx, double vy, double wx, double wy) {
    sx = fma(vx, wx, sx);
    sx = fma(vy, wy, sx);
    sy = fma(vx, wy, sy);
    sy = fma(-vy, wx, sy);
}

// Write this workgroup's partial of nv values: red[i * nw + w] holds the
// wavefront sums (nw wavefronts); summed in wavefront order.
static __device__ void block_partial_write(const double2* red, int nv, double2* partials, int pstride, int blk) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        double sx = 0.0, sy = 0.0;
        for (int w = 0; w < nw; ++w) {
            sx += red[i * nw + w].x;
            sy += red[i * nw + w].y;
        }
        partials[(size_t)i * pstride + blk] = dmk(sx, sy);
    }
}

template <typename R>
__device__ __forceinline__ cplx<R> ld(const void* p, long long idx) {
    return reinterpret_cast<const cplx<R>*>(p)[idx];
}
template <typename R>
__device__ __forceinline__ void stc(void* p, long long idx, cplx<R> v) {
    reinterpret_cast<cplx<R>*>(p)[idx] = v;
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
// Remap the workgroup index so that every XCD works through one contiguous
// range of line blocks: on strided axes neighbouring blocks share 128-byte
// cache lines (a block covers L < 8 complex values per row), and they then
// meet in the same L2 instead of each XCD fetching the whole line.
__device__ __forceinline__ int xcd_block(int i, int nb) {
    constexpr int kXcd = 8;
    const int x = i % kXcd, q = i / kXcd;
    const int base = nb / kXcd, rem = nb % kXcd;
    return x * base + min(x, rem) + q;
}

// Batched launches: workgroups of instance i are the (logical) block range
// [offs[i], offs[i+1]); returns i for block g (offs is ascending, offs[0] = 0).
__device__ __forceinline__ int batch_find(const int* offs, int count, int g) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}


// Launch `kern` with the given arguments; with events, the runtime records
// them at the kernel's start and end.
// Launch `kern` with the given arguments; with events, the runtime records
// them at the kernel's start and end.
template <typename K, typename... Args>
static hipError_t launch_k(K kern, dim3 grid, dim3 block, size_t lds, hipStream_t s, const LaunchEvents* te,
                           Args... args) {
    (void)hipGetLastError();   // clear errors of earlier, unrelated runtime calls
    if (te) {
        void* argv[] = {reinterpret_cast<void*>(&args)...};
        return hipExtLaunchKernel(reinterpret_cast<const void*>(kern), grid, block, argv, lds, s, te->start,
                                  te->stop, 0);
    }
    hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
    return hipGetLastError();
}

}  // namespace fnls
