// Kernels of libfnls (gfx950).
//
// k_pass: one fused pass over all lines along one axis of the (n,)*d grid.
// Each workgroup holds L lines in LDS.  Stages, selected at compile time:
//   load (a vector / a scaled basis vector / a combination of basis vectors)
//   -> DST-I -> divide by (omega + i Lambda) -> DST-I          (Sec. 4)
//   -> scale by -2 i omega / ((omega+1) - i D)                  (Sec. 4)
//   -> write z / set or accumulate x
//   -> Toeplitz product T_1 along the axis                      (Sec. 2.1)
//   -> output: cD D z + i ci z + cT T z  or  acc + cT T z
//   -> final: plain write | write w + Arnoldi dot products | residual b - A x
// Global loads and stores use a coalescing element map (lines interleaved on
// strided axes, rows contiguous on the last axis); the transforms use G
// threads per line.
//
// k_cgs: streaming classical Gram-Schmidt update w -= sum_i c_i v_i fused with
// the second-round dot products or with ||w||^2 and the Givens step.
//
// Reductions are two-level and in a fixed order (deterministic), without
// atomics: every workgroup writes its partial sums; the next kernel's
// workgroups each sum them again (identical totals everywhere), and a
// one-workgroup kernel (k_finish) takes the scalar decisions -- Givens step,
// residual test -- and reports them to the host.
#include <algorithm>

#include "fnls_kernels_core.hpp"

namespace fnls {

// ---------------------------------------------------------------------------
// streaming kernels
// ---------------------------------------------------------------------------

// D = rho tau |u|^2 (+ tau V), FP64 and FP32 copies.
__device__ __forceinline__ void precond_setup_body(const StreamArgs& a, int blk, int nblk) {
    const long long N = a.N;
    const double2* u = reinterpret_cast<const double2*>(a.u);
    for (long long i = (long long)blk * blockDim.x + threadIdx.x; i < N; i += (long long)nblk * blockDim.x) {
        const double2 v = u[i];
        double Dj = a.rho * a.tau * (v.x * v.x + v.y * v.y);
        if (a.V) Dj += a.tau * a.V[i];
        a.D64[i] = Dj;
        a.D32[i] = (float)Dj;
    }
}

// Solve start: per-workgroup partials of ||b||^2 (optionally writing the
// complex64 copy of b).  kEpt elements per thread, all loads issued first.
__device__ __forceinline__ void prepare_body(const StreamArgs& a, int blk) {
    __shared__ double2 s_red[kMaxWaves];
    const long long N = a.N;
    const long long base = (long long)blk * (kStreamThreads * kEpt) + threadIdx.x;
    double2 v[kEpt];
#pragma unroll
    for (int q = 0; q < kEpt; ++q) {
        const long long i = base + (long long)q * kStreamThreads;
        v[q] = i < N ? a.b64[i] : dmk(0.0, 0.0);
    }
    double nrm = 0.0;
#pragma unroll
    for (int q = 0; q < kEpt; ++q) {
        const long long i = base + (long long)q * kStreamThreads;
        nrm += v[q].x * v[q].x + v[q].y * v[q].y;
        if (a.r32 && i < N) reinterpret_cast<float2*>(a.r32)[i] = make_float2((float)v[q].x, (float)v[q].y);
    }
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = dmk(nrm, 0.0);
    __syncthreads();
    block_partial_write(s_red, 1, a.pout, a.pstride, blk);
}

// End of a cycle, flexible form: x (+)= sum_{k < st->k} y_k z_k, with z_k the
// preconditioned basis vectors P^{-1} v_k that the Arnoldi passes stored
// (complex<R>, `vbase` + k N); x in FP64.  first = 1 sets x instead of adding.
template <typename R>
__device__ __forceinline__ void zupdate_body(const StreamArgs& a, int blk) {
    using C = cplx<R>;
    const long long N = a.N;
    const int k = a.st->k;
    const long long base = (long long)blk * (kStreamThreads * kEpt) + threadIdx.x;
    double2* x = a.x64;
    double ax[kEpt], ay[kEpt];
#pragma unroll
    for (int q = 0; q < kEpt; ++q) {
        const long long i = base + (long long)q * kStreamThreads;
        const double2 v = (a.mode == 0 && i < N) ? x[i] : dmk(0.0, 0.0);
        ax[q] = v.x;
        ay[q] = v.y;
    }
    for (int kk = 0; kk < k; ++kk) {
        const C* zp = reinterpret_cast<const C*>(a.vbase) + (long long)kk * N;
        const double2 c = a.st->y[kk];
        C z[kEpt];
#pragma unroll
        for (int q = 0; q < kEpt; ++q) {
            const long long i = base + (long long)q * kStreamThreads;
            z[q] = i < N ? zp[i] : czero<C>();
        }
#pragma unroll
        for (int q = 0; q < kEpt; ++q) {
            ax[q] += c.x * (double)z[q].x - c.y * (double)z[q].y;
            ay[q] += c.x * (double)z[q].y + c.y * (double)z[q].x;
        }
    }
#pragma unroll
    for (int q = 0; q < kEpt; ++q) {
        const long long i = base + (long long)q * kStreamThreads;
        if (i < N) x[i] = dmk(ax[q], ay[q]);
    }
}

// out = conj(in) (complex128).
__global__ __launch_bounds__(256) void k_conj(const double2* in, double2* out, long long N) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
        const double2 v = in[i];
        out[i] = dmk(v.x, -v.y);
    }
}

// Gradient accumulation of one step's reverse mode (a.sol = conj(lam)):
// g_D = -Re(conj(lam) u_next) - Re(conj(lam) u_prev), g_prev += conj(w),
// g_cur += 2 dt rho g_D u_cur, g_V += dt g_D.
__global__ __launch_bounds__(256) void k_adjoint(AdjointArgs a) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.N;
         i += (long long)gridDim.x * blockDim.x) {
        const double2 s = a.sol[i];
        const double2 un = a.u_next[i], up = a.u_prev[i], uc = a.u_cur[i];
        const double gD = -(s.x * un.x - s.y * un.y) - (s.x * up.x - s.y * up.y);
        const double2 w = a.w[i];
        const double c = 2.0 * a.dt * a.rho * gD;
        double2 gp = a.g_prev[i];
        gp.x += w.x;
        gp.y -= w.y;
        if (a.g_cur) {
            double2 gc = a.g_cur[i];
            gc.x += c * uc.x;
            gc.y += c * uc.y;
            a.g_cur[i] = gc;
        } else {
            gp.x += c * uc.x;
            gp.y += c * uc.y;
        }
        a.g_prev[i] = gp;
        if (a.g_V) a.g_V[i] += a.dt * gD;
    }
}

// Classical Gram-Schmidt round on w.  MODE 0 (first update): the totals of
// the producer's partials are the dot products d_i = conj(V_i) w (i < nv) and
// ||w||^2; h_i = sigma_i d_i, w -= sum_i h_i v_i, then partials of the
// second-round dot products.  MODE 1 (second update): totals are the
// second-round d_i; w -= sum_i h_i v_i, then partials of ||w||^2.  Workgroup 0
// records h in the GMRES state (h1 + h2 is the Hessenberg column).  V_i and w
// are complex<R>; arithmetic in FP64.  Each thread owns kEpt elements
// (stride = workgroup size: every load instruction of a wavefront is
// contiguous) and issues all kEpt loads of a vector at once.
// NVR > 0 (MODE 0, nv >= NVR): the values of the first NVR basis vectors at
// the thread's elements are read once into registers and serve both the
// update and the second-round dot products (a single read of those vectors
// instead of two); vectors NVR .. nv-1 are streamed, once for the update and
// once for the dot products.
// Widest register set: six vectors would spill (one workgroup per CU leaves
// 256 VGPRs, which the basis values, w and the sums exceed).
constexpr int kCgsRegMax = 5;
template <typename R, int MODE, bool BJ = false, int NVR = 0>
__device__ __forceinline__ void cgs_body(const StreamArgs& a, int blk) {
    using C = cplx<R>;
    __shared__ double2 s_red[(kMaxRestart + 2) * kMaxWaves];
    __shared__ double2 s_tot[kMaxRestart + 2];
    __shared__ double2 s_coef[kMaxRestart + 1];
    if (launch_skipped(a.check_active, a.guard_k, a.st)) return;
    const long long N = a.N;
    int nv = a.nv;
    void* wp = a.w;
    if (BJ && a.dev_j) {
        const int j = a.st->j;
        nv = j + 1;
        wp = reinterpret_cast<C*>(wp) + (long long)j * a.jw;
    }
    GmresState* st = a.st;
    // w and the register-held basis values (or the first streamed vector)
    // are read before the dot-product totals are reduced: a barrier does not
    // wait for global loads, so they are in flight during the reduction
    const long long base = (long long)blk * (kStreamThreads * kEpt) + threadIdx.x;
    double wx[kEpt], wy[kEpt];
#pragma unroll
    for (int q = 0; q < kEpt; ++q) {
        const long long i = base + (long long)q * kStreamThreads;
        const C w = i < N ? ld<R>(wp, i) : czero<C>();
        wx[q] = w.x;
        wy[q] = w.y;
    }
    constexpr bool kRegV = (MODE == 0 && NVR > 0);
    // streamed vectors: all of them without registers; beyond the register
    // set only for the widest one (nv > kCgsRegMax is launched with
    // NVR = kCgsRegMax, smaller nv with NVR = nv), so that the narrower ones
    // keep their register counts
    constexpr bool kStream = !kRegV || NVR >= kCgsRegMax;
    auto load_v = [&](int vi, C* v) {
        const void* vp = (vi == 0) ? a.v0
                                   : (const void*)(reinterpret_cast<const C*>(a.vbase) + (long long)(vi - 1) * N);
#pragma unroll
        for (int q = 0; q < kEpt; ++q) {
            const long long i = base + (long long)q * kStreamThreads;
            v[q] = i < N ? ld<R>(vp, i) : czero<C>();
        }
    };
    C vr[kRegV ? NVR : 1][kRegV ? kEpt : 1];
    if constexpr (kRegV) {
#pragma unroll
        for (int vi = 0; vi < NVR; ++vi) load_v(vi, vr[vi]);
    }
    const int vs0 = kRegV ? NVR : 0;
    // without the register set, the double-buffered stream's first vector
    C va[kRegV ? 1 : kEpt], vb[kRegV ? 1 : kEpt];
    if constexpr (!kRegV) {
        if (vs0 < nv) load_v(vs0, va);
    }

    reduce_partials(a.pin, a.pin_stride, a.pin_nb, MODE == 0 ? nv + 1 : nv, s_tot, s_red);
    if (threadIdx.x < nv) {
        const int i = threadIdx.x;
        const double sg = st->sigma[i];
        const double2 h = dmk(s_tot[i].x * sg, s_tot[i].y * sg);
        s_coef[i] = dmk(h.x * sg, h.y * sg);
        if (blk == 0) {
            if (MODE == 0) {
                st->hcol[i] = h;
            } else {
                st->hcol[i].x += h.x;
                st->hcol[i].y += h.y;
            }
        }
    }
    if (MODE == 0 && blk == 0 && threadIdx.x == 0) st->wnorm0 = sqrt(s_tot[nv].x);
    __syncthreads();

    if constexpr (kRegV) {
#pragma unroll
        for (int vi = 0; vi < NVR; ++vi) {
            const double2 c = s_coef[vi];
#pragma unroll
            for (int q = 0; q < kEpt; ++q) {
                cmsub(wx[q], wy[q], c, vr[vi][q].x, vr[vi][q].y);
            }
        }
    }
    // streamed basis vectors, double-buffered without the register set
    // (vector vi + 1 is in flight while vector vi is applied or reduced);
    // beside the register set, one at a time (the registers are full)
    if constexpr (kStream) {
        auto apply_v = [&](int vi, const C* v) {
            const double2 c = s_coef[vi];
#pragma unroll
            for (int q = 0; q < kEpt; ++q) cmsub(wx[q], wy[q], c, v[q].x, v[q].y);
        };
        if constexpr (kRegV) {
            for (int vi = vs0; vi < nv; ++vi) {
                C v[kEpt];
                load_v(vi, v);
                apply_v(vi, v);
            }
        } else {
            for (int vi = vs0; vi < nv; vi += 2) {
                if (vi + 1 < nv) load_v(vi + 1, vb);
                apply_v(vi, va);
                if (vi + 1 < nv) {
                    if (vi + 2 < nv) load_v(vi + 2, va);
                    apply_v(vi + 1, vb);
                }
            }
        }
    }
    C wr[kEpt];
    double nrm = 0.0;
#pragma unroll
    for (int q = 0; q < kEpt; ++q) {
        const long long i = base + (long long)q * kStreamThreads;
        wr[q] = cm<R>(static_cast<R>(wx[q]), static_cast<R>(wy[q]));
        if (i < N) stc<R>(wp, i, wr[q]);
        else wr[q] = czero<C>();
        nrm = fma((double)wr[q].x, (double)wr[q].x, nrm);
        nrm = fma((double)wr[q].y, (double)wr[q].y, nrm);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int nout;
    if constexpr (kRegV) {
#pragma unroll
        for (int vi = 0; vi < NVR; ++vi) {
            double sx = 0.0, sy = 0.0;
#pragma unroll
            for (int q = 0; q < kEpt; ++q) {
                cdot_acc(sx, sy, vr[vi][q].x, vr[vi][q].y, wr[q].x, wr[q].y);
            }
            sx = wave_sum(sx);
            sy = wave_sum(sy);
            if (lane == 0) s_red[vi * kMaxWaves + wave] = dmk(sx, sy);
        }
    }
    if (MODE == 0) {
        if constexpr (kStream) {
            auto dot_v = [&](int vi, const C* v) {
                double sx = 0.0, sy = 0.0;
#pragma unroll
                for (int q = 0; q < kEpt; ++q) cdot_acc(sx, sy, v[q].x, v[q].y, wr[q].x, wr[q].y);
                sx = wave_sum(sx);
                sy = wave_sum(sy);
                if (lane == 0) s_red[vi * kMaxWaves + wave] = dmk(sx, sy);
            };
            if constexpr (kRegV) {
                for (int vi = vs0; vi < nv; ++vi) {
                    C v[kEpt];
                    load_v(vi, v);
                    dot_v(vi, v);
                }
            } else {
                if (vs0 < nv) load_v(vs0, va);
                for (int vi = vs0; vi < nv; vi += 2) {
                    if (vi + 1 < nv) load_v(vi + 1, vb);
                    dot_v(vi, va);
                    if (vi + 1 < nv) {
                        if (vi + 2 < nv) load_v(vi + 2, va);
                        dot_v(vi + 1, vb);
                    }
                }
            }
        }
        nout = nv;
    } else {
        nrm = wave_sum(nrm);
        if (lane == 0) s_red[wave] = dmk(nrm, 0.0);
        nout = 1;
    }
    __syncthreads();
    block_partial_write(s_red, nout, a.pout, a.pstride, blk);
}

// Configure GMRES limits in the device state (single thread).
__device__ __forceinline__ void config_one(GmresState* st, double tol, double outer_tol, int restart, int maxit,
                                           int fixed_iters, int max_outer, unsigned seq0) {
    st->tol = tol;
    st->inner_tol0 = tol;
    st->outer_tol = outer_tol;
    st->restart = restart;
    st->maxit = maxit;
    st->fixed_iters = fixed_iters;
    st->max_outer = max_outer;
    st->counter = 0;
    st->seq = seq0;
    st->active = 0;
    st->done = 0;
}

// Scalar decision kernel (one workgroup): sums the producer's partials and
//   FIN_K_PREPARE: initialises the GMRES state from ||b|| and reports;
//   FIN_K_GIVENS:  finishes the Arnoldi step (Givens, stopping test);
//   FIN_K_RESID:   takes the restart / refinement decision from ||b - A x||.
enum FinishKind { FIN_K_PREPARE = 0, FIN_K_GIVENS = 1, FIN_K_RESID = 2 };

__device__ __forceinline__ void finish_body(const StreamArgs& a) {
    __shared__ double2 s_red[(kMaxRestart + 2) * kMaxWaves];
    __shared__ double2 s_tot[kMaxRestart + 2];
    GmresState* st = a.st;
    if (launch_skipped(a.check_active, a.guard_k, st)) return;
    reduce_partials(a.pin, a.pin_stride, a.pin_nb, 1, s_tot, s_red);
    if (a.mode == FIN_K_GIVENS) {
        __shared__ double2 s_col[kMaxRestart + 1];
        __shared__ double2 s_sn[kMaxRestart];
        __shared__ double s_cs[kMaxRestart];
        // earlier columns of R (packed), g, sigma and y for the finish
        __shared__ double2 s_Rt[kMaxRestart * (kMaxRestart + 1) / 2];
        __shared__ double2 s_g[kMaxRestart + 1];
        __shared__ double s_sig[kMaxRestart + 1];
        __shared__ double2 s_y[kMaxRestart];
        const int j = st->j;
        for (int i = threadIdx.x; i <= j; i += blockDim.x) s_col[i] = st->hcol[i];
        for (int i = threadIdx.x; i < j; i += blockDim.x) {
            s_cs[i] = st->cs[i];
            s_sn[i] = st->sn[i];
        }
        const FinishStage fs{s_Rt, s_g, s_sig, s_y};
        stage_finish(st, j, fs, s_sig);
        __syncthreads();
        if (threadIdx.x == 0) arnoldi_finish(st, a.hs, s_tot[0].x, j, s_col, s_cs, s_sn, fs);
        return;
    }
    if (threadIdx.x != 0) return;
    if (a.mode == FIN_K_PREPARE) {
        // a single solve's limits first (no separate configuration launch;
        // batches configure their instances beforehand: cfg_restart = 0)
        if (a.cfg_restart > 0)
            config_one(st, a.cfg_tol, a.cfg_outer_tol, a.cfg_restart, a.cfg_maxit, a.cfg_fixed_iters,
                       a.cfg_max_outer, a.cfg_seq0);
        const double bn = sqrt(s_tot[0].x);
        st->bnorm = bn;
        st->refnorm = bn;
        st->relres = 1.0;
        st->total = 0;
        st->outer = 0;
        st->j = 0;
        st->k = 0;
        st->breakdown = 0;
        st->nonfinite = isfinite(bn) ? 0 : 1;
        st->est = 1.0;
        st->g[0] = dmk(bn, 0.0);
        st->sigma[0] = bn > 0.0 ? 1.0 / bn : 0.0;
        const int ok = (bn > 0.0) && isfinite(bn);
        st->active = ok;
        st->done = ok ? 0 : 1;
        if (!ok) st->relres = 0.0;
        report(st, a.hs, 0);
    } else {
        residual_finish(st, a.hs, s_tot[0].x, a.ir);
    }
}

// ---------------------------------------------------------------------------
// kernel entry points: one instance, or many instances in one launch (the
// workgroups of instance i form the block range [offs[i], offs[i+1]))
// ---------------------------------------------------------------------------
__global__ void k_config_batch(const StreamArgs* args, int count, double tol, double outer_tol, int restart,
                               int maxit, int fixed_iters, int max_outer) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) config_one(args[i].st, tol, outer_tol, restart, maxit, fixed_iters, max_outer, 0u);
}

__global__ void k_precond_setup(StreamArgs a) { precond_setup_body(a, (int)blockIdx.x, (int)gridDim.x); }
__global__ void k_precond_setup_batch(const StreamArgs* args, const int* offs, int count) {
    const int g = (int)blockIdx.x;
    const int i = batch_find(offs, count, g);
    precond_setup_body(args[i], g - offs[i], offs[i + 1] - offs[i]);
}

__global__ __launch_bounds__(kStreamThreads) void k_prepare(StreamArgs a) { prepare_body(a, (int)blockIdx.x); }
__global__ __launch_bounds__(kStreamThreads) void k_prepare_batch(const StreamArgs* args, const int* offs, int count) {
    const int g = (int)blockIdx.x;
    const int i = batch_find(offs, count, g);
    prepare_body(args[i], g - offs[i]);
}

template <typename R>
__global__ __launch_bounds__(kStreamThreads) void k_zupdate_batch(const StreamArgs* args, const int* offs, int count) {
    const int g = (int)blockIdx.x;
    const int i = batch_find(offs, count, g);
    zupdate_body<R>(args[i], g - offs[i]);
}

template <typename R, int MODE, int NVR = 0>
__global__ __launch_bounds__(kStreamThreads) void k_cgs(StreamArgs a) { cgs_body<R, MODE, false, NVR>(a, (int)blockIdx.x); }
template <typename R, int MODE>
__global__ __launch_bounds__(kStreamThreads) void k_cgs_batch(const StreamArgs* args, const int* offs, int count) {
    const int g = (int)blockIdx.x;
    const int i = batch_find(offs, count, g);
    cgs_body<R, MODE, true>(args[i], g - offs[i]);
}

__global__ __launch_bounds__(kStreamThreads) void k_finish(StreamArgs a) { finish_body(a); }

// Pre-reduction of wide partial sums (more producers than a consumer
// workgroup should read): workgroup c sums producers
// [c nb / chunks, (c + 1) nb / chunks) of each of the nv values, in a fixed
// order, into pout[i * chunks + c].
__global__ __launch_bounds__(kStreamThreads) void k_reduce_chunks(StreamArgs a, int chunks) {
    __shared__ double2 s_red[(kMaxRestart + 2) * kMaxWaves];
    __shared__ double2 s_tot[kMaxRestart + 2];
    if (launch_skipped(a.check_active, a.guard_k, a.st)) return;
    const int c = (int)blockIdx.x;
    const int b0 = (int)((long long)a.pin_nb * c / chunks);
    const int b1 = (int)((long long)a.pin_nb * (c + 1) / chunks);
    reduce_partials(a.pin + b0, a.pin_stride, b1 - b0, a.nv, s_tot, s_red);
    for (int i = threadIdx.x; i < a.nv; i += blockDim.x) a.pout[(size_t)i * chunks + c] = s_tot[i];
}
// one workgroup per instance
__global__ __launch_bounds__(kStreamThreads) void k_finish_batch(const StreamArgs* args) { finish_body(args[blockIdx.x]); }

// ---------------------------------------------------------------------------
// host-side launchers (declared in fnls_launch.h)
// ---------------------------------------------------------------------------
hipError_t launch_pass(int fp64, const PassVariant& v, const PassArgs& a, int blocks, size_t lds, hipStream_t s,
                       const LaunchEvents* te) {
    return fp64 ? launch_pass_f64(v, a, blocks, lds, s, te) : launch_pass_f32(v, a, blocks, lds, s, te);
}

hipError_t launch_pass_batch(int fp64, const PassVariant& v, int lgm, const PassArgs* args, const int* offs,
                             int count, int blocks, size_t lds, int threads, hipStream_t s) {
    return fp64 ? launch_pass_batch_f64(v, lgm, args, offs, count, blocks, lds, threads, s)
                : launch_pass_batch_f32(v, lgm, args, offs, count, blocks, lds, threads, s);
}

hipError_t launch_cgs_batch(int fp64, int mode, const StreamArgs* args, const int* offs, int count, int blocks,
                            hipStream_t s) {
    const dim3 g(blocks), b(kStreamThreads);
    if (fp64)
        return mode == 0 ? launch_k(k_cgs_batch<double, 0>, g, b, 0, s, nullptr, args, offs, count)
                         : launch_k(k_cgs_batch<double, 1>, g, b, 0, s, nullptr, args, offs, count);
    return mode == 0 ? launch_k(k_cgs_batch<float, 0>, g, b, 0, s, nullptr, args, offs, count)
                     : launch_k(k_cgs_batch<float, 1>, g, b, 0, s, nullptr, args, offs, count);
}

hipError_t launch_zupdate_batch(int fp64, const StreamArgs* args, const int* offs, int count, int blocks,
                                hipStream_t s) {
    const dim3 g(blocks), b(kStreamThreads);
    return fp64 ? launch_k(k_zupdate_batch<double>, g, b, 0, s, nullptr, args, offs, count)
                : launch_k(k_zupdate_batch<float>, g, b, 0, s, nullptr, args, offs, count);
}

hipError_t launch_prepare_batch(const StreamArgs* args, const int* offs, int count, int blocks, hipStream_t s) {
    return launch_k(k_prepare_batch, dim3(blocks), dim3(kStreamThreads), 0, s, nullptr, args, offs, count);
}

hipError_t launch_precond_setup_batch(const StreamArgs* args, const int* offs, int count, int blocks,
                                      hipStream_t s) {
    return launch_k(k_precond_setup_batch, dim3(blocks), dim3(256), 0, s, nullptr, args, offs, count);
}

hipError_t launch_finish_batch(const StreamArgs* args, int count, hipStream_t s) {
    return launch_k(k_finish_batch, dim3(count), dim3(kStreamThreads), 0, s, nullptr, args);
}

hipError_t launch_config_batch(const StreamArgs* args, int count, double tol, double outer_tol, int restart,
                               int maxit, int fixed_iters, int max_outer, hipStream_t s) {
    return launch_k(k_config_batch, dim3((count + 255) / 256), dim3(256), 0, s, nullptr, args, count, tol,
                    outer_tol, restart, maxit, fixed_iters, max_outer);
}

hipError_t launch_precond_setup(const StreamArgs& a, int blocks, hipStream_t s, const LaunchEvents* te) {
    return launch_k(k_precond_setup, dim3(blocks), dim3(kStreamThreads), 0, s, te, a);
}

hipError_t launch_prepare(const StreamArgs& a, int blocks, hipStream_t s, const LaunchEvents* te) {
    return launch_k(k_prepare, dim3(blocks), dim3(kStreamThreads), 0, s, te, a);
}

hipError_t launch_finish(const StreamArgs& a, hipStream_t s, const LaunchEvents* te) {
    return launch_k(k_finish, dim3(1), dim3(kStreamThreads), 0, s, te, a);
}

hipError_t launch_reduce_chunks(const StreamArgs& a, int chunks, hipStream_t s, const LaunchEvents* te) {
    return launch_k(k_reduce_chunks, dim3(chunks), dim3(kStreamThreads), 0, s, te, a, chunks);
}

// First update with min(nv, kCgsRegMax) basis vectors held in registers
// and the rest streamed: NVR = nv up to four vectors (those variants stream
// nothing), NVR = kCgsRegMax from five on
template <typename R>
static hipError_t launch_cgs_reg(const StreamArgs& a, dim3 g, dim3 b, hipStream_t s, const LaunchEvents* te) {
    static_assert(kCgsRegMax == 5, "one specialisation per register-set width");
    switch (a.nv) {
        case 1: return launch_k(k_cgs<R, 0, 1>, g, b, 0, s, te, a);
        case 2: return launch_k(k_cgs<R, 0, 2>, g, b, 0, s, te, a);
        case 3: return launch_k(k_cgs<R, 0, 3>, g, b, 0, s, te, a);
        case 4: return launch_k(k_cgs<R, 0, 4>, g, b, 0, s, te, a);
        default: return launch_k(k_cgs<R, 0, kCgsRegMax>, g, b, 0, s, te, a);
    }
}

hipError_t launch_cgs(int fp64, int mode, const StreamArgs& a, int blocks, hipStream_t s, const LaunchEvents* te) {
    const dim3 g(blocks), b(kStreamThreads);
    if (mode == 0 && a.nv >= 1)
        return fp64 ? launch_cgs_reg<double>(a, g, b, s, te) : launch_cgs_reg<float>(a, g, b, s, te);
    if (fp64)
        return mode == 0 ? launch_k(k_cgs<double, 0>, g, b, 0, s, te, a) : launch_k(k_cgs<double, 1>, g, b, 0, s, te, a);
    return mode == 0 ? launch_k(k_cgs<float, 0>, g, b, 0, s, te, a) : launch_k(k_cgs<float, 1>, g, b, 0, s, te, a);
}

hipError_t launch_conj(const double2* in, double2* out, long long N, hipStream_t s) {
    const int blocks = (int)std::min<long long>(4096, (N + 255) / 256);
    return launch_k(k_conj, dim3(blocks), dim3(256), 0, s, nullptr, in, out, N);
}

hipError_t launch_adjoint(const AdjointArgs& a, hipStream_t s, const LaunchEvents* te) {
    const int blocks = (int)std::min<long long>(4096, (a.N + 255) / 256);
    return launch_k(k_adjoint, dim3(blocks), dim3(256), 0, s, te, a);
}


}  // namespace fnls
