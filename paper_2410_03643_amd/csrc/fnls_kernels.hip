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
#include "fnls_common.h"
#include "fnls_device.hpp"

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
__device__ void report(GmresState* st, HostStatus* hs, int stopped) {
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
// once after the cycle stopped); 2 = it closes the cycle and was enqueued
// before the stop was known (returns at once unless the cycle has stopped).
// Every workgroup reads st->active before any write to it in the same launch.
__device__ __forceinline__ bool launch_skipped(int check_active, const GmresState* st) {
    return check_active == 1 ? st->active == 0 : (check_active == 2 ? st->active != 0 : false);
}

__device__ __forceinline__ double2 dmk(double a, double b) { double2 r; r.x = a; r.y = b; return r; }
__device__ __forceinline__ double2 ddiv(double2 a, double2 b) {
    const double den = b.x * b.x + b.y * b.y;
    return dmk((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
__device__ __forceinline__ double dabs(double2 a) { return hypot(a.x, a.y); }

// Arnoldi step finish (after the second Gram-Schmidt round): new Hessenberg
// column, Givens rotation, residual estimate, stopping decision, and -- when
// the cycle stops -- the least-squares solution y and combination
// coefficients y_i sigma_i.  Rotation convention: c = |a|/r,
// s = (a/|a|) conj(b)/r, (x, y) -> (c x + s y, -conj(s) x + c y).
// s_col holds the new Hessenberg column (rows 0..j), s_cs / s_sn the earlier
// rotations, all staged in LDS by the whole workgroup; one thread runs this.
__device__ void arnoldi_finish(GmresState* st, HostStatus* hs, double hn2, int j, double2* s_col,
                               const double* s_cs, const double2* s_sn) {
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
    const double2 gj = st->g[j];
    st->g[j + 1] = dmk(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
    st->g[j] = dmk(c * gj.x, c * gj.y);
    st->total += 1;
    const double est = dabs(st->g[j + 1]) / st->refnorm;
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
        for (int i = k - 1; i >= 0; --i) {
            double2 acc = st->g[i];
            for (int l = i + 1; l < k; ++l) {
                const double2 rl = st->R[l][i];
                const double2 yl = st->y[l];
                acc.x -= rl.x * yl.x - rl.y * yl.y;
                acc.y -= rl.x * yl.y + rl.y * yl.x;
            }
            st->y[i] = ddiv(acc, st->R[i][i]);
        }
        for (int i = 0; i < k; ++i) st->coef[i] = dmk(st->y[i].x * st->sigma[i], st->y[i].y * st->sigma[i]);
        st->active = 0;
    } else {
        st->sigma[j + 1] = 1.0 / hn;
        st->j = j + 1;
    }
    report(st, hs, stop);
}

// Decision after the recomputed residual r = b - A x (end of a GMRES cycle
// in FP64 mode, end of a refinement step in FP32-IR mode).
__device__ void residual_finish(GmresState* st, HostStatus* hs, double rn2, int ir) {
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
__device__ void reduce_partials(const double2* __restrict__ p, int ps, int nb, int nv, double2* tot,
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
__device__ void block_partial_write(const double2* red, int nv, double2* partials, int pstride, int blk) {
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

// ---------------------------------------------------------------------------
// the fused axis pass
// ---------------------------------------------------------------------------
// RMAX: largest FFT radix; G = m / RMAX threads per line, so every thread
// owns about RMAX unknowns of its line in the element phases.
template <int RMAX> struct PassThreads { static constexpr int v = 4096 / RMAX; };
template <> struct PassThreads<16> { static constexpr int v = 256; };

// LGM > 0: the line length m = 2^LGM is a compile-time constant (the host
// launches this specialisation only when a.lgm == LGM); 0: generic.
// BJ: the launch may take its iteration index from the GMRES state (a.dev_j).
template <typename R, int RMAX, int LGM, int INM, int OPS, int ZM, int OUTM, int FIN, bool BJ = false>
__device__ __forceinline__ void pass_body(const PassArgs& a, int blk_in) {
    using C = cplx<R>;
    constexpr int kMaxEptLine = RMAX;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (launch_skipped(a.check_active, a.st)) return;
    // with a fused Givens step, logical block 0 (dispatched first, so it runs
    // beside the first round of line blocks) does it; line blocks follow
    const int blk = a.gfuse ? blk_in - 1 : blk_in;
    if (a.gfuse && blk_in == 0) {
        // the previous iteration's Givens step, beside this pass's line work
        double2* s_red = reinterpret_cast<double2*>(smem_raw);   // waves
        double2* s_tot = s_red + 32;
        double2* s_col = s_tot + 2;                                // kMaxRestart + 1
        double2* s_sn = s_col + (kMaxRestart + 1);                 // kMaxRestart
        double* s_cs = reinterpret_cast<double*>(s_sn + kMaxRestart);
        reduce_partials(a.gpin, a.gpin_stride, a.gpin_nb, 1, s_tot, s_red);
        GmresState* st = a.st;
        const int j = st->j;
        for (int i = threadIdx.x; i <= j; i += blockDim.x) s_col[i] = st->hcol[i];
        for (int i = threadIdx.x; i < j; i += blockDim.x) {
            s_cs[i] = st->cs[i];
            s_sn[i] = st->sn[i];
        }
        __syncthreads();
        if (threadIdx.x == 0) arnoldi_finish(st, a.hs, s_tot[0].x, j, s_col, s_cs, s_sn);
        return;
    }

    // operands that depend on the Arnoldi iteration index
    const void* in_p = a.in;
    void* out_p = a.out;
    void* zout_p = a.zout;
    int basis_j = a.basis_j;
    if (BJ && a.dev_j) {
        const int j = a.st->j;
        basis_j = j;
        if (INM == IN_BASIS)
            in_p = (j == 0) ? a.v0 : (const void*)(reinterpret_cast<const C*>(a.vbase) + (long long)(j - 1) * a.N);
        else if (in_p)
            in_p = reinterpret_cast<const C*>(in_p) + (long long)j * a.jin;
        if (out_p) out_p = reinterpret_cast<C*>(out_p) + (long long)j * a.jout;
        if (zout_p) zout_p = reinterpret_cast<C*>(zout_p) + (long long)j * a.jz;
    }

    const int lgm = LGM ? LGM : a.lgm;
    const int m = 1 << lgm;
    const int n = m - 1;
    const int G = LGM ? (1 << LGM) / RMAX : a.G;
    const int lgG = LGM ? LGM - Lg<RMAX>::v : a.lgG;
    const int L = a.L, lgL = a.lgL;
    const int T = G * L;
    const int tid = threadIdx.x;
    const int line = tid >> lgG;
    const int lt = tid & (G - 1);
    const long long stride = a.stride;
    const bool contiguous = (stride == 1);
    // slots of one line buffer (>= m) and line stride (buffers A and B for
    // the Toeplitz product, A alone otherwise), both chosen by the host
    constexpr bool kTwoBuf = (OPS & OP_TOEP) != 0;
    const int PA = a.pa;
    const int LS = a.ls;
    // dynamic LDS: L lines | quarter twiddle table | per-line base offsets | per-line Lambda
    C* lds = reinterpret_cast<C*>(smem_raw);
    C* twl = lds + (size_t)L * LS;                    // W_m^q at tw_slot(q), q < max(1, m/4)
    const int nq = m >= 4 ? (m >> 2) : 1;
    long long* s_base = reinterpret_cast<long long*>(twl + nq);
    R* s_lamo = reinterpret_cast<R*>(s_base + L);

    const C* tw = reinterpret_cast<const C*>(a.tw);
    const R* lam = reinterpret_cast<const R*>(a.lam);
    const R* Dv = reinterpret_cast<const R*>(a.D);
    const R tscale = static_cast<R>(a.tscale);
    const int E = L * n;
    // per-thread twiddles of the compile-time plan, read while the line
    // data loads are in flight
    // (the passes that keep z across the Toeplitz product are short of
    // registers: no wl there)
    LineTw<R, RMAX, LGM, !((OPS & OP_TOEP) && OUTM == OUT_ACC_FIRST)> ltw;
    ltw.init(tw, lt);

    // coalescing element map: e -> (line l, unknown j); rows are contiguous on
    // the last axis, lines are interleaved on strided axes
    auto emap = [&](int e, int& l, int& j) {
        if (contiguous) {
            l = (n == 1) ? e : (int)__umulhi((unsigned)e, a.magic_n);
            j = e - l * n;
        } else {
            j = e >> lgL;
            l = e & (L - 1);
        }
    };

    // per-line base offset and Lambda of the other axes
    for (int l = tid; l < L; l += T) {
        const long long lg = (long long)blk * L + l;
        long long base = -1;
        R lamo = 0;
        if (lg < a.nlines) {
            const long long o = lg / stride;
            const long long i = lg - o * stride;
            base = o * (long long)n * stride + i;
            if (OPS & OP_DIV) {
                long long t = o;
                for (int ax = 0; ax < a.axis; ++ax) {
                    lamo += lam[(int)(t % n) + 1];
                    t /= n;
                }
                t = i;
                for (int ax = a.axis + 1; ax < a.d; ++ax) {
                    lamo += lam[(int)(t % n) + 1];
                    t /= n;
                }
                lamo *= tscale;
            }
        }
        s_base[l] = base;
        s_lamo[l] = lamo;
        lds[(size_t)l * LS] = czero<C>();   // slot 0: the Dirichlet zero
    }
    for (int q = tid; q < nq; q += T) twl[tw_slot<R>(q)] = tw[2 * q];
    __syncthreads();

    // ---- load phase
    {
        double sig = 1.0;
        if (INM == IN_BASIS) sig = a.st->sigma[basis_j];
        int nvc = 0;
        if (INM == IN_COMBO) nvc = a.st->k;
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const int e = tid + q * T;
            if (e < E) {
                int l, j;
                emap(e, l, j);
                const long long base = s_base[l];
                C v = czero<C>();
                if (base >= 0) {
                    const long long gi = base + (long long)j * stride;
                    if (INM == IN_PLAIN) {
                        v = ld<R>(in_p, gi);
                    } else if (INM == IN_BASIS) {
                        const C t = ld<R>(in_p, gi);
                        v = cm<R>(static_cast<R>(t.x * sig), static_cast<R>(t.y * sig));
                    } else if (a.zsum) {
                        // sum_k y_k z_k over the stored preconditioned basis
                        // (complex64 when z32), accumulated in FP64
                        double sx = 0.0, sy = 0.0;
                        for (int i = 0; i < nvc; ++i) {
                            const long long zi = (long long)i * a.N + gi;
                            double tx, ty;
                            if (a.z32) {
                                const float2 t = reinterpret_cast<const float2*>(a.vbase)[zi];
                                tx = t.x;
                                ty = t.y;
                            } else {
                                const double2 t = reinterpret_cast<const double2*>(a.vbase)[zi];
                                tx = t.x;
                                ty = t.y;
                            }
                            const double2 c = a.st->y[i];
                            sx += c.x * tx - c.y * ty;
                            sy += c.x * ty + c.y * tx;
                        }
                        v = cm<R>(static_cast<R>(sx), static_cast<R>(sy));
                    } else {
                        double sx = 0.0, sy = 0.0;
                        for (int i = 0; i < nvc; ++i) {
                            const C t = (i == 0) ? ld<R>(a.v0, gi) : ld<R>(a.vbase, (long long)(i - 1) * a.N + gi);
                            const double2 c = a.st->coef[i];
                            sx += c.x * t.x - c.y * t.y;
                            sy += c.x * t.y + c.y * t.x;
                        }
                        v = cm<R>(static_cast<R>(sx), static_cast<R>(sy));
                    }
                }
                lds[(size_t)l * LS + j + 1] = v;
            }
        }
    }
    __syncthreads();

    C* A = lds + (size_t)line * LS;
    C* B = kTwoBuf ? A + PA : A;   // B exists only for the Toeplitz product

    // ---- transform stages
    if (OPS & OP_DST1) line_dst<R, RMAX, LGM>(A, B, lgm, lt, G, tw, twl, ltw);
    if (OPS & OP_DIV) {
        const R om = static_cast<R>(a.omega);
        const R lo = s_lamo[line];
        for (int k = lt + 1; k < m; k += G) {
            const R mu = lo + tscale * lam[k];
            const R den = om * om + mu * mu;
            const C v = A[k];
            // v / (om + i mu) = v (om - i mu) / den
            A[k] = cm<R>((v.x * om + v.y * mu) / den, (v.y * om - v.x * mu) / den);
        }
        __syncthreads();
    }
    if (OPS & OP_DST2) line_dst<R, RMAX, LGM>(A, B, lgm, lt, G, tw, twl, ltw);

    constexpr bool kToep = (OPS & OP_TOEP) != 0;
    constexpr bool kKeepZ = kToep && (OUTM == OUT_ACC_FIRST);
    constexpr bool kPhase1 = (OPS & OP_SCALE) || (ZM != Z_NONE) || (OUTM == OUT_ACC_FIRST) || !kToep;
    C zreg[kKeepZ ? kMaxEptLine : 1];
    C oreg[FIN == FIN_WDOTS ? kMaxEptLine : 1];
    double nrm = 0.0;

    // ---- element phase 1: preconditioner scale, z / x outputs, Toeplitz operand
    if (kPhase1) {
        const double om = a.omega;
        // every global operand of this phase is loaded before the first
        // global store (a store could alias a later load, which would
        // serialise one memory round trip per element)
        constexpr bool kNeedD = (OPS & OP_SCALE) != 0;
        constexpr bool kNeedX = (ZM == Z_XADD);
        R dpre[kNeedD ? kMaxEptLine : 1];
        double2 xpre[kNeedX ? kMaxEptLine : 1];
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const int e = tid + q * T;
            if (kNeedD) dpre[q] = R(0);
            if (kNeedX) xpre[q] = dmk(0.0, 0.0);
            if (e >= E) continue;
            int l, j;
            emap(e, l, j);
            const long long base = s_base[l];
            if (base < 0) continue;
            const long long gi = base + (long long)j * stride;
            if (kNeedD) dpre[q] = Dv[gi];
            if (kNeedX && !a.first_cycle) xpre[q] = a.x64[gi];
        }
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const int e = tid + q * T;
            if (e >= E) continue;
            int l, j;
            emap(e, l, j);
            const long long base = s_base[l];
            C z = lds[(size_t)l * LS + j + 1];
            if (base >= 0) {
                const long long gi = base + (long long)j * stride;
                if (OPS & OP_SCALE) {
                    const R Dj = dpre[kNeedD ? q : 0];
                    // -2 i om / ((om+1) - i D) = (2 om D - 2 i om (om+1)) / ((om+1)^2 + D^2)
                    const R op1 = static_cast<R>(om + 1.0);
                    const R den = op1 * op1 + Dj * Dj;
                    const R fr = static_cast<R>(2.0 * om) * Dj / den;
                    const R fi = -static_cast<R>(2.0 * om) * op1 / den;
                    z = cm<R>(z.x * fr - z.y * fi, z.x * fi + z.y * fr);
                }
                if (ZM == Z_WRITE) stc<R>(zout_p, gi, z);
                if (ZM == Z_XSET || ZM == Z_XADD) {
                    double2 xn = dmk((double)z.x, (double)z.y);
                    if (ZM == Z_XADD && !a.first_cycle) {
                        const double2 xo = xpre[kNeedX ? q : 0];
                        xn.x += xo.x;
                        xn.y += xo.y;
                    }
                    a.x64[gi] = xn;
                    z = cm<R>(static_cast<R>(xn.x), static_cast<R>(xn.y));
                }
                if (!kToep && FIN == FIN_WRITE && out_p) stc<R>(out_p, gi, z);
            }
            if (kKeepZ) zreg[q] = z;
            if (kToep) lds[(size_t)l * LS + j + 1] = z;
        }
        if (kToep) __syncthreads();
    }

    // ---- Toeplitz product and element phase 2
    if (kToep) {
        line_toeplitz<R, RMAX, LGM>(A, B, lgm, lt, G, tw, twl, reinterpret_cast<const R*>(a.sym_e),
                         reinterpret_cast<const R*>(a.sym_o), tscale, ltw);
        const R cT = static_cast<R>(a.cT);
        // operands first (see element phase 1)
        constexpr bool kFirst = (OUTM == OUT_ACC_FIRST);
        constexpr bool kResid = (FIN == FIN_RESID);
        R dq[kFirst ? kMaxEptLine : 1];
        C accq[kFirst ? 1 : kMaxEptLine];
        double2 bq[kResid ? kMaxEptLine : 1];
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const int e = tid + q * T;
            if (kFirst) dq[q] = R(0);
            else accq[q] = czero<C>();
            if (kResid) bq[q] = dmk(0.0, 0.0);
            if (e >= E) continue;
            int l, j;
            emap(e, l, j);
            const long long base = s_base[l];
            if (base < 0) continue;
            const long long gi = base + (long long)j * stride;
            if (kFirst) dq[q] = Dv[gi];
            else accq[q] = ld<R>(a.acc_in, gi);
            if (kResid) bq[q] = a.b64[gi];
        }
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const int e = tid + q * T;
            if (FIN == FIN_WDOTS) oreg[q] = czero<C>();
            if (e >= E) continue;
            int l, j;
            emap(e, l, j);
            const long long base = s_base[l];
            if (base < 0) continue;
            const long long gi = base + (long long)j * stride;
            const int s = j + 1;
            const C* Al = lds + (size_t)l * LS;
            const C tz = cadd(Al[s], cmulc(Al[PA + s], tw[s]));
            C o;
            if (OUTM == OUT_ACC_FIRST) {
                const R Dj = dq[kFirst ? q : 0];
                const R cD = static_cast<R>(a.cD) * Dj, ci = static_cast<R>(a.ci);
                const C z = zreg[kKeepZ ? q : 0];
                o = cm<R>(cD * z.x - ci * z.y + cT * tz.x, cD * z.y + ci * z.x + cT * tz.y);
            } else {
                const C acc = accq[kFirst ? 0 : q];
                o = cm<R>(acc.x + cT * tz.x, acc.y + cT * tz.y);
            }
            if (FIN == FIN_WRITE) {
                if (out_p) stc<R>(out_p, gi, o);
            } else if (FIN == FIN_WDOTS) {
                stc<R>(out_p, gi, o);
                oreg[q] = o;
                nrm += (double)o.x * o.x + (double)o.y * o.y;
            } else {
                const double2 b = bq[kResid ? q : 0];
                const double2 r = dmk(b.x - (double)o.x, b.y - (double)o.y);
                a.r64[gi] = r;
                if (a.r32) reinterpret_cast<float2*>(a.r32)[gi] = make_float2((float)r.x, (float)r.y);
                nrm += r.x * r.x + r.y * r.y;
            }
        }
    }
    if (FIN == FIN_WRITE) return;

    // ---- reductions: Arnoldi dot products (conj(v_i) w) or ||r||^2.  The
    // line buffers are free now; their LDS holds the per-wavefront sums
    // (the host sizes the allocation for (kMaxRestart + 2) * waves entries).
    __syncthreads();
    double2* s_red = reinterpret_cast<double2*>(smem_raw);
    const int nwv = T >> 6;
    const int lane = tid & 63, wave = tid >> 6;
    int nv = 1;
    if (FIN == FIN_WDOTS) {
        const int nb = basis_j + 1;
        nv = nb + 1;
        // global index of each element (-1: none) and double-buffered basis
        // loads: vector i + 1 is in flight while vector i is reduced
        long long gq[kMaxEptLine];
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const int e = tid + q * T;
            gq[q] = -1;
            if (e >= E) continue;
            int l, j;
            emap(e, l, j);
            const long long base = s_base[l];
            if (base >= 0) gq[q] = base + (long long)j * stride;
        }
        auto load_vec = [&](int i, C* v) {
            const C* src = (i == 0) ? reinterpret_cast<const C*>(a.v0)
                                    : reinterpret_cast<const C*>(a.vbase) + (long long)(i - 1) * a.N;
#pragma unroll
            for (int q = 0; q < kMaxEptLine; ++q) v[q] = gq[q] >= 0 ? src[gq[q]] : czero<C>();
        };
        auto reduce_vec = [&](int i, const C* v) {
            double sx = 0.0, sy = 0.0;
#pragma unroll
            for (int q = 0; q < kMaxEptLine; ++q) {
                const C w = oreg[FIN == FIN_WDOTS ? q : 0];
                sx += (double)v[q].x * w.x + (double)v[q].y * w.y;
                sy += (double)v[q].x * w.y - (double)v[q].y * w.x;
            }
            sx = wave_sum(sx);
            sy = wave_sum(sy);
            if (lane == 0) s_red[i * nwv + wave] = dmk(sx, sy);
        };
        // two register buffers with compile-time indices (no scratch)
        C va[kMaxEptLine], vb[kMaxEptLine];
        load_vec(0, va);
        for (int i = 0; i < nb; i += 2) {
            if (i + 1 < nb) load_vec(i + 1, vb);
            reduce_vec(i, va);
            if (i + 1 < nb) {
                if (i + 2 < nb) load_vec(i + 2, va);
                reduce_vec(i + 1, vb);
            }
        }
        nrm = wave_sum(nrm);
        if (lane == 0) s_red[nb * nwv + wave] = dmk(nrm, 0.0);
    } else {
        nrm = wave_sum(nrm);
        if (lane == 0) s_red[wave] = dmk(nrm, 0.0);
    }
    __syncthreads();
    block_partial_write(s_red, nv, a.pout, a.pstride, blk);
}

template <typename R, int RMAX, int LGM, int INM, int OPS, int ZM, int OUTM, int FIN>
__global__ __launch_bounds__(PassThreads<RMAX>::v) void k_pass(PassArgs a) {
    pass_body<R, RMAX, LGM, INM, OPS, ZM, OUTM, FIN>(a, xcd_block((int)blockIdx.x, (int)gridDim.x));
}

// One launch over the lines of many instances (each with its own PassArgs);
// LGM > 0: every instance has lines of length 2^LGM (compile-time plan).
template <typename R, int RMAX, int LGM, int INM, int OPS, int ZM, int OUTM, int FIN>
__global__ __launch_bounds__(PassThreads<RMAX>::v) void k_pass_batch(const PassArgs* args, const int* offs,
                                                                      int count) {
    const int g = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int i = batch_find(offs, count, g);
    pass_body<R, RMAX, LGM, INM, OPS, ZM, OUTM, FIN, true>(args[i], g - offs[i]);
}

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
// NVR > 0 (MODE 0, nv = NVR known at launch): the basis values of the
// thread's elements are read once into registers and serve both the update
// and the second-round dot products (a single read of V instead of two).
template <typename R, int MODE, bool BJ = false, int NVR = 0>
__device__ __forceinline__ void cgs_body(const StreamArgs& a, int blk) {
    using C = cplx<R>;
    __shared__ double2 s_red[(kMaxRestart + 2) * kMaxWaves];
    __shared__ double2 s_tot[kMaxRestart + 2];
    __shared__ double2 s_coef[kMaxRestart + 1];
    if (launch_skipped(a.check_active, a.st)) return;
    const long long N = a.N;
    int nv = a.nv;
    void* wp = a.w;
    if (BJ && a.dev_j) {
        const int j = a.st->j;
        nv = j + 1;
        wp = reinterpret_cast<C*>(wp) + (long long)j * a.jw;
    }
    GmresState* st = a.st;
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
    C vr[kRegV ? NVR : 1][kRegV ? kEpt : 1];
    if constexpr (kRegV) {
#pragma unroll
        for (int vi = 0; vi < NVR; ++vi) {
            const void* vp = (vi == 0) ? a.v0
                                       : (const void*)(reinterpret_cast<const C*>(a.vbase) + (long long)(vi - 1) * N);
#pragma unroll
            for (int q = 0; q < kEpt; ++q) {
                const long long i = base + (long long)q * kStreamThreads;
                vr[vi][q] = i < N ? ld<R>(vp, i) : czero<C>();
            }
        }
#pragma unroll
        for (int vi = 0; vi < NVR; ++vi) {
            const double2 c = s_coef[vi];
#pragma unroll
            for (int q = 0; q < kEpt; ++q) {
                cmsub(wx[q], wy[q], c, vr[vi][q].x, vr[vi][q].y);
            }
        }
    } else {
        for (int vi = 0; vi < nv; ++vi) {
            const void* vp = (vi == 0) ? a.v0
                                       : (const void*)(reinterpret_cast<const C*>(a.vbase) + (long long)(vi - 1) * N);
            const double2 c = s_coef[vi];
            C v[kEpt];
#pragma unroll
            for (int q = 0; q < kEpt; ++q) {
                const long long i = base + (long long)q * kStreamThreads;
                v[q] = i < N ? ld<R>(vp, i) : czero<C>();
            }
#pragma unroll
            for (int q = 0; q < kEpt; ++q) {
                cmsub(wx[q], wy[q], c, v[q].x, v[q].y);
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
        nout = NVR;
    } else if (MODE == 0) {
        for (int vi = 0; vi < nv; ++vi) {
            const void* vp = (vi == 0) ? a.v0
                                       : (const void*)(reinterpret_cast<const C*>(a.vbase) + (long long)(vi - 1) * N);
            C v[kEpt];
#pragma unroll
            for (int q = 0; q < kEpt; ++q) {
                const long long i = base + (long long)q * kStreamThreads;
                v[q] = i < N ? ld<R>(vp, i) : czero<C>();
            }
            double sx = 0.0, sy = 0.0;
#pragma unroll
            for (int q = 0; q < kEpt; ++q) {
                cdot_acc(sx, sy, v[q].x, v[q].y, wr[q].x, wr[q].y);
            }
            sx = wave_sum(sx);
            sy = wave_sum(sy);
            if (lane == 0) s_red[vi * kMaxWaves + wave] = dmk(sx, sy);   // blockDim 256: kMaxWaves waves
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
enum FinishKind { FIN_K_PREPARE = 0, FIN_K_GIVENS = 1, FIN_K_RESID = 2, FIN_K_REDUCE = 3 };

__device__ __forceinline__ void finish_body(const StreamArgs& a) {
    __shared__ double2 s_red[(kMaxRestart + 2) * kMaxWaves];
    __shared__ double2 s_tot[kMaxRestart + 2];
    GmresState* st = a.st;
    if (launch_skipped(a.check_active, st)) return;
    const int nv = (a.mode == FIN_K_REDUCE) ? a.nv : 1;
    reduce_partials(a.pin, a.pin_stride, a.pin_nb, nv, s_tot, s_red);
    if (a.mode == FIN_K_REDUCE) {
        // totals written contiguously: the partials of a single producer
        // workgroup with stride 1 (pout holds kMaxRestart + 2 values)
        for (int i = threadIdx.x; i < nv; i += blockDim.x) a.pout[i] = s_tot[i];
        return;
    }
    if (a.mode == FIN_K_GIVENS) {
        __shared__ double2 s_col[kMaxRestart + 1];
        __shared__ double2 s_sn[kMaxRestart];
        __shared__ double s_cs[kMaxRestart];
        const int j = st->j;
        for (int i = threadIdx.x; i <= j; i += blockDim.x) s_col[i] = st->hcol[i];
        for (int i = threadIdx.x; i < j; i += blockDim.x) {
            s_cs[i] = st->cs[i];
            s_sn[i] = st->sn[i];
        }
        __syncthreads();
        if (threadIdx.x == 0) arnoldi_finish(st, a.hs, s_tot[0].x, j, s_col, s_cs, s_sn);
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
// one workgroup per instance
__global__ __launch_bounds__(kStreamThreads) void k_finish_batch(const StreamArgs* args) { finish_body(args[blockIdx.x]); }

// ---------------------------------------------------------------------------
// host-side launchers (declared in fnls_launch.h)
// ---------------------------------------------------------------------------
}  // namespace fnls

#include <hip/hip_ext.h>

#include <algorithm>

#include "fnls_launch.h"

namespace fnls {

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

template <typename R, int RMAX, int LGM, int INM, int OPS, int ZM, int OUTM, int FIN>
static hipError_t launch_pass_t(const PassArgs& a, int blocks, size_t lds, hipStream_t s, const LaunchEvents* te) {
    auto kern = k_pass<R, RMAX, LGM, INM, OPS, ZM, OUTM, FIN>;
    // dynamic LDS above 64 KiB must be allowed per kernel; remember the largest granted
    static size_t granted = 64 * 1024;
    if (lds > granted) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        granted = lds;
    }
    if (a.G * a.L > PassThreads<RMAX>::v) return hipErrorInvalidConfiguration;
    if (LGM && (a.lgm != LGM || a.G != (1 << LGM) / RMAX)) return hipErrorInvalidConfiguration;
    return launch_k(kern, dim3(blocks), dim3(a.G * a.L), lds, s, te, a);
}

template <typename R, int INM, int OPS, int ZM, int OUTM, int FIN>
static hipError_t launch_pass_r(int rmax, const PassArgs& a, int blocks, size_t lds, hipStream_t s,
                                const LaunchEvents* te) {
    if (a.lgm == 10) {   // m = 1024: compile-time plan
        if (rmax == 4) return launch_pass_t<R, 4, 10, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
        if (rmax == 8) return launch_pass_t<R, 8, 10, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
    }
    // m = 512 and 256 (d = 2, n = 511; d = 3, n = 255): compile-time radix-4 plans
    if (a.lgm == 9 && rmax == 4) return launch_pass_t<R, 4, 9, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
    if (a.lgm == 8 && rmax == 4) return launch_pass_t<R, 4, 8, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
    switch (rmax) {
        case 4: return launch_pass_t<R, 4, 0, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
        case 8: return launch_pass_t<R, 8, 0, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
        case 16: return launch_pass_t<R, 16, 0, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
        default: return hipErrorInvalidValue;
    }
}

#define FNLS_PASS_CASE(R, INM, OPS, ZM, OUTM, FIN)                                            \
    if (v.inm == INM && v.ops == (OPS) && v.zm == ZM && v.outm == OUTM && v.fin == FIN)       \
        return launch_pass_r<R, INM, OPS, ZM, OUTM, FIN>(v.rmax, a, blocks, lds, s, te);

template <typename R>
static hipError_t dispatch_pass(const PassVariant& v, const PassArgs& a, int blocks, size_t lds, hipStream_t s,
                                const LaunchEvents* te) {
    constexpr int DST = OP_DST1;
    constexpr int DDD = OP_DST1 | OP_DIV | OP_DST2;
    constexpr int LASTDST = OP_DST1 | OP_SCALE;
    constexpr int LASTDST_T = OP_DST1 | OP_SCALE | OP_TOEP;
    constexpr int FULL1 = OP_DST1 | OP_DIV | OP_DST2 | OP_SCALE;
    constexpr int FULL1_T = FULL1 | OP_TOEP;
    constexpr int TOEP = OP_TOEP;
    // forward / middle sine transforms
    FNLS_PASS_CASE(R, IN_PLAIN, DST, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_BASIS, DST, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, DDD, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_BASIS, DDD, Z_NONE, OUT_LINE, FIN_WRITE)
    // last sine transform of the preconditioner (d >= 2)
    FNLS_PASS_CASE(R, IN_PLAIN, LASTDST, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, LASTDST_T, Z_WRITE, OUT_ACC_FIRST, FIN_WRITE)
    // d = 1: the whole preconditioned operator on one line
    FNLS_PASS_CASE(R, IN_PLAIN, FULL1, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_BASIS, FULL1_T, Z_NONE, OUT_ACC_FIRST, FIN_WDOTS)
    FNLS_PASS_CASE(R, IN_COMBO, FULL1_T, Z_XADD, OUT_ACC_FIRST, FIN_RESID)
    FNLS_PASS_CASE(R, IN_COMBO, FULL1, Z_XADD, OUT_LINE, FIN_WRITE)
    // Toeplitz passes
    FNLS_PASS_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_FIRST, FIN_WRITE)
    // end of a cycle (d >= 2): x (+)= sum_k y_k z_k, then the residual's first axis
    FNLS_PASS_CASE(R, IN_COMBO, TOEP, Z_XADD, OUT_ACC_FIRST, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_FIRST, FIN_RESID)
    FNLS_PASS_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_NEXT, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_NEXT, FIN_WDOTS)
    FNLS_PASS_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_NEXT, FIN_RESID)
    return hipErrorInvalidValue;
}

hipError_t launch_pass(int fp64, const PassVariant& v, const PassArgs& a, int blocks, size_t lds, hipStream_t s,
                       const LaunchEvents* te) {
    return fp64 ? dispatch_pass<double>(v, a, blocks, lds, s, te) : dispatch_pass<float>(v, a, blocks, lds, s, te);
}

// ---- batched launches (radix 4, 1024 threads per workgroup; line length
// 2^LGM for every instance of the launch, or generic with LGM = 0) ----
template <typename R, int LGM, int INM, int OPS, int ZM, int OUTM, int FIN>
static hipError_t launch_pass_batch_l(const PassArgs* args, const int* offs, int count, int blocks, size_t lds,
                                      int threads, hipStream_t s) {
    auto kern = k_pass_batch<R, 4, LGM, INM, OPS, ZM, OUTM, FIN>;
    static size_t granted = 64 * 1024;
    if (lds > granted) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        granted = lds;
    }
    if (!args) return hipSuccess;   // attribute only (before a graph capture)
    if (threads != PassThreads<4>::v) return hipErrorInvalidConfiguration;
    return launch_k(kern, dim3(blocks), dim3(threads), lds, s, nullptr, args, offs, count);
}

template <typename R, int INM, int OPS, int ZM, int OUTM, int FIN>
static hipError_t launch_pass_batch_t(int lgm, const PassArgs* args, const int* offs, int count, int blocks,
                                      size_t lds, int threads, hipStream_t s) {
    switch (lgm) {
        case 10: return launch_pass_batch_l<R, 10, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
        case 9: return launch_pass_batch_l<R, 9, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
        case 8: return launch_pass_batch_l<R, 8, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
        default: return launch_pass_batch_l<R, 0, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
    }
}

#define FNLS_BATCH_CASE(R, INM, OPS, ZM, OUTM, FIN)                                             \
    if (v.inm == INM && v.ops == (OPS) && v.zm == ZM && v.outm == OUTM && v.fin == FIN)         \
        return launch_pass_batch_t<R, INM, OPS, ZM, OUTM, FIN>(lgm, args, offs, count, blocks, lds, threads, s);

template <typename R>
static hipError_t dispatch_pass_batch(const PassVariant& v, int lgm, const PassArgs* args, const int* offs,
                                      int count, int blocks, size_t lds, int threads, hipStream_t s) {
    constexpr int DST = OP_DST1;
    constexpr int DDD = OP_DST1 | OP_DIV | OP_DST2;
    constexpr int LASTDST_T = OP_DST1 | OP_SCALE | OP_TOEP;
    constexpr int TOEP = OP_TOEP;
    FNLS_BATCH_CASE(R, IN_PLAIN, DST, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_BATCH_CASE(R, IN_BASIS, DST, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_BATCH_CASE(R, IN_PLAIN, DDD, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_BATCH_CASE(R, IN_PLAIN, LASTDST_T, Z_WRITE, OUT_ACC_FIRST, FIN_WRITE)
    FNLS_BATCH_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_FIRST, FIN_WRITE)
    FNLS_BATCH_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_NEXT, FIN_WRITE)
    FNLS_BATCH_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_NEXT, FIN_WDOTS)
    FNLS_BATCH_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_NEXT, FIN_RESID)
    return hipErrorInvalidValue;
}

hipError_t launch_pass_batch(int fp64, const PassVariant& v, int lgm, const PassArgs* args, const int* offs,
                             int count, int blocks, size_t lds, int threads, hipStream_t s) {
    return fp64 ? dispatch_pass_batch<double>(v, lgm, args, offs, count, blocks, lds, threads, s)
                : dispatch_pass_batch<float>(v, lgm, args, offs, count, blocks, lds, threads, s);
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

// First update with nv basis vectors held in registers (nv <= kCgsRegMax)
template <typename R>
static hipError_t launch_cgs_reg(const StreamArgs& a, dim3 g, dim3 b, hipStream_t s, const LaunchEvents* te) {
    switch (a.nv) {
        case 1: return launch_k(k_cgs<R, 0, 1>, g, b, 0, s, te, a);
        case 2: return launch_k(k_cgs<R, 0, 2>, g, b, 0, s, te, a);
        case 3: return launch_k(k_cgs<R, 0, 3>, g, b, 0, s, te, a);
        case 4: return launch_k(k_cgs<R, 0, 4>, g, b, 0, s, te, a);
        default: return launch_k(k_cgs<R, 0, 5>, g, b, 0, s, te, a);
    }
}
// (six vectors would spill: one workgroup per CU leaves 256 VGPRs, which
// the basis values, w and the sums exceed)
constexpr int kCgsRegMax = 5;

hipError_t launch_cgs(int fp64, int mode, const StreamArgs& a, int blocks, hipStream_t s, const LaunchEvents* te) {
    const dim3 g(blocks), b(kStreamThreads);
    if (mode == 0 && a.nv >= 1 && a.nv <= kCgsRegMax)
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
