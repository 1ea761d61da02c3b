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
// Reductions are two-level and in a fixed order (deterministic): every
// workgroup writes its partial sums, the last workgroup to arrive (device-
// scope atomic counter) sums the partials and updates the GMRES state.
#include "fnls_common.h"
#include "fnls_device.hpp"

namespace fnls {

enum OpBits { OP_DST1 = 1, OP_DIV = 2, OP_DST2 = 4, OP_SCALE = 8, OP_TOEP = 16 };
constexpr int kMaxEptLine = 16;   // elements per thread in the element phases of k_pass
constexpr int kMaxWaves = 4;     // every kernel here runs at most 256 threads

// ---------------------------------------------------------------------------
// status reporting
// ---------------------------------------------------------------------------
__device__ void report(GmresState* st, HostStatus* hs, int stopped) {
    st->seq += 1;
    if (hs) {
        hs->total = st->total;
        hs->stopped = stopped;
        hs->done = st->done;
        hs->breakdown = st->breakdown;
        hs->nonfinite = st->nonfinite;
        hs->outer = st->outer;
        hs->est = st->est;
        hs->relres = st->relres;
        hs->bnorm = st->bnorm;
        if (st->total >= 1 && st->total <= 64) hs->hist[st->total - 1] = st->hist[st->total - 1];
        __threadfence_system();
        hs->seq = st->seq;
        __threadfence_system();
    }
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
__device__ void arnoldi_finish(GmresState* st, HostStatus* hs, double hn2) {
    const int j = st->j;
    const double hn = sqrt(hn2);
    double2* col = st->R[j];   // column j is built in place (rows 0..j)
    for (int i = 0; i <= j; ++i) col[i] = st->hcol[i];
    for (int i = 0; i < j; ++i) {
        const double c = st->cs[i];
        const double2 s = st->sn[i];
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

// Sum nv per-workgroup partials (layout [i][pstride]) in the last workgroup.
// Returns true in the last workgroup; tot[i] (LDS) then holds the totals.
__device__ bool last_block_reduce(double2* partials, int pstride, int nv, GmresState* st, double2* tot) {
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(&st->counter, 1u);
        s_last = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    const int nb = gridDim.x;
    for (int i = wave; i < nv; i += nw) {
        double sx = 0.0, sy = 0.0;
        const double2* p = partials + (size_t)i * pstride;
        for (int b = lane; b < nb; b += 64) {
            const double2 v = p[b];
            sx += v.x;
            sy += v.y;
        }
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        if (lane == 0) tot[i] = dmk(sx, sy);
    }
    __syncthreads();
    return true;
}

// Write this workgroup's partial of nv values: each thread contributes
// acc[i] via the LDS array red[i][wave] (already wave-reduced by caller).
__device__ void block_partial_write(const double2* red, int nv, double2* partials, int pstride) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        double sx = 0.0, sy = 0.0;
        for (int w = 0; w < nw; ++w) {
            sx += red[i * kMaxWaves + w].x;
            sy += red[i * kMaxWaves + w].y;
        }
        partials[(size_t)i * pstride + blockIdx.x] = dmk(sx, sy);
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

// ---------------------------------------------------------------------------
// the fused axis pass
// ---------------------------------------------------------------------------
template <typename R, int INM, int OPS, int ZM, int OUTM, int FIN>
__global__ __launch_bounds__(256) void k_pass(PassArgs a) {
    using C = cplx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (a.check_active && a.st->active == 0) return;

    const int n = a.n, m = a.m, G = a.G, L = a.L, lgL = a.lgL;
    const int T = G * L;
    const int tid = threadIdx.x;
    const int line = tid >> a.lgG;
    const int lt = tid & (G - 1);
    const long long stride = a.stride;
    const bool contiguous = (stride == 1);
    const int LS = 2 * m + 2;
    C* lds = reinterpret_cast<C*>(smem_raw);
    __shared__ R s_lamo[256];
    __shared__ long long s_base[256];
    __shared__ double2 s_red[(kMaxRestart + 2) * kMaxWaves];
    __shared__ double2 s_tot[kMaxRestart + 2];

    const C* tw = reinterpret_cast<const C*>(a.tw);
    const R* lam = reinterpret_cast<const R*>(a.lam);
    const R* Dv = reinterpret_cast<const R*>(a.D);
    const R tscale = static_cast<R>(a.tscale);
    const int E = L * n;

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
        const long long lg = (long long)blockIdx.x * L + l;
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
    __syncthreads();

    // ---- load phase
    {
        double sig = 1.0;
        if (INM == IN_BASIS) sig = a.st->sigma[a.basis_j];
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
                        v = ld<R>(a.in, gi);
                    } else if (INM == IN_BASIS) {
                        const C t = ld<R>(a.in, gi);
                        v = cm<R>(static_cast<R>(t.x * sig), static_cast<R>(t.y * sig));
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
    C* B = A + m + 1;

    // ---- transform stages
    if (OPS & OP_DST1) line_dst<R>(A, B, m, lt, G, tw);
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
    if (OPS & OP_DST2) line_dst<R>(A, B, m, lt, G, tw);

    constexpr bool kToep = (OPS & OP_TOEP) != 0;
    constexpr bool kKeepZ = kToep && (OUTM == OUT_ACC_FIRST);
    constexpr bool kPhase1 = (OPS & OP_SCALE) || (ZM != Z_NONE) || (OUTM == OUT_ACC_FIRST) || !kToep;
    C zreg[kKeepZ ? kMaxEptLine : 1];
    C oreg[FIN == FIN_WDOTS ? kMaxEptLine : 1];
    double nrm = 0.0;

    // ---- element phase 1: preconditioner scale, z / x outputs, Toeplitz operand
    if (kPhase1) {
        const double om = a.omega;
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
                    const R Dj = Dv[gi];
                    // -2 i om / ((om+1) - i D) = (2 om D - 2 i om (om+1)) / ((om+1)^2 + D^2)
                    const R op1 = static_cast<R>(om + 1.0);
                    const R den = op1 * op1 + Dj * Dj;
                    const R fr = static_cast<R>(2.0 * om) * Dj / den;
                    const R fi = -static_cast<R>(2.0 * om) * op1 / den;
                    z = cm<R>(z.x * fr - z.y * fi, z.x * fi + z.y * fr);
                }
                if (ZM == Z_WRITE) stc<R>(a.zout, gi, z);
                if (ZM == Z_XSET || ZM == Z_XADD) {
                    double2 xn = dmk((double)z.x, (double)z.y);
                    if (ZM == Z_XADD && !a.first_cycle) {
                        const double2 xo = a.x64[gi];
                        xn.x += xo.x;
                        xn.y += xo.y;
                    }
                    a.x64[gi] = xn;
                    z = cm<R>(static_cast<R>(xn.x), static_cast<R>(xn.y));
                }
                if (!kToep && FIN == FIN_WRITE && a.out) stc<R>(a.out, gi, z);
            }
            if (kKeepZ) zreg[q] = z;
            if (kToep) lds[(size_t)l * LS + j + 1] = z;
        }
        if (kToep) __syncthreads();
    }

    // ---- Toeplitz product and element phase 2
    if (kToep) {
        line_toeplitz<R>(A, B, m, lt, G, tw, reinterpret_cast<const R*>(a.sym_e),
                         reinterpret_cast<const R*>(a.sym_o), tscale);
        const R cT = static_cast<R>(a.cT);
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
            const C tz = cadd(Al[s], cmulc(Al[m + 1 + s], tw[s]));
            C o;
            if (OUTM == OUT_ACC_FIRST) {
                const R Dj = Dv[gi];
                const R cD = static_cast<R>(a.cD) * Dj, ci = static_cast<R>(a.ci);
                const C z = zreg[kKeepZ ? q : 0];
                o = cm<R>(cD * z.x - ci * z.y + cT * tz.x, cD * z.y + ci * z.x + cT * tz.y);
            } else {
                const C acc = ld<R>(a.acc_in, gi);
                o = cm<R>(acc.x + cT * tz.x, acc.y + cT * tz.y);
            }
            if (FIN == FIN_WRITE) {
                if (a.out) stc<R>(a.out, gi, o);
            } else if (FIN == FIN_WDOTS) {
                stc<R>(a.out, gi, o);
                oreg[q] = o;
                nrm += (double)o.x * o.x + (double)o.y * o.y;
            } else {
                const double2 b = a.b64[gi];
                const double2 r = dmk(b.x - (double)o.x, b.y - (double)o.y);
                a.r64[gi] = r;
                if (a.r32) reinterpret_cast<float2*>(a.r32)[gi] = make_float2((float)r.x, (float)r.y);
                nrm += r.x * r.x + r.y * r.y;
            }
        }
    }
    if (FIN == FIN_WRITE) return;

    // ---- reductions: Arnoldi dot products (conj(v_i) w) or ||r||^2
    const int lane = tid & 63, wave = tid >> 6;
    int nv = 1;
    if (FIN == FIN_WDOTS) {
        const int nb = a.basis_j + 1;
        nv = nb + 1;
        for (int i = 0; i < nb; ++i) {
            double sx = 0.0, sy = 0.0;
#pragma unroll
            for (int q = 0; q < kMaxEptLine; ++q) {
                const int e = tid + q * T;
                if (e >= E) continue;
                int l, j;
                emap(e, l, j);
                const long long base = s_base[l];
                if (base < 0) continue;
                const long long gi = base + (long long)j * stride;
                const C v = (i == 0) ? ld<R>(a.v0, gi) : ld<R>(a.vbase, (long long)(i - 1) * a.N + gi);
                const C w = oreg[FIN == FIN_WDOTS ? q : 0];
                sx += (double)v.x * w.x + (double)v.y * w.y;
                sy += (double)v.x * w.y - (double)v.y * w.x;
            }
            sx = wave_sum(sx);
            sy = wave_sum(sy);
            if (lane == 0) s_red[i * kMaxWaves + wave] = dmk(sx, sy);
        }
        nrm = wave_sum(nrm);
        if (lane == 0) s_red[nb * kMaxWaves + wave] = dmk(nrm, 0.0);
    } else {
        nrm = wave_sum(nrm);
        if (lane == 0) s_red[wave] = dmk(nrm, 0.0);
    }
    __syncthreads();
    block_partial_write(s_red, nv, a.partials, a.pstride);
    if (!last_block_reduce(a.partials, a.pstride, nv, a.st, s_tot)) return;
    if (tid == 0) {
        GmresState* st = a.st;
        st->counter = 0;
        if (FIN == FIN_WDOTS) {
            const int nb = nv - 1;
            for (int i = 0; i < nb; ++i) {
                const double sg = st->sigma[i];
                const double2 h = dmk(s_tot[i].x * sg, s_tot[i].y * sg);
                st->hcol[i] = h;
                st->coef[i] = dmk(h.x * sg, h.y * sg);
            }
            st->wnorm0 = sqrt(s_tot[nb].x);
        } else {
            residual_finish(st, a.hs, s_tot[0].x, a.ir);
        }
    }
}

// ---------------------------------------------------------------------------
// streaming kernels
// ---------------------------------------------------------------------------

// D = rho tau |u|^2 (+ tau V), FP64 and FP32 copies.
__global__ void k_precond_setup(StreamArgs a) {
    const long long N = a.N;
    const double2* u = reinterpret_cast<const double2*>(a.u);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
        const double2 v = u[i];
        double Dj = a.rho * a.tau * (v.x * v.x + v.y * v.y);
        if (a.V) Dj += a.tau * a.V[i];
        a.D64[i] = Dj;
        a.D32[i] = (float)Dj;
    }
}

// Solve start: ||b||^2 (optionally writing the complex64 copy of b), then the
// last workgroup initialises the GMRES state.
__global__ __launch_bounds__(256) void k_prepare(StreamArgs a) {
    __shared__ double2 s_red[(kMaxRestart + 2) * kMaxWaves];
    __shared__ double2 s_tot[kMaxRestart + 2];
    const long long N = a.N;
    double nrm = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
        const double2 v = a.b64[i];
        nrm += v.x * v.x + v.y * v.y;
        if (a.r32) reinterpret_cast<float2*>(a.r32)[i] = make_float2((float)v.x, (float)v.y);
    }
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = dmk(nrm, 0.0);
    __syncthreads();
    block_partial_write(s_red, 1, a.partials, a.pstride);
    if (!last_block_reduce(a.partials, a.pstride, 1, a.st, s_tot)) return;
    if (threadIdx.x == 0) {
        GmresState* st = a.st;
        st->counter = 0;
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
    }
}

// w -= sum_{i<nv} coef_i V_i, then either the dot products conj(V_i) w
// (mode 0, second Gram-Schmidt round) or ||w||^2 and the Arnoldi finish
// (mode 1).  V_i and w are complex<R>; arithmetic in FP64.
template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_cgs(StreamArgs a) {
    using C = cplx<R>;
    __shared__ double2 s_red[(kMaxRestart + 2) * kMaxWaves];
    __shared__ double2 s_tot[kMaxRestart + 2];
    if (a.check_active && a.st->active == 0) return;
    const long long N = a.N;
    const int nv = a.nv;
    GmresState* st = a.st;
    C wreg[kEpt];
    long long idx[kEpt];
    const long long T = (long long)gridDim.x * blockDim.x;
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
#pragma unroll
    for (int q = 0; q < kEpt; ++q) {
        idx[q] = t0 + q * T;
        if (idx[q] < N) {
            const C w = ld<R>(a.w, idx[q]);
            double sx = w.x, sy = w.y;
            for (int i = 0; i < nv; ++i) {
                const C v = (i == 0) ? ld<R>(a.v0, idx[q]) : ld<R>(a.vbase, (long long)(i - 1) * N + idx[q]);
                const double2 c = st->coef[i];
                sx -= c.x * v.x - c.y * v.y;
                sy -= c.x * v.y + c.y * v.x;
            }
            const C wn = cm<R>(static_cast<R>(sx), static_cast<R>(sy));
            stc<R>(a.w, idx[q], wn);
            wreg[q] = wn;
            nrm += (double)wn.x * wn.x + (double)wn.y * wn.y;
        } else {
            wreg[q] = czero<C>();
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int nout;
    if (MODE == 0) {
        for (int i = 0; i < nv; ++i) {
            double sx = 0.0, sy = 0.0;
#pragma unroll
            for (int q = 0; q < kEpt; ++q) {
                if (idx[q] >= N) continue;
                const C v = (i == 0) ? ld<R>(a.v0, idx[q]) : ld<R>(a.vbase, (long long)(i - 1) * N + idx[q]);
                const C w = wreg[q];
                sx += (double)v.x * w.x + (double)v.y * w.y;
                sy += (double)v.x * w.y - (double)v.y * w.x;
            }
            sx = wave_sum(sx);
            sy = wave_sum(sy);
            if (lane == 0) s_red[i * kMaxWaves + wave] = dmk(sx, sy);
        }
        nout = nv;
    } else {
        nrm = wave_sum(nrm);
        if (lane == 0) s_red[wave] = dmk(nrm, 0.0);
        nout = 1;
    }
    __syncthreads();
    block_partial_write(s_red, nout, a.partials, a.pstride);
    if (!last_block_reduce(a.partials, a.pstride, nout, st, s_tot)) return;
    if (threadIdx.x == 0) {
        st->counter = 0;
        if (MODE == 0) {
            for (int i = 0; i < nv; ++i) {
                const double s = st->sigma[i];
                const double2 h = dmk(s_tot[i].x * s, s_tot[i].y * s);
                st->hcol[i].x += h.x;
                st->hcol[i].y += h.y;
                st->coef[i] = dmk(h.x * s, h.y * s);
            }
        } else {
            arnoldi_finish(st, a.hs, s_tot[0].x);
        }
    }
}

// Configure GMRES limits in the device state (single thread).
__global__ void k_config(GmresState* st, double tol, double outer_tol, int restart, int maxit, int fixed_iters,
                         int max_outer) {
    st->tol = tol;
    st->outer_tol = outer_tol;
    st->restart = restart;
    st->maxit = maxit;
    st->fixed_iters = fixed_iters;
    st->max_outer = max_outer;
    st->counter = 0;
    st->active = 0;
    st->done = 0;
}

// ---------------------------------------------------------------------------
// host-side launchers (declared in fnls_launch.h)
// ---------------------------------------------------------------------------
}  // namespace fnls

#include "fnls_launch.h"

namespace fnls {

template <typename R, int INM, int OPS, int ZM, int OUTM, int FIN>
static hipError_t launch_pass_t(const PassArgs& a, int blocks, size_t lds, hipStream_t s) {
    auto kern = k_pass<R, INM, OPS, ZM, OUTM, FIN>;
    // dynamic LDS above 64 KiB must be allowed per kernel; remember the largest granted
    static size_t granted = 64 * 1024;
    if (lds > granted) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        granted = lds;
    }
    (void)hipGetLastError();   // clear errors of earlier, unrelated runtime calls
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(a.G * a.L), lds, s, a);
    return hipGetLastError();
}

#define FNLS_PASS_CASE(R, INM, OPS, ZM, OUTM, FIN)                                            \
    if (v.inm == INM && v.ops == (OPS) && v.zm == ZM && v.outm == OUTM && v.fin == FIN)       \
        return launch_pass_t<R, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s);

template <typename R>
static hipError_t dispatch_pass(const PassVariant& v, const PassArgs& a, int blocks, size_t lds, hipStream_t s) {
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
    FNLS_PASS_CASE(R, IN_COMBO, DST, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, DDD, Z_NONE, OUT_LINE, FIN_WRITE)
    // last sine transform of the preconditioner (d >= 2)
    FNLS_PASS_CASE(R, IN_PLAIN, LASTDST, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, LASTDST, Z_XSET, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, LASTDST, Z_XADD, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, LASTDST_T, Z_WRITE, OUT_ACC_FIRST, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, LASTDST_T, Z_XADD, OUT_ACC_FIRST, FIN_WRITE)
    // d = 1: the whole preconditioned operator on one line
    FNLS_PASS_CASE(R, IN_PLAIN, FULL1, Z_NONE, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_BASIS, FULL1_T, Z_NONE, OUT_ACC_FIRST, FIN_WDOTS)
    FNLS_PASS_CASE(R, IN_COMBO, FULL1_T, Z_XADD, OUT_ACC_FIRST, FIN_RESID)
    FNLS_PASS_CASE(R, IN_COMBO, FULL1, Z_XADD, OUT_LINE, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_COMBO, FULL1, Z_XSET, OUT_LINE, FIN_WRITE)
    // Toeplitz passes
    FNLS_PASS_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_FIRST, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_FIRST, FIN_RESID)
    FNLS_PASS_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_NEXT, FIN_WRITE)
    FNLS_PASS_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_NEXT, FIN_WDOTS)
    FNLS_PASS_CASE(R, IN_PLAIN, TOEP, Z_NONE, OUT_ACC_NEXT, FIN_RESID)
    return hipErrorInvalidValue;
}

hipError_t launch_pass(int fp64, const PassVariant& v, const PassArgs& a, int blocks, size_t lds, hipStream_t s) {
    return fp64 ? dispatch_pass<double>(v, a, blocks, lds, s) : dispatch_pass<float>(v, a, blocks, lds, s);
}

hipError_t launch_precond_setup(const StreamArgs& a, int blocks, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_precond_setup, dim3(blocks), dim3(kStreamThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_prepare(const StreamArgs& a, int blocks, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(kStreamThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cgs(int fp64, int mode, const StreamArgs& a, int blocks, hipStream_t s) {
    (void)hipGetLastError();
    if (fp64) {
        if (mode == 0) hipLaunchKernelGGL((k_cgs<double, 0>), dim3(blocks), dim3(kStreamThreads), 0, s, a);
        else hipLaunchKernelGGL((k_cgs<double, 1>), dim3(blocks), dim3(kStreamThreads), 0, s, a);
    } else {
        if (mode == 0) hipLaunchKernelGGL((k_cgs<float, 0>), dim3(blocks), dim3(kStreamThreads), 0, s, a);
        else hipLaunchKernelGGL((k_cgs<float, 1>), dim3(blocks), dim3(kStreamThreads), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_config(GmresState* st, double tol, double outer_tol, int restart, int maxit, int fixed_iters,
                         int max_outer, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_config, dim3(1), dim3(1), 0, s, st, tol, outer_tol, restart, maxit, fixed_iters, max_outer);
    return hipGetLastError();
}

}  // namespace fnls
