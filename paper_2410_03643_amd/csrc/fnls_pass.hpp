// The fused axis-pass kernel of libfnls (see fnls_kernels.hip for the
// overview) and its launchers, instantiated once per precision by
// fnls_pass64.hip and fnls_pass32.hip.
#pragma once

#include <algorithm>

#include "fnls_kernels_core.hpp"

namespace fnls {

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
// Preconditioner diagonal: v / (omega + i mu_k), mu_k = lo + tscale lambda_k
// (lo: the other axes' share for this line) = v (omega - i mu_k) / den, with
// one division per unknown.
template <typename R>
struct DivPost {
    R om, lo, tscale;
    const R* lam;
    __device__ __forceinline__ cplx<R> operator()(int k, cplx<R> v) const {
        const R mu = lo + tscale * lam[k];
        const R rden = R(1) / (om * om + mu * mu);
        return cm<R>((v.x * om + v.y * mu) * rden, (v.y * om - v.x * mu) * rden);
    }
};

template <typename R, int RMAX, int LGM, int INM, int OPS, int ZM, int OUTM, int FIN, bool BJ = false>
__device__ __forceinline__ void pass_body(const PassArgs& a, int blk_in) {
    using C = cplx<R>;
    constexpr int kMaxEptLine = RMAX;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (launch_skipped(a.check_active, a.guard_k, a.st)) return;
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

    // compile-time plans with at most one wavefront per line synchronise the
    // line transforms within the wavefront
    constexpr bool kWS = LGM > 0 && ((1 << LGM) / RMAX) <= 64;
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

    // Coalescing element map: element q < kMaxEptLine of this thread is
    // e = tid + q T of the workgroup's L n unknowns.  Rows of the contiguous
    // axis lie back to back (e = l n + j, global index blk L n + e); lines of
    // strided axes are interleaved (e = j L + l), and since T is a multiple
    // of L the thread keeps one line l = tid mod L while j advances by
    // T / L = G per element.  Both give the global index and the LDS slot
    // without a 64-bit multiply or an LDS read per element.  Each phase forms
    // its context (the line's base offset, read from LDS) anew, so that no
    // 64-bit index stays live in registers across the transforms.
    struct Elem {
        long long gi;   // global index (meaningful when valid)
        int j;          // unknown along the line
        int slot;       // LDS slot l LS + j + 1
        bool in;        // e < L n
        bool valid;     // in, and the line exists
    };
    struct ElemCtx {
        int t;          // the thread index, opaque to the compiler (below)
        long long gi0;  // strided: global index of element 0; contiguous: blk L n
        bool ok;        // strided: the thread's line exists
    };
    auto elem_ctx = [&]() {
        ElemCtx c;
        // an opaque copy of the thread index per phase: the indices of one
        // phase are not merged with the same expressions of an earlier phase,
        // which would keep them live in registers across the transforms
        c.t = tid;
        asm volatile("" : "+v"(c.t));
        if (contiguous) {
            c.gi0 = (long long)blk * L * n;
            c.ok = true;
        } else {
            const long long b = s_base[c.t & (L - 1)];
            c.gi0 = b + (long long)(c.t >> lgL) * stride;
            c.ok = b >= 0;
        }
        return c;
    };
    // the same context before the per-line set-up: the thread forms its
    // line's base offset itself (32-bit: lines and strides stay below 2^32)
    auto elem_ctx_direct = [&]() {
        ElemCtx c;
        c.t = tid;
        asm volatile("" : "+v"(c.t));
        if (contiguous) {
            c.gi0 = (long long)blk * L * n;
            c.ok = true;
        } else {
            const unsigned lg = (unsigned)blk * (unsigned)L + (unsigned)(c.t & (L - 1));
            const unsigned st = (unsigned)stride;
            const unsigned o = lg / st;
            const unsigned i = lg - o * st;
            c.ok = (long long)lg < a.nlines;
            c.gi0 = (long long)o * n * stride + i + (long long)(c.t >> lgL) * stride;
        }
        return c;
    };
    auto elem = [&](const ElemCtx& c, int q) {
        Elem r;
        const int e = c.t + q * T;
        r.in = e < E;
        if (contiguous) {
            const int l = (n == 1) ? e : (int)__umulhi((unsigned)e, a.magic_n);
            r.j = e - l * n;
            r.slot = l * LS + r.j + 1;
            r.gi = c.gi0 + e;
            r.valid = r.in && r.gi < (long long)a.nlines * n;
        } else {
            r.j = (c.t >> lgL) + q * G;
            r.slot = (c.t & (L - 1)) * LS + r.j + 1;
            r.gi = c.gi0 + q * ((long long)G * stride);
            r.valid = r.in && c.ok;
        }
        return r;
    };

    // IN_CGS: totals of the second-round dot products d_i (every workgroup,
    // in the same fixed order), h_i = sigma_i d_i and the update coefficients
    // h_i sigma_i (basis vector i is stored as v_i / sigma_i); workgroup 0
    // completes the Hessenberg column.  The line buffers serve as reduction
    // scratch before the per-line set-up below overwrites them.
    constexpr bool kCgs = (INM == IN_CGS);
    __shared__ double2 s_cgs[kCgs ? 2 * (kMaxRestart + 2) : 1];
    __shared__ double s_wn[kCgs ? 16 : 1];
    // FP64 IN_CGS: w and the first basis vector are read before the totals
    // are reduced (a barrier does not wait for global loads, so they are in
    // flight during the reduction), with the element map formed before the
    // per-line set-up.
    constexpr bool kCgs64 = kCgs && sizeof(R) == 8;
    constexpr int kCq = kCgs64 ? kMaxEptLine : 1;
    long long cg_gq[kCq];
    double cg_wx[kCq], cg_wy[kCq];
    C cg_ta[kCq], cg_tb[kCq];
    auto cg_load_vec = [&](int i, C* t) {
        const C* src = (i == 0) ? reinterpret_cast<const C*>(a.v0)
                                : reinterpret_cast<const C*>(a.vbase) + (long long)(i - 1) * a.N;
#pragma unroll
        for (int q = 0; q < kCq; ++q) t[q] = cg_gq[q] >= 0 ? src[cg_gq[q]] : czero<C>();
    };
    if constexpr (kCgs64) {
        const ElemCtx ec = elem_ctx_direct();
#pragma unroll
        for (int q = 0; q < kCq; ++q) {
            const Elem el = elem(ec, q);
            cg_gq[q] = el.valid ? el.gi : -1;
            cg_wx[q] = 0.0;
            cg_wy[q] = 0.0;
            if (el.valid) {
                const C wv = ld<R>(in_p, el.gi);
                cg_wx[q] = wv.x;
                cg_wy[q] = wv.y;
            }
        }
        cg_load_vec(0, cg_ta);
    }
    if constexpr (kCgs) {
        const int nv = basis_j + 1;
        double2* s_tot = s_cgs;
        double2* s_coef = s_cgs + (kMaxRestart + 2);
        reduce_partials(a.cgs_pin, a.cgs_stride, a.cgs_nb, nv, s_tot, reinterpret_cast<double2*>(smem_raw));
        if (tid < nv) {
            const double sg = a.st->sigma[tid];
            const double2 h = dmk(s_tot[tid].x * sg, s_tot[tid].y * sg);
            s_coef[tid] = dmk(h.x * sg, h.y * sg);
            if (blk == 0) {
                a.st->hcol[tid].x += h.x;
                a.st->hcol[tid].y += h.y;
            }
        }
        __syncthreads();
    }

    // IN_PLAIN / IN_BASIS: the line data's loads are issued before the
    // per-line set-up (whose global reads and barrier they then overlap);
    // complex64 also issues the accumulator's loads here
    constexpr bool kAccEarly = (OPS & OP_TOEP) != 0 && OUTM == OUT_ACC_NEXT;
    static_assert(!(kCgs && kAccEarly), "the fused Gram-Schmidt load phase reads no accumulator");
    constexpr bool kInEarly = (INM == IN_PLAIN || INM == IN_BASIS);
    // (FP64: the accumulator's loads are issued behind the line data's LDS
    // writes, and complete during the transforms; complex64 measured faster
    // with both issued together)
    constexpr bool kAccLate = sizeof(R) == 8;
    C vin[kInEarly ? kMaxEptLine : 1];
    C accq[kAccEarly ? kMaxEptLine : 1];
    if constexpr (kInEarly) {
        const ElemCtx ec = elem_ctx_direct();
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const Elem el = elem(ec, q);
            vin[q] = czero<C>();
            if constexpr (kAccEarly && !kAccLate) accq[q] = czero<C>();
            if (el.valid) {
                if constexpr (kAccEarly && !kAccLate) accq[q] = ld<R>(a.acc_in, el.gi);
                vin[q] = ld<R>(in_p, el.gi);
            }
        }
    }

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
    double wnrm = 0.0;   // IN_CGS: this thread's part of ||w||^2
    // the accumulator of the other axes' Toeplitz products is loaded in the
    // load phase, so its loads are in flight during the transforms
    {
        double sig = 1.0;
        if (INM == IN_BASIS) sig = a.st->sigma[basis_j];
        int nvc = 0;
        if (INM == IN_COMBO) nvc = a.st->k;
        const ElemCtx ec = elem_ctx();
        if constexpr (INM == IN_PLAIN || INM == IN_BASIS) {
            // every global load of the phase was issued before the first
            // LDS write (a write waits for its value, and would otherwise hold
            // back the next element's loads: one memory round trip each)
#pragma unroll
            for (int q = 0; q < kMaxEptLine; ++q) {
                const Elem el = elem(ec, q);
                if (el.in) {
                    C v = vin[q];
                    if (INM == IN_BASIS && el.valid) v = cm<R>(static_cast<R>(v.x * sig), static_cast<R>(v.y * sig));
                    lds[el.slot] = v;
                }
            }
            if constexpr (kAccEarly && kAccLate) {
#pragma unroll
                for (int q = 0; q < kMaxEptLine; ++q) {
                    const Elem el = elem(ec, q);
                    accq[q] = el.valid ? ld<R>(a.acc_in, el.gi) : czero<C>();
                }
            }
        } else if constexpr (kCgs && sizeof(R) == 8) {
            // w -= sum_i c_i v_i as explicit fused multiply-adds in the order
            // of the streaming update (same rounding).  The basis vectors are
            // the outer loop, so each of them is read for all of the thread's
            // elements at once, and the next one is in flight while the
            // current one is applied (measured faster for FP64 only; complex64
            // bases take the per-element loop below).
            const double2* s_coef = s_cgs + (kMaxRestart + 2);
            auto apply_vec = [&](int i, const C* t) {
                const double2 c = s_coef[i];
#pragma unroll
                for (int q = 0; q < kMaxEptLine; ++q) cmsub(cg_wx[q], cg_wy[q], c, t[q].x, t[q].y);
            };
            for (int i = 0; i <= basis_j; i += 2) {
                if (i + 1 <= basis_j) cg_load_vec(i + 1, cg_tb);
                apply_vec(i, cg_ta);
                if (i + 1 <= basis_j) {
                    if (i + 2 <= basis_j) cg_load_vec(i + 2, cg_ta);
                    apply_vec(i + 1, cg_tb);
                }
            }
#pragma unroll
            for (int q = 0; q < kMaxEptLine; ++q) {
                const Elem el = elem(ec, q);
                if (el.in) {
                    C v = czero<C>();
                    if (el.valid) {
                        v = cm<R>(static_cast<R>(cg_wx[q]), static_cast<R>(cg_wy[q]));
                        stc<R>(const_cast<void*>(in_p), el.gi, v);
                        wnrm = fma((double)v.x, (double)v.x, wnrm);
                        wnrm = fma((double)v.y, (double)v.y, wnrm);
                    }
                    lds[el.slot] = v;
                }
            }
        } else if constexpr (INM == IN_COMBO && !kAccEarly) {
            // sum_k c_k t_k over the k stored vectors (the preconditioned
            // basis z_k, complex64 when z32, with the coefficients y; else the
            // basis v_k with coef), accumulated in FP64.  The vectors are the
            // outer loop, so each is read for all of the thread's elements at
            // once, and the next one is in flight while the current one is
            // added.
            long long gq[kMaxEptLine];
            double sx[kMaxEptLine], sy[kMaxEptLine];
#pragma unroll
            for (int q = 0; q < kMaxEptLine; ++q) {
                const Elem el = elem(ec, q);
                gq[q] = el.valid ? el.gi : -1;
                sx[q] = 0.0;
                sy[q] = 0.0;
            }
            const bool zs = a.zsum != 0, z32 = a.z32 != 0;
            auto load_vec = [&](int i, double2* t) {
#pragma unroll
                for (int q = 0; q < kMaxEptLine; ++q) {
                    double2 v = dmk(0.0, 0.0);
                    if (gq[q] >= 0) {
                        if (zs) {
                            const long long zi = (long long)i * a.N + gq[q];
                            if (z32) {
                                const float2 f = reinterpret_cast<const float2*>(a.vbase)[zi];
                                v = dmk(f.x, f.y);
                            } else {
                                v = reinterpret_cast<const double2*>(a.vbase)[zi];
                            }
                        } else {
                            const C u = (i == 0) ? ld<R>(a.v0, gq[q]) : ld<R>(a.vbase, (long long)(i - 1) * a.N + gq[q]);
                            v = dmk(u.x, u.y);
                        }
                    }
                    t[q] = v;
                }
            };
            auto add_vec = [&](int i, const double2* t) {
                const double2 c = zs ? a.st->y[i] : a.st->coef[i];
#pragma unroll
                for (int q = 0; q < kMaxEptLine; ++q) {
                    sx[q] += c.x * t[q].x - c.y * t[q].y;
                    sy[q] += c.x * t[q].y + c.y * t[q].x;
                }
            };
            double2 ta[kMaxEptLine], tb[kMaxEptLine];
            if (nvc > 0) load_vec(0, ta);
            for (int i = 0; i < nvc; i += 2) {
                if (i + 1 < nvc) load_vec(i + 1, tb);
                add_vec(i, ta);
                if (i + 1 < nvc) {
                    if (i + 2 < nvc) load_vec(i + 2, ta);
                    add_vec(i + 1, tb);
                }
            }
#pragma unroll
            for (int q = 0; q < kMaxEptLine; ++q) {
                const Elem el = elem(ec, q);
                if (el.in) lds[el.slot] = el.valid ? cm<R>(static_cast<R>(sx[q]), static_cast<R>(sy[q])) : czero<C>();
            }
        } else {
#pragma unroll
            for (int q = 0; q < kMaxEptLine; ++q) {
                const Elem el = elem(ec, q);
                if constexpr (kAccEarly) accq[q] = czero<C>();
                if (el.in) {
                    C v = czero<C>();
                    if (el.valid) {
                        const long long gi = el.gi;
                        if constexpr (kAccEarly) accq[q] = ld<R>(a.acc_in, gi);
                        if constexpr (kCgs) {
                            // the same update and rounding, one element at a time
                            const C wv = ld<R>(in_p, gi);
                            double wx = wv.x, wy = wv.y;
                            const double2* s_coef = s_cgs + (kMaxRestart + 2);
                            for (int i = 0; i <= basis_j; ++i) {
                                const C t = (i == 0) ? ld<R>(a.v0, gi) : ld<R>(a.vbase, (long long)(i - 1) * a.N + gi);
                                cmsub(wx, wy, s_coef[i], t.x, t.y);
                            }
                            v = cm<R>(static_cast<R>(wx), static_cast<R>(wy));
                            stc<R>(const_cast<void*>(in_p), gi, v);
                            wnrm = fma((double)v.x, (double)v.x, wnrm);
                            wnrm = fma((double)v.y, (double)v.y, wnrm);
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
                    lds[el.slot] = v;
                }
            }
        }
    }
    if constexpr (kCgs) {
        // wavefront sums of ||w||^2 (the barrier below orders them before
        // thread 0 adds them in wavefront order)
        wnrm = wave_sum(wnrm);
        if ((tid & 63) == 0) s_wn[tid >> 6] = wnrm;
    }
    __syncthreads();
    if constexpr (kCgs) {
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < (T >> 6); ++w) sum += s_wn[w];
            a.pout[blk] = dmk(sum, 0.0);
        }
    }

    C* A = lds + (size_t)line * LS;
    C* B = kTwoBuf ? A + PA : A;   // B exists only for the Toeplitz product

    // ---- transform stages (line-local: with WS, G <= 64 threads per line,
    // each wavefront transforms its own lines without workgroup barriers)
    if constexpr ((OPS & OP_DIV) != 0) {
        // the division by (omega + i mu_k) is applied to the first transform's
        // outputs before they are stored
        static_assert((OPS & OP_DST1) && (OPS & OP_DST2), "division between two sine transforms");
        const DivPost<R> div{static_cast<R>(a.omega), s_lamo[line], tscale, lam};
        line_dst<R, RMAX, LGM, decltype(ltw), kWS>(A, B, lgm, lt, G, tw, twl, ltw, div);
    } else if (OPS & OP_DST1) {
        line_dst<R, RMAX, LGM, decltype(ltw), kWS>(A, B, lgm, lt, G, tw, twl, ltw);
    }
    if (OPS & OP_DST2) line_dst<R, RMAX, LGM, decltype(ltw), kWS>(A, B, lgm, lt, G, tw, twl, ltw);
    // the element phases read every line of the workgroup
    if constexpr (kWS && (OPS & (OP_DST1 | OP_DIV | OP_DST2)) != 0) __syncthreads();

    constexpr bool kToep = (OPS & OP_TOEP) != 0;
    constexpr bool kKeepZ = kToep && (OUTM == OUT_ACC_FIRST);
    constexpr bool kPhase1 = (OPS & OP_SCALE) || (ZM != Z_NONE) || (OUTM == OUT_ACC_FIRST) || !kToep;
    C zreg[kKeepZ ? kMaxEptLine : 1];
    C oreg[FIN == FIN_WDOTS ? kMaxEptLine : 1];
    double nrm = 0.0;

    // ---- element phase 1: preconditioner scale, z / x outputs, Toeplitz operand
    if (kPhase1) {
        const double om = a.omega;
        const ElemCtx ec = elem_ctx();
        // every global operand of this phase is loaded before the first
        // global store (a store could alias a later load, which would
        // serialise one memory round trip per element)
        constexpr bool kNeedD = (OPS & OP_SCALE) != 0;
        constexpr bool kNeedX = (ZM == Z_XADD);
        R dpre[kNeedD ? kMaxEptLine : 1];
        double2 xpre[kNeedX ? kMaxEptLine : 1];
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const Elem el = elem(ec, q);
            if (kNeedD) dpre[q] = R(0);
            if (kNeedX) xpre[q] = dmk(0.0, 0.0);
            if (!el.valid) continue;
            if (kNeedD) dpre[q] = Dv[el.gi];
            if (kNeedX && !a.first_cycle) xpre[q] = a.x64[el.gi];
        }
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const Elem el = elem(ec, q);
            if (!el.in) continue;
            C z = lds[el.slot];
            if (el.valid) {
                const long long gi = el.gi;
                if (OPS & OP_SCALE) {
                    const R Dj = dpre[kNeedD ? q : 0];
                    // -2 i om / ((om+1) - i D) = (2 om D - 2 i om (om+1)) / ((om+1)^2 + D^2),
                    // one reciprocal per unknown
                    const R op1 = static_cast<R>(om + 1.0);
                    const R rden = R(1) / (op1 * op1 + Dj * Dj);
                    const R fr = static_cast<R>(2.0 * om) * Dj * rden;
                    const R fi = -static_cast<R>(2.0 * om) * op1 * rden;
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
            if (kToep) lds[el.slot] = z;
        }
        if (kToep) __syncthreads();
    }

    // ---- Toeplitz product and element phase 2
    if (kToep) {
        line_toeplitz<R, RMAX, LGM, decltype(ltw), kWS>(A, B, lgm, lt, G, tw, twl,
                                                         reinterpret_cast<const R*>(a.sym_e),
                                                         reinterpret_cast<const R*>(a.sym_o), tscale, ltw);
        if constexpr (kWS) __syncthreads();   // element phase 2 reads every line
        const R cT = static_cast<R>(a.cT);
        const ElemCtx ec = elem_ctx();
        // operands first (see element phase 1)
        constexpr bool kFirst = (OUTM == OUT_ACC_FIRST);
        constexpr bool kResid = (FIN == FIN_RESID);
        R dq[kFirst ? kMaxEptLine : 1];
        double2 bq[kResid ? kMaxEptLine : 1];
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const Elem el = elem(ec, q);
            if (kFirst) dq[q] = R(0);
            if (kResid) bq[q] = dmk(0.0, 0.0);
            if (!el.valid) continue;
            if (kFirst) dq[q] = Dv[el.gi];
            if (kResid) bq[q] = a.b64[el.gi];
        }
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const Elem el = elem(ec, q);
            if (FIN == FIN_WDOTS) oreg[q] = czero<C>();
            if (!el.valid) continue;
            const long long gi = el.gi;
            const int s = el.j + 1;
            const C tz = cadd(lds[el.slot], cmulc(lds[el.slot + PA], tw[s]));
            C o;
            if (OUTM == OUT_ACC_FIRST) {
                const R Dj = dq[kFirst ? q : 0];
                const R cD = static_cast<R>(a.cD) * Dj, ci = static_cast<R>(a.ci);
                const C z = zreg[kKeepZ ? q : 0];
                o = cm<R>(cD * z.x - ci * z.y + cT * tz.x, cD * z.y + ci * z.x + cT * tz.y);
            } else {
                const C acc = accq[kAccEarly ? q : 0];
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
        const ElemCtx ec = elem_ctx();
#pragma unroll
        for (int q = 0; q < kMaxEptLine; ++q) {
            const Elem el = elem(ec, q);
            gq[q] = el.valid ? el.gi : -1;
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
    // compile-time plans for m = 1024, 512 and 256 (d = 2, n = 1023 and 511;
    // d = 3, n = 255); those with G = m / rmax <= 64 threads per line
    // transform each line within one wavefront (no workgroup barriers)
    if (a.lgm == 10) {
        if (rmax == 4) return launch_pass_t<R, 4, 10, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
        if (rmax == 8) return launch_pass_t<R, 8, 10, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
        if (rmax == 16) return launch_pass_t<R, 16, 10, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
    }
    if (a.lgm == 9 && rmax == 4) return launch_pass_t<R, 4, 9, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
    if (a.lgm == 9 && rmax == 8) return launch_pass_t<R, 8, 9, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
    if (a.lgm == 8 && rmax == 4) return launch_pass_t<R, 4, 8, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
    if (a.lgm == 8 && rmax == 8) return launch_pass_t<R, 8, 8, INM, OPS, ZM, OUTM, FIN>(a, blocks, lds, s, te);
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
hipError_t dispatch_pass(const PassVariant& v, const PassArgs& a, int blocks, size_t lds, hipStream_t s,
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
    FNLS_PASS_CASE(R, IN_BASIS, LASTDST_T, Z_WRITE, OUT_ACC_FIRST, FIN_WRITE)
    // second Gram-Schmidt update fused with the next step's first sine transform
    FNLS_PASS_CASE(R, IN_CGS, DST, Z_NONE, OUT_LINE, FIN_WRITE)
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

// ---- batched launches: radix 4 (or 8 for the compile-time line lengths),
// G * L threads per workgroup; line length 2^LGM for every instance of the
// launch, or generic with LGM = 0 (radix 4) ----
template <typename R, int RMAX, int LGM, int INM, int OPS, int ZM, int OUTM, int FIN>
static hipError_t launch_pass_batch_l(const PassArgs* args, const int* offs, int count, int blocks, size_t lds,
                                      int threads, hipStream_t s) {
    auto kern = k_pass_batch<R, RMAX, LGM, INM, OPS, ZM, OUTM, FIN>;
    static size_t granted = 64 * 1024;
    if (lds > granted) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        granted = lds;
    }
    if (!args) return hipSuccess;   // attribute only (before a graph capture)
    if (threads > PassThreads<RMAX>::v || threads % 64 != 0) return hipErrorInvalidConfiguration;
    return launch_k(kern, dim3(blocks), dim3(threads), lds, s, nullptr, args, offs, count);
}

template <typename R, int INM, int OPS, int ZM, int OUTM, int FIN>
static hipError_t launch_pass_batch_t(int lgm, int rmax, const PassArgs* args, const int* offs, int count,
                                      int blocks, size_t lds, int threads, hipStream_t s) {
    if (rmax == 8) {
        switch (lgm) {
            case 10: return launch_pass_batch_l<R, 8, 10, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
            case 9: return launch_pass_batch_l<R, 8, 9, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
            case 8: return launch_pass_batch_l<R, 8, 8, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (rmax != 4) return hipErrorInvalidValue;
    switch (lgm) {
        case 10: return launch_pass_batch_l<R, 4, 10, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
        case 9: return launch_pass_batch_l<R, 4, 9, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
        case 8: return launch_pass_batch_l<R, 4, 8, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
        default: return launch_pass_batch_l<R, 4, 0, INM, OPS, ZM, OUTM, FIN>(args, offs, count, blocks, lds, threads, s);
    }
}

#define FNLS_BATCH_CASE(R, INM, OPS, ZM, OUTM, FIN)                                             \
    if (v.inm == INM && v.ops == (OPS) && v.zm == ZM && v.outm == OUTM && v.fin == FIN)         \
        return launch_pass_batch_t<R, INM, OPS, ZM, OUTM, FIN>(lgm, v.rmax, args, offs, count, blocks, lds, threads, s);

template <typename R>
hipError_t dispatch_pass_batch(const PassVariant& v, int lgm, const PassArgs* args, const int* offs,
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

}  // namespace fnls
