// Device building blocks of libfnls (gfx950): complex arithmetic, in-register
// DFTs, a Stockham radix-16/8/4/2 line FFT in LDS, and the two line operators
// of the method -- the orthonormal DST-I (sine transform S of Sec. 4) and the
// symmetric Toeplitz product T_1 x (Sec. 2.1) -- both on length m = n + 1
// complex FFTs.
//
// DST-I of length n = m - 1 (y_k = sqrt(2/m) sum_j x_j sin(pi j k / m)):
// with x_0 = x_m = 0, a_j = x_j - x_{m-j}, b_j = (x_j + x_{m-j}) W_{2m}^j
// (W_L = exp(-2 pi i / L)), the odd extension's length-2m DFT Z satisfies
// Z_{2p} = FFT_m(a)_p and Z_{2p+1} = FFT_m(b)_p, and y_k = (i / sqrt(2m)) Z_k.
//
// Toeplitz product: T_1 is the leading n x n block of the symmetric circulant
// of length 2m whose first column is mu c_|k| (zero at k = n, n+1, n+2); its
// eigenvalues are s_q, q < 2m (s_q = lambda_q, the tau eigenvalues, for
// 1 <= q <= n).  Splitting the length-2m transform of the zero-padded line into
// even and odd frequencies gives
//   T_1 x = 1/2 [ IFFT_m(s_even . FFT_m(x)) + W_{2m}^{-j} IFFT_m(s_odd . FFT_m(W_{2m}^j x)) ],
// two length-m convolutions (the 1/(2m) is folded into s_even, s_odd).
//
// Line layout in LDS: slot s in [0, m) holds unknown s (1-based), slot 0 is
// the Dirichlet zero.  Each line owns two buffers A and B of m (+1 pad)
// complex values; G threads of the workgroup work on one line.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

namespace fnls {

template <typename R> struct CT;
template <> struct CT<double> { using C = double2; };
template <> struct CT<float> { using C = float2; };
template <typename R> using cplx = typename CT<R>::C;

template <typename R> __device__ __forceinline__ cplx<R> cm(R a, R b) {
    cplx<R> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
    C r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.y * b.x - a.x * b.y;
    return r;
}
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }
template <typename C> __device__ __forceinline__ C cneg(C a) { C r; r.x = -a.x; r.y = -a.y; return r; }
template <typename C> __device__ __forceinline__ C czero() { C r; r.x = 0; r.y = 0; return r; }

template <typename To, typename From> __device__ __forceinline__ cplx<To> ccast(From a) {
    return cm<To>(static_cast<To>(a.x), static_cast<To>(a.y));
}

// multiply by -i (forward transform) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C rot90(C a) {
    C r;
    if (INV) { r.x = -a.y; r.y = a.x; }
    else     { r.x = a.y;  r.y = -a.x; }
    return r;
}

// cos / sin of 2 pi j / 16
__host__ __device__ constexpr double kc16(int j) {
    switch (j & 15) {
        case 0: return 1.0;
        case 1: return 0.92387953251128675613;
        case 2: return 0.70710678118654752440;
        case 3: return 0.38268343236508977173;
        case 4: return 0.0;
        case 5: return -0.38268343236508977173;
        case 6: return -0.70710678118654752440;
        case 7: return -0.92387953251128675613;
        case 8: return -1.0;
        case 9: return -0.92387953251128675613;
        case 10: return -0.70710678118654752440;
        case 11: return -0.38268343236508977173;
        case 12: return 0.0;
        case 13: return 0.38268343236508977173;
        case 14: return 0.70710678118654752440;
        default: return 0.92387953251128675613;
    }
}
__host__ __device__ constexpr double ks16(int j) { return kc16(j - 4); }

// a * W_16^J (forward W = exp(-2 pi i / 16); inverse uses the conjugate)
template <int J, bool INV, typename C> __device__ __forceinline__ C tw16(C a) {
    constexpr int j = J & 15;
    if constexpr (j == 0) {
        return a;
    } else if constexpr (j == 4) {
        return rot90<INV>(a);
    } else if constexpr (j == 8) {
        return cneg(a);
    } else if constexpr (j == 12) {
        return rot90<!INV>(a);
    } else {
        using R = decltype(a.x);
        const R c = static_cast<R>(kc16(j));
        const R s = INV ? static_cast<R>(ks16(j)) : static_cast<R>(-ks16(j));
        C r;
        r.x = a.x * c - a.y * s;
        r.y = a.x * s + a.y * c;
        return r;
    }
}

template <bool INV, typename C> __device__ __forceinline__ void dft2(C& a, C& b) {
    C t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <bool INV, typename C> __device__ __forceinline__ void dft4(C& v0, C& v1, C& v2, C& v3) {
    C t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = rot90<INV>(csub(v1, v3));
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, t3);
    v3 = csub(t1, t3);
}

// In-register DFT of length RAD in natural order.
template <int RAD, bool INV, typename C> __device__ __forceinline__ void dft(C* v) {
    if constexpr (RAD == 2) {
        dft2<INV>(v[0], v[1]);
    } else if constexpr (RAD == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3]);
    } else if constexpr (RAD == 8) {
        // n = 4 n1 + n2, k = k1 + 2 k2
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) dft2<INV>(v[n2], v[4 + n2]);
        v[5] = tw16<2, INV>(v[5]);
        v[6] = tw16<4, INV>(v[6]);
        v[7] = tw16<6, INV>(v[7]);
        dft4<INV>(v[0], v[1], v[2], v[3]);
        dft4<INV>(v[4], v[5], v[6], v[7]);
        C t[8];
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            t[2 * k2] = v[k2];
            t[2 * k2 + 1] = v[4 + k2];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = t[i];
    } else {
        static_assert(RAD == 16, "radix");
        // n = 4 n1 + n2, k = k1 + 4 k2; Y[n2][k1] kept at v[4 k1 + n2]
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
        v[5] = tw16<1, INV>(v[5]);
        v[6] = tw16<2, INV>(v[6]);
        v[7] = tw16<3, INV>(v[7]);
        v[9] = tw16<2, INV>(v[9]);
        v[10] = tw16<4, INV>(v[10]);
        v[11] = tw16<6, INV>(v[11]);
        v[13] = tw16<3, INV>(v[13]);
        v[14] = tw16<6, INV>(v[14]);
        v[15] = tw16<9, INV>(v[15]);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
        C t[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = t[i];
    }
}

// LDS layout of a line: slot s in natural order, no padding.  gfx950's LDS
// (measured with its bank-conflict counter): a 64-lane ds_read_b128 is
// served in four cycles of 16 lanes (lanes sharing bit 5 and the parity of
// bits 2..4 of the lane index) from 64 banks of 4 bytes, ds_read_b64 in two
// cycles of 32 lanes (bit 5); ds_write_b128 in eight cycles of 8 consecutive
// lanes and ds_write_b64 in four cycles of 16 from 32 banks.  A cycle is free
// of conflicts when its lanes touch distinct slots of one bank row, so
// contiguous runs of slots (any offset) are free for reads and writes.  The
// strided stores of the early radix-4 stages and of the sine-transform output
// are made free by rotating, per lane, the order in which a thread writes its
// four outputs (out_rot); the stride-2 reads of the sine-transform scan by
// rotating its two reads (scan_rot).  For interleaved lines of strided axes
// the host chooses the line stride so that the element writes are free.
// Quarter twiddle table slot of W_m^q: the low two bits of q are XORed with
// bits 4..5 (16-byte values) or 5..6 (8-byte values), so that reads at
// stride 4 (q = 4 k) as well as consecutive reads fall into distinct banks.
template <typename R>
__device__ __forceinline__ int tw_slot(int q) { return q ^ ((q >> (sizeof(R) == 8 ? 4 : 5)) & 3); }

template <typename R>
__device__ __forceinline__ int out_rot() {
    const int lane = threadIdx.x & 63;
    return sizeof(R) == 8 ? (((lane >> 2) & 1) | (((lane >> 1) & 1) << 1))    // 16-byte values
                          : (((lane >> 2) & 1) | (((lane >> 3) & 1) << 1));   // 8-byte values
}
// Radix-8 stage (Ns = 1) stores: three lane bits select the output order.
template <typename R>
__device__ __forceinline__ int out_rot8() {
    const int lane = threadIdx.x & 63;
    return sizeof(R) == 8 ? (lane & 7) : ((lane >> 1) & 7);
}
template <typename R>
__device__ __forceinline__ int scan_rot() {
    const int lane = threadIdx.x & 63;
    return sizeof(R) == 8 ? ((lane >> 3) & 1) : ((lane >> 4) & 1);
}

// Radix-4 stages with Ns < 16 store output r of a butterfly at position
// (r + s) mod 4 of its four slots, s = out_rot() (a cyclic lane rotation:
// over each write cycle it covers the same slot positions as r ^ s, so the
// strided stores stay free of bank conflicts).  Output register i holds
// y_{(i + s) mod 4} when input q of the butterfly is multiplied by
// W_4^{q s} (inverse: W_4^{-q s}) beforehand: y_{r+s} = sum_q W_4^{r q}
// (W_4^{q s} x_q).  Those factors are powers of i, applied exactly by
// swapping and negating parts (rot_inputs), or folded into the stage's
// twiddle W^k -> W^k W_4^s, whose powers W^{q k} W_4^{q s} carry them; no
// register permutation (selects on every value) is needed.
template <typename R> __device__ __forceinline__ R xor_sign(R x, unsigned m);
template <> __device__ __forceinline__ double xor_sign<double>(double x, unsigned m) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x)) ^
                                 (static_cast<unsigned long long>(m) << 32);
    return __longlong_as_double(static_cast<long long>(b));
}
template <> __device__ __forceinline__ float xor_sign<float>(float x, unsigned m) {
    return __int_as_float(__float_as_int(x) ^ static_cast<int>(m));
}
// v i^e (e mod 4): (x, y), (-y, x), (-x, -y), (y, -x)
template <typename R>
__device__ __forceinline__ cplx<R> mul_ipow(cplx<R> v, int e) {
    const bool odd = (e & 1) != 0;
    const unsigned mre = ((e + 1) & 2) ? 0x80000000u : 0u;
    const unsigned mim = (e & 2) ? 0x80000000u : 0u;
    const R a = odd ? v.y : v.x;
    const R b = odd ? v.x : v.y;
    return cm<R>(xor_sign<R>(a, mre), xor_sign<R>(b, mim));
}
// inputs of a twiddle-free radix-4 butterfly times W_4^{q s} (forward,
// W_4 = -i) or W_4^{-q s} (inverse)
template <bool INV, typename C>
__device__ __forceinline__ void rot_inputs(C* v, int s) {
    using R = decltype(v[0].x);
    v[1] = mul_ipow<R>(v[1], INV ? s : -s);
    v[2] = mul_ipow<R>(v[2], 2 * s);
    v[3] = mul_ipow<R>(v[3], INV ? -s : s);
}

// One Stockham (self-sorting, decimation in time) stage of radix RAD on one
// line buffer X, computed in registers.  The caller places a barrier between
// stage_load and stage_store (in-place update).  Ns = 2^lgNs is the product of
// the radices of the earlier stages.  twl[q] = W_m^q (q < m/4) lives in LDS.
template <typename R, int RAD, int RMAX>
struct StageRegs {
    cplx<R> v[RMAX / RAD][RAD];
};

// W_m^q for any q < m from the quarter table twl[q'] = W_m^{q'}, q' < m/4:
// W_m^{q + t m/4} = (-i)^t W_m^q.
template <typename R>
__device__ __forceinline__ cplx<R> tw_quarter(const cplx<R>* twl, int q, int lgm) {
    const int t = q >> (lgm - 2);
    const cplx<R> w = twl[tw_slot<R>(q & ((1 << (lgm - 2)) - 1))];
    // (-i)^t w = i^{-t} w without divergent branches (part swap and sign
    // flips)
    return mul_ipow<R>(w, -t);
}

template <int RAD> struct Lg;
template <> struct Lg<2> { static constexpr int v = 1; };
template <> struct Lg<4> { static constexpr int v = 2; };
template <> struct Lg<8> { static constexpr int v = 3; };
template <> struct Lg<16> { static constexpr int v = 4; };

// Per-thread twiddles of the compile-time radix-4 plan (m = 4^NST, G = m/4,
// one butterfly per thread and stage): thread lt's butterfly in stage s
// (Ns = 4^s) needs W_{4 Ns}^{lt mod Ns} only.  In the quarter table W_m^q
// that is q = (lt mod Ns) m / (4 Ns), a stride of m / (4 Ns) slots across
// lanes; the table's slot order (tw_slot) serves strides 1 and 4 without
// bank conflicts, i.e. the last two stages of m = 1024.  Stage 1 selects
// among the constants W_16^k and stage 2 keeps its twiddle in a register.
// wl = W_{2m}^{lt}: the factors W_{2m}^{lt + i G} of the sine-transform and
// Toeplitz pre-passes are wl W_8^i.
// WL = false (kernels short of registers): the pre-pass factors are read
// from the global table instead of being formed from wl.
template <typename R, int RMAX, int LGM, bool WL = true>
struct LineTw {
    static constexpr bool kReg = (RMAX == 4 && LGM >= 8 && LGM % 2 == 0);
    static constexpr bool kW2 = false;   // stage-2 register (else a 4-way conflicting table read)
    static constexpr bool kWl = kReg && WL;
    cplx<R> w2;
    cplx<R> wl;
    // tw[s] = W_{2m}^s, s < 2m (global table)
    __device__ __forceinline__ void init(const cplx<R>* __restrict__ tw, int lt) {
        if constexpr (kReg) {
            if constexpr (kW2) w2 = tw[2 * ((lt & 15) << (LGM - 6))];   // W_64^{lt mod 16}
            if constexpr (kWl) wl = tw[lt];
        }
    }
    // W_16^{lt mod 4} W_4^s (s = out_rot(): the stage's outputs rotate)
    __device__ __forceinline__ static cplx<R> stage1(int lt) {
        const int k = lt & 3;
        const R c = k == 0 ? R(1) : (k == 1 ? static_cast<R>(kc16(1)) : (k == 2 ? static_cast<R>(kc16(2)) : static_cast<R>(kc16(3))));
        const R sn = k == 0 ? R(0) : (k == 1 ? static_cast<R>(ks16(1)) : (k == 2 ? static_cast<R>(ks16(2)) : static_cast<R>(ks16(3))));
        return mul_ipow<R>(cm<R>(c, -sn), -out_rot<R>());
    }
};

// W_{2 RMAX}^i as exact constants (forward sign), i < 2 RMAX, RMAX <= 8.
template <typename R, int RMAX>
__device__ __forceinline__ cplx<R> w2r(int i) {
    const int j = i * (8 / RMAX);
    return cm<R>(static_cast<R>(kc16(j)), static_cast<R>(-ks16(j)));
}

// Twiddles W^{r k} of this thread's butterflies in one stage; they are the
// same for every buffer of a line, so a stage over buffers A and B forms them
// once.  WR: wr is this thread's twiddle W_{Ns RAD}^k of the stage (LineTw);
// otherwise it is read from the LDS quarter table.  Radix-4 stages with
// Ns < 16 rotate their outputs (rot_inputs): a register twiddle comes
// rotated (LineTw::stage1), a table twiddle is rotated here, and a
// twiddle-free stage rotates its inputs in stage_load_tw.
template <typename R, int RAD, int RMAX>
struct StageTw {
    cplx<R> w[RMAX / RAD][RAD];
};
template <typename R, int RAD, int RMAX, bool INV, bool WR = false>
__device__ __forceinline__ void stage_tw(StageTw<R, RAD, RMAX>& t, int lgm, int lgNs, int lt, int G,
                                         const cplx<R>* twl, cplx<R> wr = cplx<R>{}) {
    using C = cplx<R>;
    constexpr int PER = RMAX / RAD;
    const int nb = (1 << lgm) >> Lg<RAD>::v;
    const int tsh = lgm - lgNs - Lg<RAD>::v;   // W_{Ns RAD}^q = W_m^{q << tsh}
    const int srot = (RAD == 4 && lgNs < 4) ? out_rot<R>() : 0;
    // every lane of a stage with twiddles multiplies (W^0 = 1 is exact in
    // the table and in the register twiddles), so no lane diverges
    if (lgNs == 0) return;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int b = lt + q * G;
        if (b < nb) {
            const int k = b & ((1 << lgNs) - 1);
            // one table read per butterfly; W^{r k} as products of W^k
            // (depth <= 4 multiplications, a few ulps)
            C* w = t.w[q];
            if constexpr (WR) w[1] = wr;
            else w[1] = tw_quarter<R>(twl, k << tsh, lgm);
            if (INV) w[1].y = -w[1].y;
            if constexpr (RAD == 4 && !WR)
                if (lgNs < 4) w[1] = mul_ipow<R>(w[1], INV ? srot : -srot);
            if constexpr (RAD >= 4) {
                w[2] = cmul(w[1], w[1]);
                w[3] = cmul(w[2], w[1]);
            }
            if constexpr (RAD >= 8) {
                w[4] = cmul(w[2], w[2]);
                w[5] = cmul(w[4], w[1]);
                w[6] = cmul(w[4], w[2]);
                w[7] = cmul(w[4], w[3]);
            }
            if constexpr (RAD >= 16) {
                w[8] = cmul(w[4], w[4]);
#pragma unroll
                for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
            }
        }
    }
}
// One Stockham stage's loads of buffer X, twiddles t (stage_tw) and
// butterflies, in registers.
template <typename R, int RAD, int RMAX, bool INV>
__device__ __forceinline__ void stage_load_tw(StageRegs<R, RAD, RMAX>& g, const cplx<R>* X, int lgm, int lgNs,
                                              int lt, int G, const StageTw<R, RAD, RMAX>& t) {
    constexpr int PER = RMAX / RAD;
    const int nb = (1 << lgm) >> Lg<RAD>::v;
    const int srot = (RAD == 4 && lgNs < 4) ? out_rot<R>() : 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int b = lt + q * G;
        if (b < nb) {
#pragma unroll
            for (int r = 0; r < RAD; ++r) g.v[q][r] = X[b + r * nb];
            if (lgNs > 0) {
#pragma unroll
                for (int r = 1; r < RAD; ++r) g.v[q][r] = cmul(g.v[q][r], t.w[q][r]);
            } else if constexpr (RAD == 4) {
                rot_inputs<INV>(g.v[q], srot);
            }
            dft<RAD, INV>(g.v[q]);
        }
    }
}
template <typename R, int RAD, int RMAX, bool INV, bool WR = false>
__device__ __forceinline__ void stage_load(StageRegs<R, RAD, RMAX>& g, const cplx<R>* X, int lgm, int lgNs, int lt,
                                           int G, const cplx<R>* twl, cplx<R> wr = cplx<R>{}) {
    StageTw<R, RAD, RMAX> t;
    stage_tw<R, RAD, RMAX, INV, WR>(t, lgm, lgNs, lt, G, twl, wr);
    stage_load_tw<R, RAD, RMAX, INV>(g, X, lgm, lgNs, lt, G, t);
}

// (u0, u1) = sw ? (a1, a0) : (a0, a1), component-wise selects on values
template <typename C>
__device__ __forceinline__ void csel2(C a0, C a1, bool sw, C& u0, C& u1) {
    u0.x = sw ? a1.x : a0.x;
    u0.y = sw ? a1.y : a0.y;
    u1.x = sw ? a0.x : a1.x;
    u1.y = sw ? a0.y : a1.y;
}
// u_i = a_{i ^ rot}, i < 4
template <typename C>
__device__ __forceinline__ void rot4(C a0, C a1, C a2, C a3, int rot, C& u0, C& u1, C& u2, C& u3) {
    C v0, v1, v2, v3;
    csel2(a0, a1, (rot & 1) != 0, v0, v1);
    csel2(a2, a3, (rot & 1) != 0, v2, v3);
    csel2(v0, v2, (rot & 2) != 0, u0, u2);
    csel2(v1, v3, (rot & 2) != 0, u1, u3);
}

// Radix 4: output register i (which holds y_{(i + s) mod 4}, see
// rot_inputs) goes to slot position (i + s) mod 4.  Radix 2 and 8: store i of
// a thread writes output r = i ^ rot (the rotation is applied with selects,
// so the register indices stay static).
template <typename R, int RAD, int RMAX>
__device__ __forceinline__ void stage_store(const StageRegs<R, RAD, RMAX>& g, cplx<R>* X, int lgm, int lgNs, int lt,
                                            int G) {
    using C = cplx<R>;
    constexpr int PER = RMAX / RAD;
    const int nb = (1 << lgm) >> Lg<RAD>::v;
    const int Ns = 1 << lgNs;
    // stages with Ns >= 16 (radix 8: Ns >= 8) store contiguous runs already;
    // only the earlier ones rotate
    const int rot = (RAD == 8) ? (Ns < 8 ? out_rot8<R>() : 0)
                               : ((Ns < 16) ? (out_rot<R>() & (RAD <= 4 ? RAD - 1 : 0)) : 0);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int b = lt + q * G;
        if (b < nb) {
            const int k = b & (Ns - 1);
            const int base = ((b - k) << Lg<RAD>::v) + k;
            if constexpr (RAD == 4) {
#pragma unroll
                for (int i = 0; i < 4; ++i) X[base + ((i + rot) & 3) * Ns] = g.v[q][i];
            } else if constexpr (RAD == 8) {
                // u_i = v_{i ^ rot} by three rounds of conditional pair swaps
                C u[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) u[r] = g.v[q][r];
#pragma unroll
                for (int bit = 1; bit < 8; bit <<= 1) {
                    const bool sw = (rot & bit) != 0;
#pragma unroll
                    for (int r = 0; r < 8; ++r)
                        if ((r & bit) == 0) {
                            C a0 = u[r], a1 = u[r | bit];
                            csel2(a0, a1, sw, u[r], u[r | bit]);
                        }
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) X[base + (i ^ rot) * Ns] = u[i];
            } else if constexpr (RAD == 2) {
                const C a0 = g.v[q][0], a1 = g.v[q][1];
                C u0, u1;
                csel2(a0, a1, (rot & 1) != 0, u0, u1);
                X[base + (0 ^ rot) * Ns] = u0;
                X[base + (1 ^ rot) * Ns] = u1;
            } else {
#pragma unroll
                for (int r = 0; r < RAD; ++r) X[base + r * Ns] = g.v[q][r];
            }
        }
    }
}

// Synchronisation of the threads of one line.  WS (wave sync): every line
// lies within one wavefront (G <= 64 threads, G dividing 64), so the line's
// exchanges through LDS need no workgroup barrier: a wavefront's LDS accesses
// execute in issue order, and the wavefront-scope fences keep the compiler
// from moving LDS reads and writes across the point.  The wavefronts of a
// workgroup then run their lines' transforms independently.  Otherwise a
// workgroup barrier.
template <bool WS>
__device__ __forceinline__ void line_sync() {
    if constexpr (WS) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Stage on A and (optionally) B.  For RMAX <= 8 both buffers' butterflies
// are in registers together (twice the independent work between the two
// barriers): load+compute A and B | barrier | store A and B | barrier.
// For RMAX = 16 one buffer's registers are live at a time:
// load+compute A | barrier | store A, load+compute B | barrier | store B,
// and the next stage's first barrier (or the one ending line_fft) orders
// "store B" before any later read of B.
template <typename R, int RAD, int RMAX, bool INV, bool WR = false, bool WS = false>
__device__ __forceinline__ void stockham_stage(cplx<R>* A, cplx<R>* B, bool both, int lgm, int lgNs, int lt,
                                               int G, const cplx<R>* twl, cplx<R> wr = cplx<R>{}) {
    if constexpr (RMAX <= 8) {
        StageRegs<R, RAD, RMAX> ga, gb;
        StageTw<R, RAD, RMAX> t;   // one set of twiddles for both buffers
        stage_tw<R, RAD, RMAX, INV, WR>(t, lgm, lgNs, lt, G, twl, wr);
        stage_load_tw<R, RAD, RMAX, INV>(ga, A, lgm, lgNs, lt, G, t);
        if (both) stage_load_tw<R, RAD, RMAX, INV>(gb, B, lgm, lgNs, lt, G, t);
        line_sync<WS>();
        stage_store<R, RAD, RMAX>(ga, A, lgm, lgNs, lt, G);
        if (both) stage_store<R, RAD, RMAX>(gb, B, lgm, lgNs, lt, G);
        line_sync<WS>();
    } else {
        StageRegs<R, RAD, RMAX> g;
        stage_load<R, RAD, RMAX, INV>(g, A, lgm, lgNs, lt, G, twl);
        line_sync<WS>();
        stage_store<R, RAD, RMAX>(g, A, lgm, lgNs, lt, G);
        if (both) {
            stage_load<R, RAD, RMAX, INV>(g, B, lgm, lgNs, lt, G, twl);
            line_sync<WS>();
            stage_store<R, RAD, RMAX>(g, B, lgm, lgNs, lt, G);
        } else {
            line_sync<WS>();
        }
    }
}

// Compile-time stage plan (m = 2^LGM known at compile time): every index,
// bound and radix folds to a constant.
// Stages LGNS .. LGEND - 1 (default: through the last one).
template <typename R, bool INV, int RMAX, int LGM, int LGNS, typename LT, bool WS, int LGEND = LGM>
__device__ __forceinline__ void fft_stages_ct(cplx<R>* A, cplx<R>* B, bool both, int lt, const cplx<R>* twl,
                                              const LT& lw) {
    if constexpr (LGNS < LGEND) {
        constexpr int rem = LGM - LGNS;
        constexpr int lr = rem < Lg<RMAX>::v ? rem : Lg<RMAX>::v;
        constexpr int G = (1 << LGM) / RMAX;
        constexpr bool kReg = LT::kReg && (LGNS == 2 || (LGNS == 4 && LT::kW2));
        cplx<R> wr{};
        if constexpr (kReg) {
            if constexpr (LGNS == 2) wr = LT::stage1(lt);
            else wr = lw.w2;
        }
        stockham_stage<R, (1 << lr), RMAX, INV, kReg, WS>(A, B, both, LGM, LGNS, lt, G, twl, wr);
        fft_stages_ct<R, INV, RMAX, LGM, LGNS + lr, LT, WS, LGEND>(A, B, both, lt, twl, lw);
    }
}

// Length-m FFT (unnormalised) of line buffer A (and B), natural order in and
// out (m = 2^lgm), radices up to RMAX (G >= m / RMAX threads per line).
// LGM > 0 selects the compile-time plan for m = 2^LGM.  Ends with a line
// synchronisation (WS: the compile-time plans with G <= 64 only).
template <typename R, bool INV, int RMAX, int LGM, typename LT, bool WS = false>
__device__ __forceinline__ void line_fft(cplx<R>* A, cplx<R>* B, bool both, int lgm, int lt, int G,
                                         const cplx<R>* twl, const LT& lw) {
    static_assert(!WS || LGM > 0, "wave sync needs a compile-time plan");
    if constexpr (LGM > 0) {
        fft_stages_ct<R, INV, RMAX, LGM, 0, LT, WS>(A, B, both, lt, twl, lw);
    } else {
        constexpr int LGMAX = Lg<RMAX>::v;
        int lgNs = 0;
        while (lgNs < lgm) {
            const int rem = lgm - lgNs;
            const int lr = rem < LGMAX ? rem : LGMAX;
            if (lr == 4) {
                if constexpr (RMAX >= 16) stockham_stage<R, 16, RMAX, INV>(A, B, both, lgm, lgNs, lt, G, twl);
            } else if (lr == 3) {
                if constexpr (RMAX >= 8) stockham_stage<R, 8, RMAX, INV>(A, B, both, lgm, lgNs, lt, G, twl);
            } else if (lr == 2) {
                stockham_stage<R, 4, RMAX, INV>(A, B, both, lgm, lgNs, lt, G, twl);
            } else {
                stockham_stage<R, 2, RMAX, INV>(A, B, both, lgm, lgNs, lt, G, twl);
            }
            lgNs += lr;
        }
    }
    line_sync<WS>();
}

// Cross-lane moves without LDS: DPP (data-parallel primitives) on 32-bit
// halves, lanes without a source lane reading 0; readlane broadcasts one
// lane's value to the wavefront.
template <int CTRL, typename R>
__device__ __forceinline__ R dpp_mov(R v) {
    if constexpr (sizeof(R) == 8) {
        const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
        const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, true);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
        return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    } else {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
    }
}
template <typename R>
__device__ __forceinline__ R read_lane(R v, int lane) {
    if constexpr (sizeof(R) == 8) {
        const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
        const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, lane);
        const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
        return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
    }
}
// DPP controls: row_shr:d (within rows of 16 lanes), quad_perm [1,0,3,2] and
// [2,3,0,1], row_half_mirror, row_mirror.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppQuadSwap1 = 0xB1, kDppQuadSwap2 = 0x4E, kDppHalfMirror = 0x141, kDppRowMirror = 0x140;

// Exclusive prefix sum of v over the G threads of a line (threads lt = 0..G-1
// are consecutive lanes of the workgroup, G a power of two).  Segments of 16
// lanes or more: a tree scan within each row of 16 lanes by DPP row shifts,
// then the totals of the segment's earlier rows; narrower segments use lane
// shuffles.  Lines wider than a wavefront add the totals of their earlier
// wavefronts from LDS.  Must be reached by the whole workgroup (full
// wavefronts).
template <typename R>
__device__ __forceinline__ cplx<R> line_exclusive_scan(cplx<R> v, int G) {
    using C = cplx<R>;
    __shared__ C s_wtot[16];   // one total per wavefront (<= 1024 threads)
    const int lane = threadIdx.x & 63;
    const int sw = G < 64 ? G : 64;     // segment width
    C inc = v;
    C exc;
    if (sw >= 16) {
        inc.x += dpp_mov<kDppRowShr1>(inc.x);
        inc.y += dpp_mov<kDppRowShr1>(inc.y);
        inc.x += dpp_mov<kDppRowShr2>(inc.x);
        inc.y += dpp_mov<kDppRowShr2>(inc.y);
        inc.x += dpp_mov<kDppRowShr4>(inc.x);
        inc.y += dpp_mov<kDppRowShr4>(inc.y);
        inc.x += dpp_mov<kDppRowShr8>(inc.x);
        inc.y += dpp_mov<kDppRowShr8>(inc.y);
        exc.x = dpp_mov<kDppRowShr1>(inc.x);   // 0 in the first lane of a row
        exc.y = dpp_mov<kDppRowShr1>(inc.y);
        // totals of rows 0, 1, 2 of the wavefront
        const C r0 = cm<R>(read_lane(inc.x, 15), read_lane(inc.y, 15));
        const C r1 = cm<R>(read_lane(inc.x, 31), read_lane(inc.y, 31));
        const C r2 = cm<R>(read_lane(inc.x, 47), read_lane(inc.y, 47));
        const int row = lane >> 4;
        C add = czero<C>();
        if (sw == 32) {
            if (row == 1) add = r0;
            if (row == 3) add = r2;
        } else if (sw == 64) {
            const C r01 = cadd(r0, r1);
            if (row == 1) add = r0;
            if (row == 2) add = r01;
            if (row == 3) add = cadd(r01, r2);
        }
        inc = cadd(inc, add);
        exc = cadd(exc, add);
    } else {
        const int ls = lane & (sw - 1);     // position in the segment
        for (int d = 1; d < sw; d <<= 1) {
            const R tx = __shfl_up(inc.x, d, sw);
            const R ty = __shfl_up(inc.y, d, sw);
            if (ls >= d) {
                inc.x += tx;
                inc.y += ty;
            }
        }
        exc.x = __shfl_up(inc.x, 1, sw);
        exc.y = __shfl_up(inc.y, 1, sw);
        if (ls == 0) exc = czero<C>();
    }
    if (G > 64) {
        const int wave = threadIdx.x >> 6;
        if (lane == 63) s_wtot[wave] = inc;
        __syncthreads();
        const int w0 = (threadIdx.x - (threadIdx.x & (G - 1))) >> 6;   // first wavefront of the line
        for (int w = w0; w < wave; ++w) exc = cadd(exc, s_wtot[w]);
        __syncthreads();   // s_wtot is reused by the next call
    }
    return exc;
}

// Orthonormal DST-I of the line in A (slots 1..m-1), result in A, with one
// length-m FFT.  With x_0 = x_m = 0, a_j = x_j - x_{m-j} and
// b_j = (x_j + x_{m-j}) W_{2m}^j, the transforms A = FFT_m(a), B = FFT_m(b)
// give y_{2p} = (i/sqrt(2m)) A_p and y_{2p+1} = (i/sqrt(2m)) B_p.  Only
// C = FFT_m(a + b) is computed: a is odd about m/2 (A_{m-p} = -A_p) and b
// changes sign under j -> m - j after the half-sample shift
// (B_{m-1-p} = -B_p), so C_p + C_{m-p} = B_p - B_{p-1} and B_0 = C_0:
// B_p = C_0 + sum_{q=1..p} (C_q + C_{m-q}), A_p = C_p - B_p.  The sum is a
// prefix scan over p < m/2 (each thread owns a contiguous range of p).
// Caller has synchronised after writing A.  tw[s] = W_{2m}^s (global table).
// B is not used.  post(k, y_k) is applied to every output k >= 1 before it
// is stored (an elementwise operation fused into the transform's last step).
struct DstNoPost {
    template <typename C>
    __device__ __forceinline__ C operator()(int, C v) const { return v; }
};
template <typename R, int RMAX, int LGM, typename LT, bool WS = false, typename POST = DstNoPost>
__device__ __forceinline__ void line_dst(cplx<R>* A, cplx<R>* B, int lgm, int lt, int G,
                                         const cplx<R>* __restrict__ tw, const cplx<R>* twl, const LT& lw,
                                         const POST& post = POST{}) {
    using C = cplx<R>;
    constexpr bool kReg = LT::kReg;
    (void)B;
    const int m = 1 << lgm;
    const int half = m >> 1;
    // c_j = a_j + b_j for the pair (j, m - j); w = W_{2m}^j
    auto pre = [&](int j, C w) {
        if (j == 0) {
            A[0] = czero<C>();
        } else {
            const C xj = A[j];
            if (j == half) {
                // a = 0, b = 2 x W_{2m}^{m/2} = -2 i x
                A[j] = cm<R>(R(2) * xj.y, R(-2) * xj.x);
            } else {
                const C xmj = A[m - j];
                const C a = csub(xj, xmj);
                const C sw = cadd(xj, xmj);
                A[j] = cadd(a, cmul(sw, w));        // a_j + s_j W^j
                A[m - j] = csub(cneg(a), cmulc(sw, w));   // -a_j + s_j W^{m-j} = -a_j - s_j conj(W^j)
            }
        }
    };
    if constexpr (kReg) {
        // Compile-time radix-4 plan: the first FFT stage of thread lt reads
        // slots s_r = lt + r G (G = m / 4).  The thread forms those four
        // pre-processed values itself from x_s and x_{m-s} (the mirror slots
        // m - s_r are the first-stage slots of thread G - lt), so the
        // pre-processing needs no LDS round trip.  Slots s_0, s_1 < m/2 take
        // a_j + s_j W^j (j = s_r, thread lt's own pairs, W_{2m}^j = wl W_8^r);
        // s_2, s_3 > m/2 take -a_j - s_j conj(W^j) with j = m - s_r, the
        // pairs of thread G - lt (W_{2m}^j = wl' W_8^{3-r}, wl' = W_{2m}^{G-lt}),
        // computed with the same operations as that thread would.  Thread 0:
        // s_0 = 0 is the Dirichlet zero, s_2 = m/2 is the middle value, and
        // s_3 = m - G pairs with its own s_1.
        constexpr int Gc = (1 << LGM) / 4;
        static_assert(RMAX == 4, "register plan");
        const int mt = (Gc - lt) & (Gc - 1);   // mirror thread (thread 0: itself)
        C xs[4], xm[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            xs[r] = A[lt + r * Gc];
            xm[r] = A[(m - lt - r * Gc) & (m - 1)];   // slot m - s_r (thread 0, r = 0: unused)
        }
        C w[4];
        if constexpr (LT::kWl) {
            const C wm = tw[mt];
            w[0] = cmul(lw.wl, w2r<R, 4>(0));
            w[1] = cmul(lw.wl, w2r<R, 4>(1));
            w[2] = cmul(wm, w2r<R, 4>(1));
            w[3] = cmul(wm, w2r<R, 4>(0));
        } else {
            w[0] = tw[lt];
            w[1] = tw[lt + Gc];
            w[2] = tw[mt + Gc];
            w[3] = tw[mt];
        }
        if (lt == 0) w[3] = w[1];
        StageRegs<R, 4, 4> g;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const C a = csub(xs[r], xm[r]);
            const C sw = cadd(xs[r], xm[r]);
            g.v[0][r] = cadd(a, cmul(sw, w[r]));
        }
#pragma unroll
        for (int r = 2; r < 4; ++r) {
            // x_j = xm[r], x_{m-j} = xs[r]
            const C a = csub(xm[r], xs[r]);
            const C sw = cadd(xm[r], xs[r]);
            g.v[0][r] = csub(cneg(a), cmulc(sw, w[r]));
        }
        if (lt == 0) {
            g.v[0][0] = czero<C>();
            g.v[0][2] = cm<R>(R(2) * xs[2].y, R(-2) * xs[2].x);   // a = 0, b = -2 i x
        }
        rot_inputs<false>(g.v[0], out_rot<R>());   // the stage's outputs rotate
        dft<4, false>(g.v[0]);
        line_sync<WS>();
        stage_store<R, 4, 4>(g, A, LGM, 0, lt, Gc);
        line_sync<WS>();
        fft_stages_ct<R, false, 4, LGM, 2, LT, WS>(A, A, false, lt, twl, lw);
    } else {
        for (int j = lt; j <= half; j += G) pre(j, j < half ? tw[j] : czero<C>());
        line_sync<WS>();
        line_fft<R, false, RMAX, LGM, LT, WS>(A, A, false, lgm, lt, G, twl, lw);
    }
    // p range of this thread: [lt E, lt E + E), E = half / G (G <= half unless m < 2 RMAX... E >= 1)
    constexpr int PER = RMAX / 2;
    const int E = half >= G ? half / G : 1;
    const int p0 = lt * E;
    const R sc = static_cast<R>(1.0 / sqrt(2.0 * m));
    if (PER == 2 && E == 2) {
        // two values of p per thread: C_p and C_{m-p} are read, and the four
        // outputs y_{4 lt .. 4 lt + 3} written, in lane-rotated order (the
        // reads at stride 2 and the writes at stride 4 across lanes are then
        // free of bank conflicts)
        const int sr = scan_rot<R>();
        const C f0 = A[p0 + sr], f1 = A[p0 + (sr ^ 1)];
        const int q0 = p0 + sr, q1 = p0 + (sr ^ 1);
        const C g0 = A[q0 > 0 ? m - q0 : 0], g1 = A[q1 > 0 ? m - q1 : 0];
        C c0p, c1p, m0p, m1p;
        csel2(f0, f1, sr != 0, c0p, c1p);     // C_{p0}, C_{p0+1}
        csel2(g0, g1, sr != 0, m0p, m1p);     // C_{m-p0}, C_{m-p0-1}
        C run = (p0 > 0) ? cadd(c0p, m0p) : czero<C>();
        const C d0 = run;
        run = cadd(run, cadd(c1p, m1p));
        const C d1 = run;
        const C c0 = A[0];
        const C off = cadd(c0, line_exclusive_scan<R>(run, G));
        line_sync<WS>();   // every read of C is done before the outputs overwrite it
        const C b0 = cadd(off, d0), b1 = cadd(off, d1);
        const C a0 = csub(c0p, b0), a1 = csub(c1p, b1);
        // y = (i sc) v: y_{2p} from A_p, y_{2p+1} from B_p
        const int o = 2 * p0;
        const R y0r = (p0 == 0) ? R(0) : -sc * a0.y, y0i = (p0 == 0) ? R(0) : sc * a0.x;
        C y0 = cm<R>(y0r, y0i);
        if (p0 != 0) y0 = post(o, y0);
        const C y1 = post(o + 1, cm<R>(-sc * b0.y, sc * b0.x));
        const C y2 = post(o + 2, cm<R>(-sc * a1.y, sc * a1.x));
        const C y3 = post(o + 3, cm<R>(-sc * b1.y, sc * b1.x));
        const int rot = out_rot<R>();
        C u0, u1, u2, u3;
        rot4(y0, y1, y2, y3, rot, u0, u1, u2, u3);
        A[o + (0 ^ rot)] = u0;
        A[o + (1 ^ rot)] = u1;
        A[o + (2 ^ rot)] = u2;
        A[o + (3 ^ rot)] = u3;
    } else {
        C cp[PER], dinc[PER];
        C run = czero<C>();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int p = p0 + e;
            if (e < E && p < half) {
                cp[e] = A[p];
                if (p > 0) run = cadd(run, cadd(cp[e], A[m - p]));
                dinc[e] = run;
            }
        }
        const C c0 = A[0];
        const C off = cadd(c0, line_exclusive_scan<R>(run, G));
        line_sync<WS>();   // every read of C is done before the outputs overwrite it
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int p = p0 + e;
            if (e < E && p < half) {
                const C bp = cadd(off, dinc[e]);
                const C ap = csub(cp[e], bp);
                // y = (i sc) v
                A[2 * p] = (p == 0) ? czero<C>() : post(2 * p, cm<R>(-sc * ap.y, sc * ap.x));
                A[2 * p + 1] = post(2 * p + 1, cm<R>(-sc * bp.y, sc * bp.x));
            }
        }
    }
    line_sync<WS>();
}

// Toeplitz convolution core: on exit A holds IFFT_m(s_e FFT_m(x)) and B holds
// IFFT_m(s_o FFT_m(W^j x)); the product at slot j is A[j] + conj(W_{2m}^j) B[j].
template <typename R, int RMAX, int LGM, typename LT, bool WS = false>
__device__ __forceinline__ void line_toeplitz(cplx<R>* A, cplx<R>* B, int lgm, int lt, int G,
                                              const cplx<R>* __restrict__ tw, const cplx<R>* twl,
                                              const R* __restrict__ sym_e, const R* __restrict__ sym_o,
                                              R tscale, const LT& lw) {
    const int m = 1 << lgm;
    if constexpr (LT::kReg) {
        // Compile-time radix-4 plan (G = m / 4, one butterfly per thread and
        // stage).  The first stage of a transform reads slots lt + r G, and
        // the last stage writes its outputs to the same slots, so the
        // W_{2m}^j pre-multiplication of B is applied to the first stage's
        // registers, and the symbol multiplication joins the forward
        // transform's last stage to the inverse transform's first stage
        // without a round trip through LDS.  Same operations, same order.
        using C = cplx<R>;
        constexpr int Gc = (1 << LGM) / 4;
        static_assert(RMAX == 4, "register plan");
        {
            StageRegs<R, 4, 4> ga, gb;
#pragma unroll
            for (int r = 0; r < 4; ++r) ga.v[0][r] = A[lt + r * Gc];
            // both buffers' first-stage outputs rotate (rot_inputs)
            rot_inputs<false>(ga.v[0], out_rot<R>());
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if constexpr (LT::kWl) gb.v[0][r] = cmul(ga.v[0][r], cmul(lw.wl, w2r<R, 4>(r)));
                else gb.v[0][r] = cmul(ga.v[0][r], tw[lt + r * Gc]);
            }
            dft<4, false>(ga.v[0]);
            dft<4, false>(gb.v[0]);
            line_sync<WS>();
            stage_store<R, 4, 4>(ga, A, LGM, 0, lt, Gc);
            stage_store<R, 4, 4>(gb, B, LGM, 0, lt, Gc);
            line_sync<WS>();
        }
        fft_stages_ct<R, false, 4, LGM, 2, LT, WS, LGM - 2>(A, B, true, lt, twl, lw);
        {
            // forward last stage (no register twiddle: LGM - 2 >= 6)
            StageRegs<R, 4, 4> ga, gb;
            R se[4], so[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                se[r] = sym_e[lt + r * Gc] * tscale;
                so[r] = sym_o[lt + r * Gc] * tscale;
            }
            StageTw<R, 4, 4> t;
            stage_tw<R, 4, 4, false>(t, LGM, LGM - 2, lt, Gc, twl);
            stage_load_tw<R, 4, 4, false>(ga, A, LGM, LGM - 2, lt, Gc, t);
            stage_load_tw<R, 4, 4, false>(gb, B, LGM, LGM - 2, lt, Gc, t);
            // output r belongs to slot lt + r G; inverse stage 0 (twiddle-free)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ga.v[0][r] = cscale(ga.v[0][r], se[r]);
                gb.v[0][r] = cscale(gb.v[0][r], so[r]);
            }
            rot_inputs<true>(ga.v[0], out_rot<R>());
            rot_inputs<true>(gb.v[0], out_rot<R>());
            dft<4, true>(ga.v[0]);
            dft<4, true>(gb.v[0]);
            line_sync<WS>();
            stage_store<R, 4, 4>(ga, A, LGM, 0, lt, Gc);
            stage_store<R, 4, 4>(gb, B, LGM, 0, lt, Gc);
            line_sync<WS>();
        }
        fft_stages_ct<R, true, 4, LGM, 2, LT, WS>(A, B, true, lt, twl, lw);
        (void)m;
        (void)G;
    } else {
        for (int s = lt; s < m; s += G) B[s] = cmul(A[s], tw[s]);
        line_sync<WS>();
        line_fft<R, false, RMAX, LGM, LT, WS>(A, B, true, lgm, lt, G, twl, lw);
        for (int p = lt; p < m; p += G) {
            A[p] = cscale(A[p], sym_e[p] * tscale);
            B[p] = cscale(B[p], sym_o[p] * tscale);
        }
        line_sync<WS>();
        line_fft<R, true, RMAX, LGM, LT, WS>(A, B, true, lgm, lt, G, twl, lw);
    }
}

// ---------------------------------------------------------------------------
// wavefront / workgroup reductions (fixed order: deterministic)
// ---------------------------------------------------------------------------
// Sum over the 64 lanes of a (full) wavefront, the same value in every lane:
// pairs, quads, half rows and rows by DPP, then the four row totals.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_mov<kDppQuadSwap1>(v);
    v += dpp_mov<kDppQuadSwap2>(v);
    v += dpp_mov<kDppHalfMirror>(v);
    v += dpp_mov<kDppRowMirror>(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

}  // namespace fnls
