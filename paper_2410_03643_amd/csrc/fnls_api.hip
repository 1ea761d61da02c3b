// C ABI of libfnls (declared in include/fnls.h): context, workspace layout,
// host assembly of the tables, and the GMRES / GMRES-IR drivers that
// sequence the kernels of fnls_kernels.hip on the context's stream.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fnls.h"
#include "fnls_common.h"
#include "fnls_launch.h"

using namespace fnls;

namespace {

constexpr size_t kAlign = 256;
constexpr int kEvents = 8;
constexpr size_t kStaticLds = 8 * 1024;    // static LDS of k_pass (reduction scratch)
// lines per workgroup of the transform passes at m = 1024 (more for smaller m)
constexpr int kRowLines = 1;
constexpr int kColLines = 4;
// producers with more workgroups than this get an explicit reduction kernel
// (kReduceChunks workgroups, each summing a contiguous chunk of them)
constexpr int kRedundantMax = 1024;
constexpr int kReduceChunks = 64;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Host-side trace range (roctx): one per solve-level API call and one per
// restart cycle, so that a profiler recording markers (rocprofv3
// --marker-trace) shows where the host spends its time between the kernels.
// Without such a profiler a push or pop is a call that returns at once.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

bool valid_n(int n) {
    if (n < 1 || n > 1023) return false;
    const int m = n + 1;
    return (m & (m - 1)) == 0;
}

long long ipow(int n, int d) {
    long long r = 1;
    for (int i = 0; i < d; ++i) r *= n;
    return r;
}

struct Geo {
    int G, L, blocks, rmax;
    size_t lds;
    long long stride, nlines;
};

// Transform-pass configuration per (precision, axis kind): the largest FFT
// radix (threads per line G = m / rmax) and the lines per workgroup at
// m = 1024 (scaled up for shorter lines so a workgroup keeps its size).
struct PassConfig {
    int rmax[2][2];    // [fp64][strided axis]
    int lines[2][2];
};

// Default schedule for line length m (m = 0: before assembly).  Radix 4
// everywhere: radix 8 and 16 (also with the one-wavefront-per-line plans at
// m = 256, 512, 1024) measured slower at every size.  Lines per workgroup as
// measured best for FP64 and FP32 solves at d = 2, n = 1023 and 511 and
// d = 3, n = 255 (fastest of 81 schedules each); other lengths take the
// n = 1023 choice.
PassConfig default_pass_config(int m = 0) {
    PassConfig p;   // [FP32 = 0, FP64 = 1][contiguous = 0, strided = 1]
    for (int f = 0; f < 2; ++f)
        for (int st = 0; st < 2; ++st) p.rmax[f][st] = 4;
    p.lines[0][0] = 1;
    p.lines[0][1] = 4;
    p.lines[1][0] = 1;
    p.lines[1][1] = 2;
    if (m == 512) {
        p.lines[0][1] = 1;
        p.lines[1][1] = 1;
    } else if (m == 256) {
        p.lines[0][0] = 2;
        p.lines[0][1] = 2;
    }
    return p;
}

int pass_threads_max(int rmax) { return rmax == 16 ? 256 : 4096 / rmax; }

// Transform-pass schedules found by fnls_autotune, per line length m,
// precision and axis kind, for the whole process: contexts assembled later
// with the same m start from them, and batches use them for their
// line-length classes.
struct TunedTable {
    std::mutex mu;
    std::map<long long, std::pair<int, int>> tab;   // key m * 4 + fp64 * 2 + strided -> (rmax, lines)
};
TunedTable& tuned_table() {
    static TunedTable t;
    return t;
}
bool tuned_get(int m, bool fp64, bool strided, int* rmax, int* lines) {
    TunedTable& t = tuned_table();
    std::lock_guard<std::mutex> lock(t.mu);
    auto it = t.tab.find((long long)m * 4 + (fp64 ? 2 : 0) + (strided ? 1 : 0));
    if (it == t.tab.end()) return false;
    *rmax = it->second.first;
    *lines = it->second.second;
    return true;
}
void tuned_put(int m, bool fp64, bool strided, int rmax, int lines) {
    TunedTable& t = tuned_table();
    std::lock_guard<std::mutex> lock(t.mu);
    t.tab[(long long)m * 4 + (fp64 ? 2 : 0) + (strided ? 1 : 0)] = std::make_pair(rmax, lines);
}

// LDS line layout of a pass kernel: a line buffer holds pa >= m slots and
// consecutive lines are ls slots apart (2 pa with the Toeplitz buffer).  On
// strided axes the lanes of a wavefront spread over L interleaved lines; the
// element writes of one LDS write cycle (8 lanes of 16-byte values, 16 of
// 8-byte ones, on a 128-byte bank row) stay apart when
// ls * size = 128 / L modulo 256 / L bytes.  ls is the smallest stride >= k m
// (k buffers) that gives it (k m itself for a single line or when none
// does); with two buffers B starts pa = m + (ls - 2 m) / 2 slots after A, so
// an odd stride (16-byte values, 8 lines) leaves its spare slot after B.
void line_layout(int m, int L, bool fp64, bool two, int* pa, int* ls) {
    const int elem = fp64 ? 16 : 8;
    const int k = two ? 2 : 1;
    int extra = 0;
    if (L >= 2 && 128 / L >= elem) {
        const int target = 128 / L / elem, mod = 256 / L / elem;   // in slots
        for (int d = 0; d < mod; ++d)
            if ((k * m + d) % mod == target) {
                extra = d;
                break;
            }
    }
    *ls = k * m + extra;
    *pa = two ? m + extra / 2 : *ls;
}

Geo pass_geo(int d, int n, int axis, bool fp64, size_t max_dyn_lds, const PassConfig& cfg) {
    Geo g;
    const int m = n + 1;
    const bool contiguous = (axis == d - 1);
    const int col = contiguous ? 0 : 1;
    g.rmax = cfg.rmax[fp64 ? 1 : 0][col];
    g.G = std::max(1, m / g.rmax);
    const int tmax = pass_threads_max(g.rmax);
    // LDS of L lines with buffers A and B (line_layout), the quarter twiddle
    // table, per-line base offset (8 B) and Lambda (elem/2 B)
    auto lds_of = [&](int L) {
        int pa = 0, ls = 0;
        line_layout(m, L, fp64, true, &pa, &ls);
        const size_t elem = fp64 ? 16 : 8;
        return (size_t)L * ls * elem + (size_t)(m >= 4 ? m / 4 : 1) * elem + (size_t)L * (8 + elem / 2);
    };
    const int gref = 1024 / g.rmax;
    int L = cfg.lines[fp64 ? 1 : 0][col] * std::max(1, gref / g.G);
    L = std::max(1, std::min(L, tmax / g.G));
    while (L > 1 && lds_of(L) > max_dyn_lds) L /= 2;
    while (g.G * L < 64) L *= 2;   // whole wavefronts
    g.L = L;
    g.lds = lds_of(L);
    g.stride = ipow(n, d - 1 - axis);
    g.nlines = ipow(n, d - 1);
    g.blocks = (int)((g.nlines + L - 1) / L);
    return g;
}

int stream_blocks(long long N) {
    return (int)std::max<long long>(1, (N + (long long)kStreamThreads * kEpt - 1) / ((long long)kStreamThreads * kEpt));
}

struct Layout {
    // operator region (offsets from the context's workspace): tables, the
    // diagonal, the stepper's right-hand side and the adjoint solution
    size_t tw64, tw32, syme64, symo64, lam64, syme32, symo32, lam32, D64, D32, bbuf, adj;
    size_t op_total;
    // solver scratch (offsets from the scratch base, which follows the
    // operator region in the workspace): GMRES state, partial sums, work
    // vectors, the preconditioned basis Z and the Krylov basis V
    size_t state, p1, p2, p3, pr, px, t1, t2, Z, acc, r64, V;
    size_t scr_total;
    size_t total;
    int pstride;
};

// Solver scratch of one restart length (offsets from the scratch base).
void scratch_layout(Layout& l, int d, int n, int restart) {
    const long long N = ipow(n, d);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    l.state = take(sizeof(GmresState));
    // partial sums: at most one workgroup per line (any pass configuration)
    // or per streaming chunk
    const int pmax = (int)std::max<long long>(stream_blocks(N), ipow(n, d - 1));
    l.pstride = pmax;
    const size_t pwide = (size_t)(kMaxRestart + 2) * pmax * 16;
    l.p1 = take(pwide);
    l.p2 = take(pwide);
    l.p3 = take((size_t)pmax * 16);
    l.pr = take((size_t)pmax * 16);
    l.px = take((size_t)(kMaxRestart + 2) * kReduceChunks * 16);
    l.t1 = take((size_t)N * 16);
    l.t2 = take((size_t)N * 16);
    l.Z = take((size_t)N * 16 * restart);   // preconditioned basis z_j = P^{-1} v_j
    l.acc = take((size_t)N * 16);
    l.r64 = take((size_t)N * 16);
    l.V = take((size_t)N * 16 * restart);
    l.scr_total = off;
}

Layout make_layout(int d, int n, int restart) {
    Layout l;
    const int m = n + 1;
    const long long N = ipow(n, d);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    l.tw64 = take((size_t)2 * m * 16);
    l.tw32 = take((size_t)2 * m * 8);
    l.syme64 = take((size_t)m * 8);
    l.symo64 = take((size_t)m * 8);
    l.lam64 = take((size_t)m * 8);
    l.syme32 = take((size_t)m * 4);
    l.symo32 = take((size_t)m * 4);
    l.lam32 = take((size_t)m * 4);
    l.D64 = take((size_t)N * 8);
    l.D32 = take((size_t)N * 4);
    l.bbuf = take((size_t)N * 16);
    l.adj = take((size_t)N * 16);   // adjoint solution (reverse mode)
    l.op_total = off;
    scratch_layout(l, d, n, restart);
    l.total = l.op_total + l.scr_total;
    return l;
}

// Solver scratch of fnls_solve_noalloc: one file-scope array per device,
// held from the code object's load until the process ends.  Host code never
// uses the array's name as an address (on the host it is a stand-in, not a
// device address): static_scratch() takes each device's address from
// hipGetSymbolAddress once, with that device current, and every later use
// goes through that pointer.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;

// This device's address of `scratch` (nullptr if it cannot be had); the
// caller has made `device` current.
char* static_scratch(int device) {
    static std::mutex mu;
    static char* addr[kMaxDevices] = {};
    static bool tried[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!tried[device]) {
        tried[device] = true;
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) addr[device] = static_cast<char*>(p);
        else (void)hipGetLastError();
    }
    return addr[device];
}

}  // namespace

struct fnls_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t max_dyn_lds = 64 * 1024;
    std::string err;
    // parameters
    int assembled = 0;
    double alpha = 0, rho = 0, h = 0, tau = 0;
    int d = 0, n = 0, m = 0;
    long long N = 0;
    int restart_cap = 0;
    double tscale = 1.0;
    double omega = 1.0;
    int have_D = 0;
    const double* Vpot = nullptr;   // potential added to D by the steppers (fnls_set_potential)
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    char* scr = nullptr;            // solver scratch base (ws + lay.op_total, or the static scratch)
    char* static_scr = nullptr;     // this device's static scratch array (fnls_solve_noalloc)
    Layout lay{};
    HostStatus* hs = nullptr;       // pinned, device-written
    HostStatus* hs_dev = nullptr;
    unsigned seq_base = 0;          // HostStatus::seq of this solve's configuration (reports follow it)
    int fuse = 0;                   // Givens step of iteration j in the first pass of j + 1
    int restart_cur = 0;            // restart length of the running cycle
    int poll_delay_us = 0;          // testing aid: the host sleeps before each status wait
    fnls_host_stats stats{};        // host sequencing counters (fnls_get_host_stats)
    // optional per-launch timing (fnls_timing / fnls_timing_report)
    struct TimingRec {
        int cls;
        LaunchEvents ev;
        double bytes;       // every vector the launch reads or writes, once each
        double bytes_min;   // the launch's share of the method's minimal traffic
    };
    int timing = 0;
    std::vector<TimingRec> recs;
    std::vector<hipEvent_t> evpool;
    size_t evused = 0;
    std::vector<std::string> class_names;
    int cur_k = 0;   // basis size of the combination being formed (byte accounting)
    PassConfig pcfg = default_pass_config();

    template <typename T> T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }      // operator region
    template <typename T> T* sc(size_t off) { return reinterpret_cast<T*>(scr + off); }     // solver scratch
    GmresState* st() { return sc<GmresState>(lay.state); }
};

static int set_err(fnls_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return set_err(ctx, FNLS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// ---------------------------------------------------------------------------
// optional per-launch timing with HIP events
// ---------------------------------------------------------------------------
namespace {

hipEvent_t pool_event(fnls_ctx* c) {
    if (c->evused == c->evpool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->evpool.push_back(e);
    }
    return c->evpool[c->evused++];
}

int class_id(fnls_ctx* c, const std::string& name) {
    for (size_t i = 0; i < c->class_names.size(); ++i)
        if (c->class_names[i] == name) return (int)i;
    c->class_names.push_back(name);
    return (int)c->class_names.size() - 1;
}

// Start a timing record for the next launch: returns the events the runtime
// records at that kernel's start and end, or nullptr when timing is off.
const LaunchEvents* timing_begin(fnls_ctx* c, const std::string& name, double bytes, double bytes_min) {
    if (!c->timing) return nullptr;
    fnls_ctx::TimingRec r;
    r.cls = class_id(c, name);
    r.ev.start = pool_event(c);
    r.ev.stop = pool_event(c);
    r.bytes = bytes;
    r.bytes_min = bytes_min;
    if (!r.ev.start || !r.ev.stop) return nullptr;
    c->recs.push_back(r);
    return &c->recs.back().ev;
}

// Drop the record of a launch that failed (its events were never recorded).
void timing_failed(fnls_ctx* c, const LaunchEvents* te) {
    if (te && !c->recs.empty()) c->recs.pop_back();
}

}  // namespace

// ---------------------------------------------------------------------------
// pass sequencing
// ---------------------------------------------------------------------------
namespace {

PassArgs base_args(fnls_ctx* c, bool fp64, int axis, const Geo& g) {
    PassArgs a;
    std::memset(&a, 0, sizeof a);
    a.n = c->n;
    a.m = c->m;
    a.d = c->d;
    a.axis = axis;
    a.G = g.G;
    a.L = g.L;
    a.lgG = 0;
    while ((1 << a.lgG) < g.G) ++a.lgG;
    a.lgm = 0;
    while ((1 << a.lgm) < c->m) ++a.lgm;
    a.lgL = 0;
    while ((1 << a.lgL) < g.L) ++a.lgL;
    // ceil(2^32 / n) for n >= 2 (n = 1 is handled in the kernel without it)
    a.magic_n = c->n >= 2 ? (unsigned)((((unsigned long long)1 << 32) + (unsigned)c->n - 1) / (unsigned)c->n) : 0u;
    a.stride = g.stride;
    a.nlines = g.nlines;
    a.N = c->N;
    a.tw = fp64 ? (const void*)c->at<double2>(c->lay.tw64) : (const void*)c->at<float2>(c->lay.tw32);
    a.sym_e = fp64 ? (const void*)c->at<double>(c->lay.syme64) : (const void*)c->at<float>(c->lay.syme32);
    a.sym_o = fp64 ? (const void*)c->at<double>(c->lay.symo64) : (const void*)c->at<float>(c->lay.symo32);
    a.lam = fp64 ? (const void*)c->at<double>(c->lay.lam64) : (const void*)c->at<float>(c->lay.lam32);
    a.D = fp64 ? (const void*)c->at<double>(c->lay.D64) : (const void*)c->at<float>(c->lay.D32);
    a.tscale = c->tscale;
    a.omega = c->omega;
    a.pout = c->sc<double2>(c->lay.p1);
    a.pstride = c->lay.pstride;
    a.st = c->st();
    a.hs = c->hs_dev;
    return a;
}

std::string pass_name(bool fp64, const PassVariant& v, int axis) {
    std::string s = fp64 ? "pass64." : "pass32.";
    static const char* inm[] = {"", "basis.", "combo.", "cgs."};
    s += inm[v.inm];
    if (v.ops & P_DST1) s += "dst";
    if (v.ops & P_DIV) s += "_div";
    if (v.ops & P_DST2) s += "_dst";
    if (v.ops & P_SCALE) s += "_scale";
    static const char* zm[] = {"", "_z", "_xset", "_xadd"};
    s += zm[v.zm];
    if (v.ops & P_TOEP) s += (v.ops & ~P_TOEP) ? "_toep" : "toep";
    static const char* om[] = {"", "_first", "_next"};
    s += om[v.outm];
    static const char* fm[] = {"", "_wdots", "_resid"};
    s += fm[v.fin];
    s += ".ax" + std::to_string(axis);
    return s;
}

// Algorithmic bytes of one launch: every vector the pass must read once and
// write once (line data, D, accumulators, basis vectors of the dot products).
double pass_bytes(fnls_ctx* c, bool fp64, const PassVariant& v, const PassArgs& a) {
    const double N = (double)c->N, e = fp64 ? 16.0 : 8.0, dsz = fp64 ? 8.0 : 4.0;
    double b = (v.inm == IN_COMBO) ? c->cur_k * (a.zsum ? (a.z32 ? 8.0 : 16.0) : e) * N
               : (v.inm == IN_CGS) ? (2.0 + (a.basis_j + 1)) * e * N : e * N;
    if ((v.ops & P_SCALE) || v.outm == OUT_ACC_FIRST) b += dsz * N;
    if (v.zm == Z_WRITE) b += e * N;
    if (v.zm == Z_XSET) b += 16.0 * N;
    if (v.zm == Z_XADD) b += (a.first_cycle ? 16.0 : 32.0) * N;
    if (v.outm == OUT_ACC_NEXT) b += e * N;
    if (v.fin == FIN_WRITE && a.out) b += e * N;
    if (v.fin == FIN_WDOTS) b += e * N + (a.basis_j + 1) * e * N;
    if (v.fin == FIN_RESID) b += 32.0 * N + (a.r32 ? 8.0 * N : 0.0);
    return b;
}

// The launch's share of the method's minimal traffic: every vector the
// operation (preconditioned operator, Gram-Schmidt step, end-of-cycle update,
// apply_A / apply_precond / rhs) must read or write, charged once, to the
// launch that first touches it.  Intermediates between the axis passes of
// one operation (the ping-pong vectors, the accumulator, the stored z_j) and
// the later axes' re-reads of the operand cost nothing; the Arnoldi pass
// with the first dot products carries the write of w, one read of w and the
// first sweep over the basis; the recomputed true residual is outside the
// minimal model.
bool intermediate(fnls_ctx* c, const void* p) {
    const char* q = reinterpret_cast<const char*>(p);
    const size_t v = (size_t)c->N * 16;
    auto in = [&](size_t off, size_t len) { return q >= c->scr + off && q < c->scr + off + len; };
    return in(c->lay.t1, v) || in(c->lay.t2, v) || in(c->lay.acc, v) || in(c->lay.Z, c->lay.V - c->lay.Z);
}

double pass_bytes_min(fnls_ctx* c, bool fp64, const PassVariant& v, const PassArgs& a) {
    const double N = (double)c->N, e = fp64 ? 16.0 : 8.0, dsz = fp64 ? 8.0 : 4.0;
    double b = 0.0;
    if (v.inm == IN_COMBO) b += c->cur_k * (a.zsum ? (a.z32 ? 8.0 : 16.0) : e) * N;
    // second Gram-Schmidt sweep (basis, w read and written) and the next
    // step's read of its basis vector, which this pass forms in registers
    else if (v.inm == IN_CGS) b += (3.0 + (a.basis_j + 1)) * e * N;
    else if (v.outm != OUT_ACC_NEXT && a.in && !intermediate(c, a.in)) b += e * N;
    if ((v.ops & P_SCALE) || v.outm == OUT_ACC_FIRST) b += dsz * N;
    if (v.zm == Z_XSET) b += 16.0 * N;
    if (v.zm == Z_XADD) b += (a.first_cycle ? 16.0 : 32.0) * N;
    if (v.fin == FIN_WRITE && a.out && !intermediate(c, a.out)) b += e * N;
    if (v.fin == FIN_WDOTS) b += 2.0 * e * N + (a.basis_j + 1) * e * N;
    return b;
}

// Dynamic LDS of a pass: passes without the Toeplitz product keep one
// buffer per line (the sine transform needs one FFT buffer); at least 4 KB
// (the fused Givens workgroup stages its column there).
size_t pass_lds(const Geo& g, int m, bool fp64, bool two_buffers) {
    const size_t elem = fp64 ? 16 : 8;
    int pa = 0, ls = 0;
    line_layout(m, g.L, fp64, two_buffers, &pa, &ls);
    const size_t table = (size_t)(m >= 4 ? m / 4 : 1) * elem;
    const size_t lds = (size_t)g.L * ls * elem + table + (size_t)g.L * (8 + elem / 2);
    // the line buffers also hold the reduction sums at the end of the pass:
    // (kMaxRestart + 2) complex values per wavefront
    const size_t red = (size_t)(kMaxRestart + 2) * ((g.G * g.L + 63) / 64) * 16;
    return std::max<size_t>(std::max(lds, red), 4096);
}

int run_pass(fnls_ctx* c, bool fp64, int axis, PassVariant v, PassArgs& a, const Geo& g) {
    v.rmax = g.rmax;
    const size_t lds = pass_lds(g, c->m, fp64, (v.ops & P_TOEP) != 0);
    line_layout(c->m, g.L, fp64, (v.ops & P_TOEP) != 0, &a.pa, &a.ls);
    const LaunchEvents* te = c->timing ? timing_begin(c, pass_name(fp64, v, axis), pass_bytes(c, fp64, v, a),
                                                         pass_bytes_min(c, fp64, v, a)) : nullptr;
    hipError_t e = launch_pass(fp64 ? 1 : 0, v, a, g.blocks + (a.gfuse ? 1 : 0), lds, c->stream, te);
    if (e != hipSuccess) timing_failed(c, te);
    if (e != hipSuccess)
        return set_err(c, FNLS_ERR_HIP, "pass launch (axis %d, ops %d) failed: %s", axis, v.ops, hipGetErrorString(e));
    return FNLS_OK;
}

// Working vectors typed for the precision of the transform kernels.
struct Bufs {
    void* t1;
    void* t2;
    void* zbase;  // preconditioned basis vectors z_j (typed), slot j at zbase + j N
    void* acc;
    void* v0;     // basis vector 0
    void* vbase;  // basis vectors 1..
};

Bufs bufs(fnls_ctx* c, bool fp64, const void* v0_fp64) {
    Bufs b;
    b.t1 = c->sc<char>(c->lay.t1);
    b.t2 = c->sc<char>(c->lay.t2);
    b.zbase = c->sc<char>(c->lay.Z);
    b.acc = c->sc<char>(c->lay.acc);
    if (fp64) {
        b.v0 = const_cast<void*>(v0_fp64);
        b.vbase = c->sc<char>(c->lay.V);
    } else {
        float2* V32 = c->sc<float2>(c->lay.V);
        b.v0 = V32;
        b.vbase = V32 + c->N;
    }
    return b;
}

// Sine-transform passes that precede the last one: axes d-1 .. 1 forward,
// axis 0 transform-divide-transform, axes 1 .. d-2 back.  The first pass reads
// `src` with input mode `inm`; returns the buffer holding the result.
// scale_second (Arnoldi step, d >= 2): the first pass transforms the raw
// basis vector, the second applies the basis scale sigma_j, and an event
// marks the end of the first pass; givens: the first pass also carries the
// previous iteration's Givens step in an extra workgroup.
// part: 0 all passes, 1 the first pass only, 2 all passes after the first.
int precond_front(fnls_ctx* c, bool fp64, int inm, const void* src, int basis_j, Bufs& b, void** result,
                  int check_active, bool scale_second = false, bool givens = false, int part = 0) {
    const bool fused = scale_second;
    const int d = c->d;
    void* cur_in = const_cast<void*>(src);
    int cur_mode = fused ? IN_PLAIN : inm;
    void* pingpong[2] = {b.t1, b.t2};
    int pp = 0;
    int npass = 0;
    auto step = [&](int axis, int ops) -> int {
        Geo g = pass_geo(d, c->n, axis, fp64, c->max_dyn_lds, c->pcfg);
        PassArgs a = base_args(c, fp64, axis, g);
        a.in = cur_in;
        a.v0 = b.v0;
        a.vbase = b.vbase;
        a.basis_j = basis_j;
        a.out = pingpong[pp];
        a.check_active = check_active;
        if (npass == 0 && givens) {
            a.gfuse = 1;
            a.gpin = c->sc<double2>(c->lay.p3);
            a.gpin_nb = stream_blocks(c->N);
            a.gpin_stride = c->lay.pstride;
        }
        PassVariant v{cur_mode, ops, Z_NONE, OUT_LINE, FIN_WRITE};
        const bool launch = (part == 0) || (part == 1 ? npass == 0 : npass >= 1);
        int rc = launch ? run_pass(c, fp64, axis, v, a, g) : FNLS_OK;
        cur_in = pingpong[pp];
        pp ^= 1;
        cur_mode = (fused && npass == 0) ? inm : IN_PLAIN;
        ++npass;
        return rc;
    };
    int rc;
    for (int ax = d - 1; ax >= 1; --ax)
        if ((rc = step(ax, P_DST1)) != FNLS_OK) return rc;
    if ((rc = step(0, P_DST1 | P_DIV | P_DST2)) != FNLS_OK) return rc;
    for (int ax = 1; ax <= d - 2; ++ax)
        if ((rc = step(ax, P_DST1)) != FNLS_OK) return rc;
    *result = cur_in;
    return FNLS_OK;
}

// Toeplitz passes for axes d-2 .. 0 after the first one (which produced acc):
// out = acc + cT T_axis x, the last one with final mode `fin`.
int toeplitz_tail(fnls_ctx* c, bool fp64, const void* x, void* acc, int fin, void* final_out, PassArgs tmpl,
                  int check_active) {
    const int d = c->d;
    for (int ax = d - 2; ax >= 0; --ax) {
        Geo g = pass_geo(d, c->n, ax, fp64, c->max_dyn_lds, c->pcfg);
        PassArgs a = base_args(c, fp64, ax, g);
        a.in = x;
        a.acc_in = acc;
        a.cT = -1.0;
        a.check_active = check_active;
        a.guard_k = tmpl.guard_k;
        const bool last = (ax == 0);
        a.out = last ? final_out : acc;
        int f = last ? fin : FIN_WRITE;
        a.v0 = tmpl.v0;
        a.vbase = tmpl.vbase;
        a.basis_j = tmpl.basis_j;
        a.b64 = tmpl.b64;
        a.r64 = tmpl.r64;
        a.r32 = tmpl.r32;
        a.ir = tmpl.ir;
        if (tmpl.pout) a.pout = tmpl.pout;
        PassVariant v{IN_PLAIN, P_TOEP, Z_NONE, OUT_ACC_NEXT, f};
        int rc = run_pass(c, fp64, ax, v, a, g);
        if (rc != FNLS_OK) return rc;
    }
    return FNLS_OK;
}

// y = (cD D + i ci I + cT T_d) x in the precision of fp64 (complex128 or
// complex64 vectors; used by apply_A, rhs and the complex64 apply_A).
int matvec(fnls_ctx* c, bool fp64, const void* x, void* y, double cD, double ci, double cT) {
    const int d = c->d;
    Geo g = pass_geo(d, c->n, d - 1, fp64, c->max_dyn_lds, c->pcfg);
    PassArgs a = base_args(c, fp64, d - 1, g);
    a.in = x;
    a.cD = cD;
    a.ci = ci;
    a.cT = cT;
    a.out = (d == 1) ? y : c->sc<char>(c->lay.acc);
    PassVariant v{IN_PLAIN, P_TOEP, Z_NONE, OUT_ACC_FIRST, FIN_WRITE};
    int rc = run_pass(c, fp64, d - 1, v, a, g);
    if (rc != FNLS_OK || d == 1) return rc;
    void* acc = c->sc<char>(c->lay.acc);
    for (int ax = d - 2; ax >= 0; --ax) {
        Geo g2 = pass_geo(d, c->n, ax, fp64, c->max_dyn_lds, c->pcfg);
        PassArgs a2 = base_args(c, fp64, ax, g2);
        a2.in = x;
        a2.acc_in = acc;
        a2.cT = cT;
        a2.out = (ax == 0) ? y : acc;
        PassVariant v2{IN_PLAIN, P_TOEP, Z_NONE, OUT_ACC_NEXT, FIN_WRITE};
        rc = run_pass(c, fp64, ax, v2, a2, g2);
        if (rc != FNLS_OK) return rc;
    }
    return FNLS_OK;
}

int matvec64(fnls_ctx* c, const void* x, void* y, double cD, double ci, double cT) {
    return matvec(c, true, x, y, cD, ci, cT);
}

// One-workgroup decision / reduction kernel (k_finish).
int run_finish(fnls_ctx* c, const StreamArgs& s, const char* name) {
    const LaunchEvents* te = c->timing ? timing_begin(c, name, 16.0 * s.pin_nb, 0.0) : nullptr;
    hipError_t e = launch_finish(s, c->stream, te);
    if (e != hipSuccess) timing_failed(c, te);
    if (e != hipSuccess) return set_err(c, FNLS_ERR_HIP, "finish launch failed: %s", hipGetErrorString(e));
    return FNLS_OK;
}

// When the producer of s.pin had many workgroups, pre-sum its nv partials in
// kReduceChunks contiguous chunks (one workgroup each, fixed order) so that
// consumer workgroups read kReduceChunks entries per value.
int reduce_if_wide(fnls_ctx* c, StreamArgs& s, int nv) {
    if (s.pin_nb <= kRedundantMax) return FNLS_OK;
    if (nv > kMaxRestart + 2) return set_err(c, FNLS_ERR_INVALID_ARG, "reduction of %d values exceeds px", nv);
    StreamArgs r = s;
    r.nv = nv;
    r.pout = c->sc<double2>(c->lay.px);
    const LaunchEvents* te = c->timing ? timing_begin(c, "reduce.chunks", 16.0 * nv * s.pin_nb, 0.0) : nullptr;
    hipError_t e = launch_reduce_chunks(r, kReduceChunks, c->stream, te);
    if (e != hipSuccess) {
        timing_failed(c, te);
        return set_err(c, FNLS_ERR_HIP, "reduction launch failed: %s", hipGetErrorString(e));
    }
    s.pin = c->sc<double2>(c->lay.px);
    s.pin_nb = kReduceChunks;
    s.pin_stride = kReduceChunks;
    return FNLS_OK;
}

// Blocks of the pass that applies the second Gram-Schmidt update (fused with
// the next step's first sine transform along the contiguous axis): the
// producers of the ||w||^2 partials that the Givens step sums.
int cgs_dst_blocks(fnls_ctx* c, bool fp64) {
    return pass_geo(c->d, c->n, c->d - 1, fp64, c->max_dyn_lds, c->pcfg).blocks;
}

// The second Gram-Schmidt update runs fused with the next Arnoldi step's
// first sine transform unless step j is the last of the cycle's length.
bool cgs_fused(fnls_ctx* c, int j) { return c->d >= 2 && j + 1 < c->restart_cur; }

// One Arnoldi step j: w = A Ptilde^{-1} v_j into basis slot j+1, first-round
// dot products, then the two Gram-Schmidt updates.
// d >= 2: the basis vector is stored raw (v_j / sigma_j).  Its sine transform
// along the contiguous axis d-1 comes from the previous step's second
// Gram-Schmidt update, which runs fused with it (step 0: a plain pass of
// b or r), so step j starts with the remaining front passes of the
// preconditioner (the first of them carries step j-1's Givens step when
// fused); the pass that ends the preconditioner applies sigma_j.
// part (d >= 2, fused Givens steps, j >= 1): 0 the whole step, its first
// launch carrying step j-1's Givens step; 1 = only step j-1's Givens step,
// as a one-workgroup launch (issued ahead of a predicted stop, where the
// step itself is probably not needed); 2 = the whole step without it.
int run_givens(fnls_ctx* c, int nb);

int arnoldi_step(fnls_ctx* c, bool fp64, Bufs& b, int j, int part = 0) {
    const int d = c->d;
    const size_t esz = fp64 ? 16 : 8;
    void* vj = (j == 0) ? b.v0 : (void*)((char*)b.vbase + (size_t)(j - 1) * c->N * esz);
    void* w = (char*)b.vbase + (size_t)j * c->N * esz;
    int rc;
    if (d == 1) {
        Geo g = pass_geo(d, c->n, 0, fp64, c->max_dyn_lds, c->pcfg);
        PassArgs a = base_args(c, fp64, 0, g);
        a.in = vj;
        a.v0 = b.v0;
        a.vbase = b.vbase;
        a.basis_j = j;
        a.out = w;
        a.cD = 1.0;
        a.ci = 1.0;
        a.cT = -1.0;
        a.check_active = 1;
        PassVariant v{IN_BASIS, P_DST1 | P_DIV | P_DST2 | P_SCALE | P_TOEP, Z_NONE, OUT_ACC_FIRST, FIN_WDOTS};
        if ((rc = run_pass(c, fp64, 0, v, a, g)) != FNLS_OK) return rc;
    } else {
        // front passes after the contiguous axis: axes d-2 .. 1 forward,
        // axis 0 transform-divide-transform, axes 1 .. d-2 back; t1 holds
        // the contiguous axis's transform of the raw basis vector
        struct Front { int axis, ops; };
        Front fr[5];
        int nf = 0;
        for (int ax = d - 2; ax >= 1; --ax) fr[nf++] = {ax, P_DST1};
        fr[nf++] = {0, P_DST1 | P_DIV | P_DST2};
        for (int ax = 1; ax <= d - 2; ++ax) fr[nf++] = {ax, P_DST1};
        void* pp[2] = {b.t1, b.t2};
        const bool givens = c->fuse != 0 && j >= 1 && part == 0;
        if (part == 1) return run_givens(c, cgs_dst_blocks(c, fp64));
        if (j == 0) {
            // step 0: the contiguous axis's transform of the raw start vector
            Geo g = pass_geo(d, c->n, d - 1, fp64, c->max_dyn_lds, c->pcfg);
            PassArgs a = base_args(c, fp64, d - 1, g);
            a.in = vj;
            a.out = b.t1;
            a.check_active = 1;
            PassVariant v{IN_PLAIN, P_DST1, Z_NONE, OUT_LINE, FIN_WRITE};
            if ((rc = run_pass(c, fp64, d - 1, v, a, g)) != FNLS_OK) return rc;
        }
        for (int k = 0; k < nf; ++k) {
            Geo g = pass_geo(d, c->n, fr[k].axis, fp64, c->max_dyn_lds, c->pcfg);
            PassArgs a = base_args(c, fp64, fr[k].axis, g);
            a.in = pp[k & 1];
            a.out = pp[(k + 1) & 1];
            a.check_active = 1;
            if (k == 0 && givens) {
                a.gfuse = 1;
                a.gpin = c->sc<double2>(c->lay.p3);
                a.gpin_nb = cgs_dst_blocks(c, fp64);
                a.gpin_stride = c->lay.pstride;
            }
            PassVariant v{IN_PLAIN, fr[k].ops, Z_NONE, OUT_LINE, FIN_WRITE};
            if ((rc = run_pass(c, fp64, fr[k].axis, v, a, g)) != FNLS_OK) return rc;
        }
        // last sine transform (after the basis scale sigma_j), the
        // preconditioner's diagonal scale (z_j kept) and the first Toeplitz axis
        Geo g = pass_geo(d, c->n, d - 1, fp64, c->max_dyn_lds, c->pcfg);
        PassArgs a = base_args(c, fp64, d - 1, g);
        a.in = pp[nf & 1];
        a.basis_j = j;
        void* zj = (char*)b.zbase + (size_t)j * c->N * esz;
        a.zout = zj;
        a.out = b.acc;
        a.cD = 1.0;
        a.ci = 1.0;
        a.cT = -1.0;
        a.check_active = 1;
        PassVariant v{IN_BASIS, P_DST1 | P_SCALE | P_TOEP, Z_WRITE, OUT_ACC_FIRST, FIN_WRITE};
        if ((rc = run_pass(c, fp64, d - 1, v, a, g)) != FNLS_OK) return rc;
        PassArgs tmpl;
        std::memset(&tmpl, 0, sizeof tmpl);
        tmpl.v0 = b.v0;
        tmpl.vbase = b.vbase;
        tmpl.basis_j = j;
        if ((rc = toeplitz_tail(c, fp64, zj, b.acc, FIN_WDOTS, w, tmpl, 1)) != FNLS_OK) return rc;
    }
    StreamArgs s;
    std::memset(&s, 0, sizeof s);
    s.N = c->N;
    s.w = w;
    s.v0 = b.v0;
    s.vbase = b.vbase;
    s.nv = j + 1;
    s.pstride = c->lay.pstride;
    s.st = c->st();
    s.hs = c->hs_dev;
    s.check_active = 1;
    const int nb1 = pass_geo(d, c->n, 0, fp64, c->max_dyn_lds, c->pcfg).blocks;
    const int blocks = stream_blocks(c->N);
    const double esz_d = fp64 ? 16.0 : 8.0;
    const double cgs_bytes = (2.0 + (j + 1)) * esz_d * (double)c->N;
    // minimal model: three sweeps over the basis with w read once per sweep
    // and written once (the first sweep is in the Arnoldi pass)
    const double dots_min = (1.0 + (j + 1)) * esz_d * (double)c->N;
    // first Gram-Schmidt update (consumes the dots of the last pass)
    s.pin = c->sc<double2>(c->lay.p1);
    s.pin_nb = nb1;
    s.pin_stride = c->lay.pstride;
    if ((rc = reduce_if_wide(c, s, j + 2)) != FNLS_OK) return rc;
    s.pout = c->sc<double2>(c->lay.p2);
    const LaunchEvents* te = c->timing ? timing_begin(c, fp64 ? "cgs64.update_dots" : "cgs32.update_dots", cgs_bytes, dots_min) : nullptr;
    hipError_t e = launch_cgs(fp64 ? 1 : 0, 0, s, blocks, c->stream, te);
    if (e != hipSuccess) timing_failed(c, te);
    if (e != hipSuccess) return set_err(c, FNLS_ERR_HIP, "cgs launch failed: %s", hipGetErrorString(e));
    // second update (reorthogonalisation)
    s.pin = c->sc<double2>(c->lay.p2);
    s.pin_nb = blocks;
    s.pin_stride = c->lay.pstride;
    if ((rc = reduce_if_wide(c, s, j + 1)) != FNLS_OK) return rc;
    int norm_nb = blocks;
    if (cgs_fused(c, j)) {
        // fused with the next step's first sine transform along the
        // contiguous axis: w updated in place, ||w||^2 partials, t1
        Geo g = pass_geo(d, c->n, d - 1, fp64, c->max_dyn_lds, c->pcfg);
        PassArgs a = base_args(c, fp64, d - 1, g);
        a.in = w;
        a.v0 = b.v0;
        a.vbase = b.vbase;
        a.basis_j = j;
        a.cgs_pin = s.pin;
        a.cgs_nb = s.pin_nb;
        a.cgs_stride = s.pin_stride;
        a.pout = c->sc<double2>(c->lay.p3);
        a.out = b.t1;
        a.check_active = 1;
        PassVariant v{IN_CGS, P_DST1, Z_NONE, OUT_LINE, FIN_WRITE};
        if ((rc = run_pass(c, fp64, d - 1, v, a, g)) != FNLS_OK) return rc;
        norm_nb = g.blocks;
    } else {
        s.pout = c->sc<double2>(c->lay.p3);
        te = c->timing ? timing_begin(c, fp64 ? "cgs64.update_norm" : "cgs32.update_norm", cgs_bytes, cgs_bytes) : nullptr;
        e = launch_cgs(fp64 ? 1 : 0, 1, s, blocks, c->stream, te);
        if (e != hipSuccess) timing_failed(c, te);
        if (e != hipSuccess) return set_err(c, FNLS_ERR_HIP, "cgs launch failed: %s", hipGetErrorString(e));
    }
    // Givens step and stopping decision (fused: in the next iteration's first pass)
    if (c->fuse && d >= 2 && j + 1 < c->restart_cur) return FNLS_OK;
    return run_givens(c, norm_nb);
}

// The Givens step of the current Arnoldi iteration as a one-workgroup launch,
// from the nb partials of ||w||^2 in p3.
int run_givens(fnls_ctx* c, int nb) {
    StreamArgs s;
    std::memset(&s, 0, sizeof s);
    s.N = c->N;
    s.pstride = c->lay.pstride;
    s.st = c->st();
    s.hs = c->hs_dev;
    s.check_active = 1;
    s.pin = c->sc<double2>(c->lay.p3);
    s.pin_nb = nb;
    s.pin_stride = c->lay.pstride;
    int rc = reduce_if_wide(c, s, 1);
    if (rc != FNLS_OK) return rc;
    s.mode = 1;
    return run_finish(c, s, "finish.givens");
}

// End of a cycle: x (+)= Ptilde^{-1} (sum_i y_i v_i).  FP64: the recomputed
// residual r = b - A x follows in the same passes.  FP32 (IR): x is updated
// in FP64 from the FP32 correction, then the FP64 residual chain runs.
// guard 2: enqueued ahead of the stopping decision; every launch returns at
// once unless, by the time it runs, the cycle has stopped with guard_k basis
// vectors (the stop the host predicted).
int cycle_final_passes(fnls_ctx* c, bool fp64, Bufs& b, const void* b64, void* x, int first, int guard,
                       int guard_k);

int cycle_final(fnls_ctx* c, bool fp64, Bufs& b, const void* b64, void* x, int first, int guard = 0,
                int guard_k = 0) {
    int rc = cycle_final_passes(c, fp64, b, b64, x, first, guard, guard_k);
    if (rc != FNLS_OK) return rc;
    StreamArgs s;
    std::memset(&s, 0, sizeof s);
    s.check_active = guard;
    s.guard_k = guard_k;
    s.pin = c->sc<double2>(c->lay.pr);
    s.pin_nb = pass_geo(c->d, c->n, 0, true, c->max_dyn_lds, c->pcfg).blocks;
    s.pin_stride = c->lay.pstride;
    s.pstride = c->lay.pstride;
    s.st = c->st();
    s.hs = c->hs_dev;
    s.mode = 2;
    s.ir = fp64 ? 0 : 1;
    if ((rc = reduce_if_wide(c, s, 1)) != FNLS_OK) return rc;
    return run_finish(c, s, "finish.residual");
}

int cycle_final_passes(fnls_ctx* c, bool fp64, Bufs& b, const void* b64, void* x, int first, int guard,
                       int guard_k) {
    const int d = c->d;
    double2* r64 = c->sc<double2>(c->lay.r64);
    float2* r32 = fp64 ? nullptr : c->sc<float2>(c->lay.V);
    int rc;
    if (d == 1) {
        // one line: x (+)= Ptilde^{-1} (V y) in a single pass (FP64: with the residual)
        Geo g = pass_geo(d, c->n, 0, fp64, c->max_dyn_lds, c->pcfg);
        PassArgs a = base_args(c, fp64, 0, g);
        a.check_active = guard;
        a.guard_k = guard_k;
        a.v0 = b.v0;
        a.vbase = b.vbase;
        a.x64 = (double2*)x;
        a.first_cycle = first;
        if (fp64) {
            a.cD = 1.0;
            a.ci = 1.0;
            a.cT = -1.0;
            a.b64 = (const double2*)b64;
            a.r64 = r64;
            a.pout = c->sc<double2>(c->lay.pr);
            PassVariant v{IN_COMBO, P_DST1 | P_DIV | P_DST2 | P_SCALE | P_TOEP, Z_XADD, OUT_ACC_FIRST, FIN_RESID};
            return run_pass(c, true, 0, v, a, g);
        }
        PassVariant v{IN_COMBO, P_DST1 | P_DIV | P_DST2 | P_SCALE, Z_XADD, OUT_LINE, FIN_WRITE};
        if ((rc = run_pass(c, false, 0, v, a, g)) != FNLS_OK) return rc;
    }
    // FP64 residual r = b - A x (IR: with its complex64 copy as the next basis vector 0)
    Geo g = pass_geo(d, c->n, d - 1, true, c->max_dyn_lds, c->pcfg);
    PassArgs a = base_args(c, true, d - 1, g);
    a.check_active = guard;
    a.guard_k = guard_k;
    a.in = x;
    a.cD = 1.0;
    a.ci = 1.0;
    a.cT = -1.0;
    const int ir = fp64 ? 0 : 1;
    if (d == 1) {
        a.b64 = (const double2*)b64;
        a.r64 = r64;
        a.r32 = r32;
        a.ir = ir;
        a.pout = c->sc<double2>(c->lay.pr);
        PassVariant v{IN_PLAIN, P_TOEP, Z_NONE, OUT_ACC_FIRST, FIN_RESID};
        return run_pass(c, true, 0, v, a, g);
    }
    // d >= 2: the first axis pass of the residual also forms the update
    // x (+)= sum_k y_k z_k over the preconditioned basis stored by the Arnoldi
    // passes (equal to Ptilde^{-1} (V y) by linearity), in FP64, and takes the
    // new x as its Toeplitz operand
    void* acc64 = c->sc<char>(c->lay.acc);
    a.out = acc64;
    a.in = nullptr;
    a.zsum = 1;
    a.z32 = fp64 ? 0 : 1;
    a.vbase = b.zbase;
    a.x64 = (double2*)x;
    a.first_cycle = first;
    PassVariant v{IN_COMBO, P_TOEP, Z_XADD, OUT_ACC_FIRST, FIN_WRITE};
    if ((rc = run_pass(c, true, d - 1, v, a, g)) != FNLS_OK) return rc;
    PassArgs tmpl;
    std::memset(&tmpl, 0, sizeof tmpl);
    tmpl.b64 = (const double2*)b64;
    tmpl.r64 = r64;
    tmpl.r32 = r32;
    tmpl.ir = ir;
    tmpl.pout = c->sc<double2>(c->lay.pr);
    tmpl.guard_k = guard_k;
    return toeplitz_tail(c, true, x, acc64, FIN_RESID, nullptr, tmpl, guard);
}

int check_ready(fnls_ctx* c) {
    if (!c) return FNLS_ERR_INVALID_ARG;
    if (!c->assembled) return set_err(c, FNLS_ERR_STATE, "fnls_assemble has not been called");
    return FNLS_OK;
}

int check_solve_ready(fnls_ctx* c) {
    int rc = check_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!c->have_D) return set_err(c, FNLS_ERR_STATE, "fnls_precond_setup has not been called");
    return FNLS_OK;
}

// Wait for event k and return a snapshot of the host status.
// Wait until the device has reported the status after `target` iterations
// in total (hs->total >= target) or the end of the solve, and copy it.  The
// host polls the seqlock HostStatus::seq (reports of this solve carry values
// in (seq_base, seq_base + kSeqStride)) instead of waiting on events: an
// event record is a marker packet that leaves the device idle for several
// microseconds between two kernels, and there were two per Arnoldi iteration.
// After 20 ms without the report the stream is queried every 5 ms, so a
// device error ends the wait, and so does a drained stream without the
// awaited report.  (Not sooner: with a query every few microseconds the
// kernel trace showed the same gap again, before every iteration's first pass.)
constexpr unsigned kSeqStride = 1u << 24;

// A published sequence value of the current solve: even (complete) and in
// (seq_base, seq_base + kSeqStride), modulo 2^32.
bool seq_in_window(unsigned seq_base, unsigned s) {
    const unsigned rel = s - seq_base;
    return (s & 1u) == 0 && rel != 0 && rel < kSeqStride;
}

// The host takes a copied report when the sequence value read before the
// copy is a complete report of this solve, the value read after it is the
// same (no report was written in between), and the report covers the
// awaited iteration total (or ends the solve).
bool report_accepted(unsigned seq_base, unsigned s1, unsigned s2, int total, int done, int target) {
    return seq_in_window(seq_base, s1) && s1 == s2 && (total >= target || done != 0);
}

int wait_report(fnls_ctx* c, int target, HostStatus* out) {
    using clock = std::chrono::steady_clock;
    if (c->poll_delay_us > 0) std::this_thread::sleep_for(std::chrono::microseconds(c->poll_delay_us));
    bool drained = false;
    auto next_query = clock::now() + std::chrono::milliseconds(20);
    for (unsigned spin = 1;; ++spin) {
        const unsigned s1 = __atomic_load_n(&c->hs->seq, __ATOMIC_ACQUIRE);
        if (seq_in_window(c->seq_base, s1)) {
            std::memcpy(out, (const void*)c->hs, sizeof *out);
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
            const unsigned s2 = __atomic_load_n(&c->hs->seq, __ATOMIC_RELAXED);
            if (report_accepted(c->seq_base, s1, s2, out->total, out->done, target)) return FNLS_OK;
        }
        if (drained) return set_err(c, FNLS_ERR_HIP, "the device finished without reporting iteration %d", target);
        if ((spin & 1023u) == 0 && clock::now() >= next_query) {
            const hipError_t q = hipStreamQuery(c->stream);
            if (q == hipSuccess) drained = true;   // look once more: every write has landed
            else if (q != hipErrorNotReady) return set_err(c, FNLS_ERR_HIP, "stream: %s", hipGetErrorString(q));
            next_query = clock::now() + std::chrono::milliseconds(5);
        }
        __builtin_ia32_pause();
    }
}

// Arguments of the end-of-cycle passes, for enqueueing them ahead.
struct FinalArgs {
    const void* b64;
    void* x;
    int first;
};

// One GMRES cycle (iterations until the device reports a stop), with up to
// `lookahead` iterations enqueued beyond the one whose status is awaited.
// Returns FNLS_OK and sets *done when the solve ended before the cycle
// started (b == 0 or non-finite b).  *final_issued = 1 when the end-of-cycle
// passes (cycle_final) for the actual stop are already enqueued.  `cycle`:
// the number of cycles of this solve before this one (residuals reported).
int run_cycle(fnls_ctx* c, bool fp64, Bufs& b, int restart, int lookahead, int total_before, int* total_after,
              int* done, const FinalArgs& fin, int* final_issued, HostStatus* stop_status, int cycle) {
    int issued = 0, waited = 0;
    int final_k = -1;   // cycle size for which the end-of-cycle passes are enqueued
    *done = 0;
    *final_issued = 0;
    HostStatus hs;
    // first timing record of every issued iteration: launches of iterations
    // that the device skipped (issued ahead of the stopping decision) carry
    // no algorithmic bytes
    std::vector<size_t> rec_first;
    auto unbill = [&](int active) {
        if (!c->timing) return;
        for (int i = std::max(0, active); i < issued; ++i)
            for (size_t r = rec_first[i]; r < c->recs.size(); ++r) c->recs[r].bytes = c->recs[r].bytes_min = 0.0;
    };
    // fused Givens: the status of iteration j is written by the first pass of
    // iteration j + 1, which the lookahead has issued before the wait
    c->restart_cur = restart;
    c->fuse = (lookahead >= 1 && c->d >= 2 && cgs_dst_blocks(c, fp64) <= kRedundantMax &&
               stream_blocks(c->N) <= kRedundantMax) ? 1 : 0;
    // With the fused Givens step, iteration J's first pass decides whether
    // iteration J - 1 stopped the cycle.  When the estimates of the finished
    // iterations, extrapolated at their last rate, predict that stop, only
    // iteration J - 1's Givens step is issued ahead (one workgroup, not the
    // first pass of an iteration that is probably not needed); iteration J
    // follows whole once the status shows that the cycle goes on (a short
    // host round trip).
    std::vector<char> partial((size_t)restart + 1, 0);
    double est_last = 1.0, est_prev = 1.0, tol_last = 0.0;
    while (true) {
        while (issued < restart && issued <= waited + lookahead) {
            // an iteration whose predecessor was issued only as its Givens
            // step must wait for that predecessor (whose first pass would
            // have carried the next Givens step)
            if (issued >= 1 && partial[issued - 1]) break;
            rec_first.push_back(c->recs.size());
            bool first_only = false;
            // (a rate needs two estimates of this cycle: the drop from the
            // initial residual to the first estimate is much steeper than
            // later ones and predicted stops one iteration early)
            if (c->fuse && issued >= 1 && waited >= 2 && est_prev > 0.0 && tol_last > 0.0) {
                const double rate = est_last / est_prev;
                double pred = est_last;
                for (int k = waited; k < issued; ++k) pred *= rate;   // estimate of iteration issued - 1
                first_only = rate < 1.0 && pred < tol_last;
            }
            int rc = arnoldi_step(c, fp64, b, issued, first_only ? 1 : 0);
            if (rc != FNLS_OK) return rc;
            if (first_only) {
                partial[issued] = 1;
                ++c->stats.stop_predictions;
                // the predicted stop leaves a cycle of `issued` iterations:
                // enqueue its end now, guarded, so the device need not wait
                // for the host to see the stop (the launches return at once
                // unless the cycle stops with exactly that many: with more
                // than one iteration in flight an earlier one may stop it)
                if (!c->timing) {
                    if ((rc = cycle_final(c, fp64, b, fin.b64, fin.x, fin.first, 2, issued)) != FNLS_OK) return rc;
                    final_k = issued;
                }
            }
            ++issued;
        }
        // the status of iteration `waited` (with the fused Givens step it is
        // written by the first pass of iteration waited + 1, already issued)
        int rc = wait_report(c, total_before + waited + 1, &hs);
        if (rc != FNLS_OK) return rc;
        ++waited;
        if (hs.outer > cycle) {
            // this cycle's end, enqueued behind its predicted stop, has run
            // and reported the residual's decision before the host read the
            // stop report: the cycle stopped where predicted
            if (hs.total - total_before != final_k)
                return set_err(c, FNLS_ERR_HIP, "status report of cycle %d out of order", cycle);
            ++c->stats.late_reads;
            break;
        }
        if (hs.done) {
            *done = 1;
            unbill(0);
            return FNLS_OK;
        }
        if (hs.stopped || waited >= restart) break;
        est_prev = est_last;
        est_last = hs.est;
        tol_last = hs.tol;
        // the cycle goes on: issue the iteration whose Givens step alone was issued ahead
        if (partial[waited]) {
            partial[waited] = 0;
            if ((rc = arnoldi_step(c, fp64, b, waited, 2)) != FNLS_OK) return rc;
        }
    }
    *total_after = hs.total;
    c->cur_k = hs.total - total_before;   // iterations of this cycle
    *final_issued = (c->cur_k == final_k) ? 1 : 0;
    c->stats.iterations += c->cur_k;
    c->stats.ends_ahead += *final_issued;
    if (final_k > 0 && c->cur_k < final_k) ++c->stats.early_stops;
    *stop_status = hs;
    unbill(c->cur_k);
    // let any speculative (inactive) iterations drain before the final passes
    return FNLS_OK;
}

void fill_info(fnls_ctx* c, fnls_info* info, int status) {
    if (!info) return;
    const HostStatus& hs = *c->hs;
    std::memset(info, 0, sizeof *info);
    info->iters = hs.total;
    info->outer_iters = hs.outer;
    info->status = status;
    info->breakdown = hs.breakdown;
    info->relres_true = hs.relres;
    const int nh = std::min(64, hs.total);
    for (int i = 0; i < nh; ++i) info->relres_hist[i] = hs.hist[i];
}

int solve_impl(fnls_ctx* c, const fnls_c128* b, fnls_c128* x, const fnls_opts* o, fnls_info* info) {
    const bool fp64 = (o->precision == FNLS_FP64);
    const TraceRange trace(fp64 ? "fnls.solve.fp64" : "fnls.solve.fp32_ir");
    const int restart = o->restart;
    c->seq_base += kSeqStride;
    c->poll_delay_us = o->poll_delay_us;
    ++c->stats.solves;
    StreamArgs s;
    std::memset(&s, 0, sizeof s);
    s.N = c->N;
    s.b64 = reinterpret_cast<const double2*>(b);
    s.r32 = fp64 ? nullptr : c->sc<float2>(c->lay.V);
    s.pout = c->sc<double2>(c->lay.pr);
    s.pstride = c->lay.pstride;
    s.st = c->st();
    s.hs = c->hs_dev;
    {
        const LaunchEvents* te = c->timing ? timing_begin(c, "prepare", (fp64 ? 16.0 : 24.0) * (double)c->N,
                                                              (fp64 ? 16.0 : 24.0) * (double)c->N) : nullptr;
        hipError_t e = launch_prepare(s, stream_blocks(c->N), c->stream, te);
        if (e != hipSuccess) timing_failed(c, te);
        if (e != hipSuccess) return set_err(c, FNLS_ERR_HIP, "prepare launch failed: %s", hipGetErrorString(e));
        StreamArgs f = s;
        f.pin = c->sc<double2>(c->lay.pr);
        f.pin_nb = stream_blocks(c->N);
        f.pin_stride = c->lay.pstride;
        f.mode = 0;
        f.cfg_tol = fp64 ? o->tol : o->inner_tol;
        f.cfg_outer_tol = o->tol;
        f.cfg_restart = restart;
        f.cfg_maxit = o->maxit;
        f.cfg_fixed_iters = fp64 ? o->fixed_iters : 0;
        f.cfg_max_outer = fp64 ? (1 << 30) : o->max_outer;
        f.cfg_seq0 = c->seq_base;
        int rc0 = reduce_if_wide(c, f, 1);
        if (rc0 == FNLS_OK) rc0 = run_finish(c, f, "finish.prepare");
        if (rc0 != FNLS_OK) return rc0;
    }
    int first = 1;
    int status = FNLS_OK;
    int total = 0;        // iterations so far, as last reported by the device
    bool ahead = false;   // this cycle was enqueued before the last residual's decision was seen
    double relres_prev = 1.0;
    int cycle = 0;        // cycles of this solve whose end is enqueued
    while (true) {
        const TraceRange trace_cycle("fnls.cycle");
        Bufs bf = bufs(c, fp64, first ? (const void*)b : (const void*)c->sc<double2>(c->lay.r64));
        int done = 0, final_issued = 0;
        const FinalArgs fin{b, x, first};
        HostStatus stop;
        int rc = run_cycle(c, fp64, bf, restart, std::max(0, o->lookahead), total, &total, &done, fin,
                           &final_issued, &stop, cycle);
        if (rc != FNLS_OK) return rc;
        if (done && !ahead) {
            // b == 0 (x = 0) or non-finite b
            if (c->hs->nonfinite) return set_err(c, FNLS_ERR_NONFINITE, "non-finite value in b");
            HIPCHK(c, hipMemsetAsync(x, 0, (size_t)c->N * 16, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            fill_info(c, info, FNLS_OK);
            if (info) info->relres_true = 0.0;
            return FNLS_OK;
        }
        if (!done) {
            if (!final_issued && (rc = cycle_final(c, fp64, bf, b, x, first)) != FNLS_OK) return rc;
            ++c->stats.cycles;
            first = 0;
            // the residual's decision may already be in (end enqueued ahead)
            const bool decided = stop.outer > cycle;
            ++cycle;
            // When the stop estimate leaves the outer tolerance clearly unmet
            // (the recomputed residual tracks it: est relative to the cycle's
            // reference norm, which in FP32-IR is the previous residual), the
            // next cycle is enqueued at once.  Its launches return at once if
            // the residual ends the solve after all, and its first status
            // wait then returns that decision.
            const double pred = stop.est * (fp64 ? 1.0 : relres_prev);
            const bool more = decided ? (!stop.done && !stop.nonfinite)
                                      : (pred > 8.0 * o->tol && stop.total < o->maxit && !stop.breakdown &&
                                         !stop.nonfinite &&
                                         (fp64 ? o->fixed_iters == 0 : stop.outer + 1 < o->max_outer));
            if (more) {
                ++c->stats.cycles_ahead;
                ahead = true;
                relres_prev = decided ? stop.relres : pred;
                continue;
            }
        }
        ahead = false;
        // the residual's decision: a plain stream synchronisation (polling the
        // status for it measured slower than this)
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const HostStatus& hs = *c->hs;
        if (hs.nonfinite) {
            fill_info(c, info, FNLS_ERR_NONFINITE);
            return set_err(c, FNLS_ERR_NONFINITE, "non-finite value during the solve");
        }
        if (hs.done) {
            if (o->fixed_iters > 0 && fp64)
                status = FNLS_OK;
            else
                status = (hs.relres < o->tol) ? FNLS_OK : FNLS_NOT_CONVERGED;
            break;
        }
        relres_prev = hs.relres;
    }
    fill_info(c, info, status);
    return status;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void fnls_default_opts(fnls_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->tol = 1e-10;
    o->restart = 30;
    o->maxit = 2000;
    o->precision = FNLS_FP64;
    o->inner_tol = 1e-5;
    o->max_outer = 20;
    o->fixed_iters = 0;
    o->lookahead = 1;
}

const char* fnls_status_string(int s) {
    switch (s) {
        case FNLS_OK: return "ok";
        case FNLS_NOT_CONVERGED: return "not converged";
        case FNLS_ERR_INVALID_ARG: return "invalid argument";
        case FNLS_ERR_STATE: return "invalid call order";
        case FNLS_ERR_WORKSPACE: return "workspace missing or too small";
        case FNLS_ERR_NONFINITE: return "non-finite input";
        case FNLS_ERR_HIP: return "HIP runtime error";
        case FNLS_ERR_NO_DEVICE: return "no usable GPU";
        default: return "unknown status";
    }
}

size_t fnls_workspace_bytes(int d, int n, int restart) {
    if (d < 1 || d > 3 || !valid_n(n) || restart < 1 || restart > kMaxRestart) return 0;
    // the LDS budget only changes the partial-sum stride; size for the smallest budget
    return make_layout(d, n, restart).total;
}

int fnls_create(fnls_ctx** out, int device, void* hip_stream) {
    if (!out) return FNLS_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return FNLS_ERR_NO_DEVICE;
    if (device < 0 || device >= count) return FNLS_ERR_NO_DEVICE;
    fnls_ctx* c = new (std::nothrow) fnls_ctx();
    if (!c) return FNLS_ERR_HIP;
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return FNLS_ERR_NO_DEVICE;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->max_dyn_lds = (size_t)lds > kStaticLds ? (size_t)lds - kStaticLds : 0;
    if (hipHostMalloc((void**)&c->hs, sizeof(HostStatus), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        delete c;
        return FNLS_ERR_HIP;
    }
    std::memset((void*)c->hs, 0, sizeof(HostStatus));
    if (hipHostGetDevicePointer((void**)&c->hs_dev, c->hs, 0) != hipSuccess) {
        (void)hipHostFree(c->hs);
        delete c;
        return FNLS_ERR_HIP;
    }
    c->static_scr = static_scratch(device);
    *out = c;
    return FNLS_OK;
}

void fnls_destroy(fnls_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->hs) (void)hipHostFree(c->hs);
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    delete c;
}

const char* fnls_last_error(const fnls_ctx* c) { return c ? c->err.c_str() : "null context"; }

int fnls_check_assemble(double alpha, double rho, int d, int n, double h, double tau, const void* workspace,
                        size_t workspace_bytes, char* msg, size_t msg_len) {
    auto fail = [&](int code, const char* what, size_t need = 0) {
        if (msg && msg_len > 0) {
            if (need) snprintf(msg, msg_len, "%s (need %zu bytes for restart 1)", what, need);
            else snprintf(msg, msg_len, "%s", what);
        }
        return code;
    };
    if (msg && msg_len > 0) msg[0] = 0;
    if (!(alpha > 1.0 && alpha <= 2.0)) return fail(FNLS_ERR_INVALID_ARG, "alpha must lie in (1, 2]");
    if (!(rho >= 0.0) || !std::isfinite(rho)) return fail(FNLS_ERR_INVALID_ARG, "rho must be finite and >= 0");
    if (d < 1 || d > 3) return fail(FNLS_ERR_INVALID_ARG, "d must be 1, 2 or 3");
    if (!valid_n(n)) return fail(FNLS_ERR_INVALID_ARG, "n + 1 must be a power of two and n <= 1023");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(FNLS_ERR_INVALID_ARG, "h must be finite and > 0");
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(FNLS_ERR_INVALID_ARG, "tau must be finite and > 0");
    if (!workspace) return fail(FNLS_ERR_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(FNLS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (make_layout(d, n, 1).total > workspace_bytes)
        return fail(FNLS_ERR_WORKSPACE, "workspace too small", make_layout(d, n, 1).total);
    return FNLS_OK;
}

int fnls_assemble(fnls_ctx* c, double alpha, double rho, int d, int n, double h, double tau, void* workspace,
                  size_t workspace_bytes) {
    if (!c) return FNLS_ERR_INVALID_ARG;
    char why[256];
    const int chk = fnls_check_assemble(alpha, rho, d, n, h, tau, workspace, workspace_bytes, why, sizeof why);
    if (chk != FNLS_OK) return set_err(c, chk, "%s", why);
    // largest restart length that fits
    int cap = 0;
    for (int r = kMaxRestart; r >= 1; --r) {
        if (make_layout(d, n, r).total <= workspace_bytes) {
            cap = r;
            break;
        }
    }
    HIPCHK(c, hipSetDevice(c->device));
    c->alpha = alpha;
    c->rho = rho;
    c->d = d;
    c->n = n;
    c->m = n + 1;
    c->h = h;
    c->tau = tau;
    c->N = ipow(n, d);
    c->ws = reinterpret_cast<char*>(workspace);
    c->ws_bytes = workspace_bytes;
    c->restart_cap = cap;
    c->lay = make_layout(d, n, cap);
    c->scr = c->ws + c->lay.op_total;
    c->pcfg = default_pass_config(n + 1);
    for (int f = 0; f < 2; ++f)
        for (int st = 0; st < 2; ++st) {
            int rm = 0, li = 0;
            if (tuned_get(n + 1, f == 1, st == 1, &rm, &li)) {
                c->pcfg.rmax[f][st] = rm;
                c->pcfg.lines[f][st] = li;
            }
        }
    c->tscale = 1.0;
    c->have_D = 0;

    // host tables in extended precision
    const int m = n + 1;
    const long double a = alpha;
    std::vector<long double> ck(n);
    ck[0] = std::tgamma(a + 1) / (std::tgamma(a / 2 + 1) * std::tgamma(a / 2 + 1));
    for (int k = 0; k + 1 < n; ++k) ck[k + 1] = ck[k] * ((long double)k - a / 2) / ((long double)k + 1 + a / 2);
    const long double mu = (long double)tau / std::pow((long double)h, a);
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<long double> cs(2 * m), sn(2 * m);
    for (int t = 0; t < 2 * m; ++t) {
        cs[t] = std::cos(pi * t / m);
        sn[t] = std::sin(pi * t / m);
    }
    std::vector<long double> sym(2 * m);
    for (int q = 0; q < 2 * m; ++q) {
        long double acc = 0;
        for (int j = n - 1; j >= 1; --j) acc += ck[j] * cs[(int)(((long long)j * q) % (2 * m))];
        sym[q] = mu * (ck[0] + 2 * acc);
    }
    std::vector<double2> tw64(2 * m);
    std::vector<float2> tw32(2 * m);
    for (int t = 0; t < 2 * m; ++t) {
        tw64[t] = make_double2((double)cs[t], (double)-sn[t]);
        tw32[t] = make_float2((float)cs[t], (float)-sn[t]);
    }
    std::vector<double> se(m), so(m), lam(m);
    std::vector<float> se32(m), so32(m), lam32(m);
    for (int p = 0; p < m; ++p) {
        se[p] = (double)(sym[2 * p] / (2 * m));
        so[p] = (double)(sym[2 * p + 1] / (2 * m));
        lam[p] = p == 0 ? 0.0 : (double)sym[p];
        se32[p] = (float)se[p];
        so32[p] = (float)so[p];
        lam32[p] = (float)lam[p];
    }
    HIPCHK(c, hipMemcpyAsync(c->at<void>(c->lay.tw64), tw64.data(), 2 * m * sizeof(double2), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->at<void>(c->lay.tw32), tw32.data(), 2 * m * sizeof(float2), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->at<void>(c->lay.syme64), se.data(), m * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->at<void>(c->lay.symo64), so.data(), m * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->at<void>(c->lay.lam64), lam.data(), m * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->at<void>(c->lay.syme32), se32.data(), m * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->at<void>(c->lay.symo32), so32.data(), m * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->at<void>(c->lay.lam32), lam32.data(), m * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->sc<void>(c->lay.state), 0, sizeof(GmresState), c->stream));
    // the host vectors above go out of scope: finish the copies first
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->assembled = 1;
    return FNLS_OK;
}

static int precond_setup_scaled(fnls_ctx* c, const fnls_c128* u, const double* V, double omega, double tau) {
    StreamArgs s;
    std::memset(&s, 0, sizeof s);
    s.N = c->N;
    s.u = u;
    s.V = V;
    s.D64 = c->at<double>(c->lay.D64);
    s.D32 = c->at<float>(c->lay.D32);
    s.rho = c->rho;
    s.tau = tau;
    const int blocks = (int)std::min<long long>(4096, (c->N + 255) / 256);
    const LaunchEvents* te = c->timing ? timing_begin(c, "precond_setup", 28.0 * (double)c->N, 24.0 * (double)c->N) : nullptr;
    hipError_t e = launch_precond_setup(s, blocks, c->stream, te);
    if (e != hipSuccess) {
        timing_failed(c, te);
        return set_err(c, FNLS_ERR_HIP, "precond_setup launch failed: %s", hipGetErrorString(e));
    }
    c->omega = omega;
    c->have_D = 1;
    return FNLS_OK;
}

int fnls_precond_setup(fnls_ctx* c, const fnls_c128* u_cur, const double* V, double omega) {
    int rc = check_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!u_cur) return set_err(c, FNLS_ERR_INVALID_ARG, "u_cur is NULL");
    if (!(omega > 0.0) || !std::isfinite(omega)) return set_err(c, FNLS_ERR_INVALID_ARG, "omega must be > 0");
    HIPCHK(c, hipSetDevice(c->device));
    c->tscale = 1.0;
    return precond_setup_scaled(c, u_cur, V, omega, c->tau);
}

int fnls_apply_A(fnls_ctx* c, const fnls_c128* x, fnls_c128* y) {
    int rc = check_solve_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!x || !y) return set_err(c, FNLS_ERR_INVALID_ARG, "NULL vector");
    if ((const void*)x == (const void*)y) return set_err(c, FNLS_ERR_INVALID_ARG, "x and y must not alias");
    HIPCHK(c, hipSetDevice(c->device));
    return matvec64(c, x, y, 1.0, 1.0, -1.0);
}

int fnls_rhs(fnls_ctx* c, const fnls_c128* u_prev, fnls_c128* b) {
    int rc = check_solve_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!u_prev || !b) return set_err(c, FNLS_ERR_INVALID_ARG, "NULL vector");
    if ((const void*)u_prev == (const void*)b) return set_err(c, FNLS_ERR_INVALID_ARG, "u_prev and b must not alias");
    HIPCHK(c, hipSetDevice(c->device));
    return matvec64(c, u_prev, b, -1.0, 1.0, 1.0);
}

}  // extern "C"

namespace {
// z = Ptilde^{-1} r in the precision of fp64 (complex128 or complex64 vectors).
int precond_apply(fnls_ctx* c, bool fp64, const void* r, void* z) {
    Bufs b = bufs(c, fp64, nullptr);
    if (c->d == 1) {
        Geo g = pass_geo(1, c->n, 0, fp64, c->max_dyn_lds, c->pcfg);
        PassArgs a = base_args(c, fp64, 0, g);
        a.in = r;
        a.out = z;
        PassVariant v{IN_PLAIN, P_DST1 | P_DIV | P_DST2 | P_SCALE, Z_NONE, OUT_LINE, FIN_WRITE};
        return run_pass(c, fp64, 0, v, a, g);
    }
    void* t;
    int rc;
    if ((rc = precond_front(c, fp64, IN_PLAIN, r, 0, b, &t, 0)) != FNLS_OK) return rc;
    Geo g = pass_geo(c->d, c->n, c->d - 1, fp64, c->max_dyn_lds, c->pcfg);
    PassArgs a = base_args(c, fp64, c->d - 1, g);
    a.in = t;
    a.out = z;
    PassVariant v{IN_PLAIN, P_DST1 | P_SCALE, Z_NONE, OUT_LINE, FIN_WRITE};
    return run_pass(c, fp64, c->d - 1, v, a, g);
}

int check_vec_pair(fnls_ctx* c, const void* in, const void* out, const char* what) {
    int rc = check_solve_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!in || !out) return set_err(c, FNLS_ERR_INVALID_ARG, "NULL vector");
    if (in == out) return set_err(c, FNLS_ERR_INVALID_ARG, "%s must not alias", what);
    HIPCHK(c, hipSetDevice(c->device));
    return FNLS_OK;
}
}  // namespace

extern "C" {

int fnls_apply_precond(fnls_ctx* c, const fnls_c128* r, fnls_c128* z) {
    int rc = check_vec_pair(c, r, z, "r and z");
    return rc != FNLS_OK ? rc : precond_apply(c, true, r, z);
}

int fnls_apply_A_c64(fnls_ctx* c, const fnls_c64* x, fnls_c64* y) {
    int rc = check_vec_pair(c, x, y, "x and y");
    return rc != FNLS_OK ? rc : matvec(c, false, x, y, 1.0, 1.0, -1.0);
}

int fnls_apply_precond_c64(fnls_ctx* c, const fnls_c64* r, fnls_c64* z) {
    int rc = check_vec_pair(c, r, z, "r and z");
    return rc != FNLS_OK ? rc : precond_apply(c, false, r, z);
}

int fnls_get_host_stats(fnls_ctx* c, fnls_host_stats* out, int reset) {
    if (!c) return FNLS_ERR_INVALID_ARG;
    if (out) *out = c->stats;
    if (reset) std::memset(&c->stats, 0, sizeof c->stats);
    return FNLS_OK;
}

int fnls_status_report_accepted(unsigned seq_base, unsigned seq_before, unsigned seq_after, int total, int done,
                                int target) {
    return report_accepted(seq_base, seq_before, seq_after, total, done, target) ? 1 : 0;
}

int fnls_pass_geometry(int d, int n, int axis, int precision, int rmax, int lines, size_t max_dyn_lds,
                       long long out[10]) {
    if (!out || d < 1 || d > 3 || axis < 0 || axis >= d || !valid_n(n) ||
        (precision != FNLS_FP64 && precision != FNLS_FP32_IR) || (rmax != 4 && rmax != 8 && rmax != 16) ||
        lines < 1 || lines > 64 || max_dyn_lds == 0)
        return FNLS_ERR_INVALID_ARG;
    const bool fp64 = precision == FNLS_FP64;
    PassConfig cfg = default_pass_config(n + 1);
    for (int st = 0; st < 2; ++st) {
        cfg.rmax[fp64 ? 1 : 0][st] = rmax;
        cfg.lines[fp64 ? 1 : 0][st] = lines;
    }
    const Geo g = pass_geo(d, n, axis, fp64, max_dyn_lds, cfg);
    int pa2 = 0, ls2 = 0, pa1 = 0, ls1 = 0;
    line_layout(n + 1, g.L, fp64, true, &pa2, &ls2);
    line_layout(n + 1, g.L, fp64, false, &pa1, &ls1);
    const long long v[10] = {g.G, g.L, g.blocks, (long long)g.lds, g.stride, g.nlines, pa2, ls2, pa1, ls1};
    for (int i = 0; i < 10; ++i) out[i] = v[i];
    return FNLS_OK;
}

static int resolve_opts(fnls_ctx* c, const fnls_opts* in, fnls_opts* o, int restart_cap = -1) {
    if (in) *o = *in;
    else fnls_default_opts(o);
    if (restart_cap < 0) restart_cap = c->restart_cap;
    if (!(o->tol > 0.0)) return set_err(c, FNLS_ERR_INVALID_ARG, "tol must be > 0");
    if (o->restart < 1 || o->restart > restart_cap)
        return set_err(c, FNLS_ERR_WORKSPACE, "restart %d exceeds the workspace capacity %d (or < 1)", o->restart,
                       restart_cap);
    // (at most one status report per iteration plus one per cycle: a solve's
    // reports stay inside its window of the status sequence)
    if (o->maxit < 1 || o->maxit > (1 << 21)) return set_err(c, FNLS_ERR_INVALID_ARG, "maxit must lie in [1, 2^21]");
    if (o->precision != FNLS_FP64 && o->precision != FNLS_FP32_IR)
        return set_err(c, FNLS_ERR_INVALID_ARG, "unknown precision");
    if (o->precision == FNLS_FP32_IR) {
        if (!(o->inner_tol > 0.0 && o->inner_tol < 1.0)) return set_err(c, FNLS_ERR_INVALID_ARG, "inner_tol must lie in (0, 1)");
        if (o->max_outer < 1) return set_err(c, FNLS_ERR_INVALID_ARG, "max_outer must be >= 1");
        if (o->fixed_iters) return set_err(c, FNLS_ERR_INVALID_ARG, "fixed_iters is FP64-only");
    }
    if (o->fixed_iters < 0) return set_err(c, FNLS_ERR_INVALID_ARG, "fixed_iters must be >= 0");
    if (o->lookahead < 0 || o->lookahead > kEvents - 2) return set_err(c, FNLS_ERR_INVALID_ARG, "lookahead out of range");
    if (o->graph != 0 && o->graph != 1) return set_err(c, FNLS_ERR_INVALID_ARG, "graph must be 0 or 1");
    if (o->poll_delay_us < 0 || o->poll_delay_us > 1000000)
        return set_err(c, FNLS_ERR_INVALID_ARG, "poll_delay_us must lie in [0, 1e6]");
    return FNLS_OK;
}

int fnls_solve(fnls_ctx* c, const fnls_c128* b, fnls_c128* x, const fnls_opts* opts, fnls_info* info) {
    int rc = check_solve_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!b || !x) return set_err(c, FNLS_ERR_INVALID_ARG, "NULL vector");
    if ((const void*)b == (const void*)x) return set_err(c, FNLS_ERR_INVALID_ARG, "b and x must not alias");
    fnls_opts o;
    if ((rc = resolve_opts(c, opts, &o)) != FNLS_OK) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    return solve_impl(c, b, x, &o, info);
}

int fnls_solve_noalloc(fnls_ctx* c, const fnls_c128* b, fnls_c128* x, const fnls_opts* opts, fnls_info* info) {
    int rc = check_solve_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!b || !x) return set_err(c, FNLS_ERR_INVALID_ARG, "NULL vector");
    if ((const void*)b == (const void*)x) return set_err(c, FNLS_ERR_INVALID_ARG, "b and x must not alias");
    fnls_opts o;
    if ((rc = resolve_opts(c, opts, &o, kMaxRestart)) != FNLS_OK) return rc;
    Layout lay = c->lay;
    scratch_layout(lay, c->d, c->n, o.restart);
    if (lay.scr_total > kStaticScratchBytes)
        return set_err(c, FNLS_ERR_WORKSPACE, "solver scratch of %zu bytes (d %d, n %d, restart %d) exceeds the "
                       "static scratch of %zu bytes", lay.scr_total, c->d, c->n, o.restart, kStaticScratchBytes);
    if (!c->static_scr) return set_err(c, FNLS_ERR_HIP, "the device's static scratch is unavailable");
    HIPCHK(c, hipSetDevice(c->device));
    // the solve runs on the static scratch: swap the scratch base and layout
    // for the call, then restore the workspace's
    const Layout saved = c->lay;
    char* const saved_scr = c->scr;
    c->lay = lay;
    c->scr = c->static_scr;
    // the array keeps the previous call's contents: start from a cleared state
    hipError_t e = hipMemsetAsync(c->st(), 0, sizeof(GmresState), c->stream);
    if (e == hipSuccess) rc = solve_impl(c, b, x, &o, info);
    else rc = set_err(c, FNLS_ERR_HIP, "hipMemsetAsync failed: %s", hipGetErrorString(e));
    c->lay = saved;
    c->scr = saved_scr;
    return rc;
}

int fnls_step(fnls_ctx* c, const fnls_c128* u_prev, const fnls_c128* u_cur, fnls_c128* u_next,
              const fnls_opts* opts, fnls_info* info) {
    const TraceRange trace("fnls.step");
    int rc = check_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!u_prev || !u_cur || !u_next) return set_err(c, FNLS_ERR_INVALID_ARG, "NULL vector");
    if ((const void*)u_next == (const void*)u_prev || (const void*)u_next == (const void*)u_cur)
        return set_err(c, FNLS_ERR_INVALID_ARG, "u_next must not alias the inputs");
    fnls_opts o;
    if ((rc = resolve_opts(c, opts, &o)) != FNLS_OK) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    c->tscale = 1.0;
    if ((rc = precond_setup_scaled(c, u_cur, c->Vpot, c->omega > 0 ? c->omega : 1.0, c->tau)) != FNLS_OK) return rc;
    fnls_c128* bb = c->at<fnls_c128>(c->lay.bbuf);
    if ((rc = matvec64(c, u_prev, bb, -1.0, 1.0, 1.0)) != FNLS_OK) return rc;
    return solve_impl(c, bb, u_next, &o, info);
}

int fnls_first_step(fnls_ctx* c, const fnls_c128* u0, fnls_c128* u1, const fnls_opts* opts, fnls_info* info) {
    const TraceRange trace("fnls.first_step");
    int rc = check_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!u0 || !u1) return set_err(c, FNLS_ERR_INVALID_ARG, "NULL vector");
    if ((const void*)u0 == (const void*)u1) return set_err(c, FNLS_ERR_INVALID_ARG, "u1 must not alias u0");
    fnls_opts o;
    if ((rc = resolve_opts(c, opts, &o)) != FNLS_OK) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    const double omega = c->omega > 0 ? c->omega : 1.0;
    c->tscale = 0.5;
    rc = precond_setup_scaled(c, u0, c->Vpot, omega, 0.5 * c->tau);
    fnls_c128* bb = c->at<fnls_c128>(c->lay.bbuf);
    if (rc == FNLS_OK) rc = matvec64(c, u0, bb, -1.0, 1.0, 1.0);
    if (rc == FNLS_OK || rc == FNLS_NOT_CONVERGED) rc = solve_impl(c, bb, u1, &o, info);
    c->tscale = 1.0;
    c->have_D = 0;   // D belongs to the starter system; the next step recomputes it
    return rc;
}

int fnls_set_potential(fnls_ctx* c, const double* V) {
    if (!c) return FNLS_ERR_INVALID_ARG;
    c->Vpot = V;
    return FNLS_OK;
}

}  // extern "C"

namespace {
// Reverse mode of the step with time-step factor tfac (1: three-level step,
// 0.5: starter with u_prev = u_cur): lam = conj(A^{-1} conj(g_next)), then
// g_prev += conj(B conj(lam)) and the g_D terms.
int step_backward_impl(fnls_ctx* c, const fnls_c128* u_prev, const fnls_c128* u_cur, const fnls_c128* u_next,
                       const fnls_c128* g_next, fnls_c128* g_prev, fnls_c128* g_cur, double* g_V,
                       const fnls_opts* opts, fnls_info* info, double tfac) {
    fnls_opts o;
    int rc = resolve_opts(c, opts, &o);
    if (rc != FNLS_OK) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    const double omega = c->omega > 0 ? c->omega : 1.0;
    c->tscale = tfac;
    rc = precond_setup_scaled(c, u_cur, c->Vpot, omega, tfac * c->tau);
    double2* bb = c->at<double2>(c->lay.bbuf);
    double2* sol = c->at<double2>(c->lay.adj);
    if (rc == FNLS_OK) {
        hipError_t e = launch_conj(reinterpret_cast<const double2*>(g_next), bb, c->N, c->stream);
        if (e != hipSuccess) rc = set_err(c, FNLS_ERR_HIP, "conj launch failed: %s", hipGetErrorString(e));
    }
    int srt = FNLS_OK;
    if (rc == FNLS_OK) {
        srt = solve_impl(c, reinterpret_cast<const fnls_c128*>(bb), reinterpret_cast<fnls_c128*>(sol), &o, info);
        if (srt < 0) rc = srt;
    }
    // w = B sol into the (now free) right-hand-side buffer
    if (rc == FNLS_OK) rc = matvec64(c, sol, bb, -1.0, 1.0, 1.0);
    if (rc == FNLS_OK) {
        AdjointArgs a;
        std::memset(&a, 0, sizeof a);
        a.N = c->N;
        a.sol = sol;
        a.w = bb;
        a.u_prev = reinterpret_cast<const double2*>(u_prev);
        a.u_cur = reinterpret_cast<const double2*>(u_cur);
        a.u_next = reinterpret_cast<const double2*>(u_next);
        a.g_prev = reinterpret_cast<double2*>(g_prev);
        a.g_cur = reinterpret_cast<double2*>(g_cur);
        a.g_V = g_V;
        a.dt = tfac * c->tau;
        a.rho = c->rho;
        const double adj_bytes = (16.0 * 7 + (g_cur ? 32.0 : 0.0) + (g_V ? 16.0 : 0.0)) * (double)c->N;
        const LaunchEvents* te = c->timing ? timing_begin(c, "adjoint", adj_bytes, adj_bytes)
                                           : nullptr;
        hipError_t e = launch_adjoint(a, c->stream, te);
        if (e != hipSuccess) {
            timing_failed(c, te);
            rc = set_err(c, FNLS_ERR_HIP, "adjoint launch failed: %s", hipGetErrorString(e));
        }
    }
    if (rc == FNLS_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = set_err(c, FNLS_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    c->tscale = 1.0;
    if (tfac != 1.0) c->have_D = 0;
    return rc == FNLS_OK ? srt : rc;
}

bool same(const void* a, const void* b) { return a && a == b; }
}  // namespace

extern "C" {

int fnls_step_backward(fnls_ctx* c, const fnls_c128* u_prev, const fnls_c128* u_cur, const fnls_c128* u_next,
                       const fnls_c128* g_next, fnls_c128* g_prev, fnls_c128* g_cur, double* g_V,
                       const fnls_opts* opts, fnls_info* info) {
    const TraceRange trace("fnls.step_backward");
    int rc = check_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!u_prev || !u_cur || !u_next || !g_next || !g_prev || !g_cur)
        return set_err(c, FNLS_ERR_INVALID_ARG, "NULL vector");
    if (same(g_prev, g_cur) || same(g_prev, g_next) || same(g_cur, g_next) || same(g_prev, u_prev) ||
        same(g_prev, u_cur) || same(g_prev, u_next) || same(g_cur, u_prev) || same(g_cur, u_cur) ||
        same(g_cur, u_next))
        return set_err(c, FNLS_ERR_INVALID_ARG, "gradient outputs must not alias each other or the inputs");
    return step_backward_impl(c, u_prev, u_cur, u_next, g_next, g_prev, g_cur, g_V, opts, info, 1.0);
}

int fnls_first_step_backward(fnls_ctx* c, const fnls_c128* u0, const fnls_c128* u1, const fnls_c128* g1,
                             fnls_c128* g0, double* g_V, const fnls_opts* opts, fnls_info* info) {
    const TraceRange trace("fnls.first_step_backward");
    int rc = check_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!u0 || !u1 || !g1 || !g0) return set_err(c, FNLS_ERR_INVALID_ARG, "NULL vector");
    if (same(g0, g1) || same(g0, u0) || same(g0, u1))
        return set_err(c, FNLS_ERR_INVALID_ARG, "g0 must not alias the inputs");
    return step_backward_impl(c, u0, u0, u1, g1, g0, nullptr, g_V, opts, info, 0.5);
}

int fnls_timing(fnls_ctx* c, int enable) {
    if (!c) return FNLS_ERR_INVALID_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->recs.clear();
    c->evused = 0;
    c->timing = enable ? 1 : 0;
    return FNLS_OK;
}

int fnls_timing_report(fnls_ctx* c, fnls_kernel_stat* out, int max_entries) {
    if (!c || (!out && max_entries > 0) || max_entries < 0) return FNLS_ERR_INVALID_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int ncls = (int)c->class_names.size();
    std::vector<fnls_kernel_stat> agg(ncls);
    for (int i = 0; i < ncls; ++i) {
        std::memset(&agg[i], 0, sizeof(fnls_kernel_stat));
        std::snprintf(agg[i].name, sizeof agg[i].name, "%s", c->class_names[i].c_str());
    }
    for (const auto& r : c->recs) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, r.ev.start, r.ev.stop));
        agg[r.cls].launches += 1;
        agg[r.cls].total_ms += ms;
        agg[r.cls].bytes += r.bytes;
        agg[r.cls].bytes_min += r.bytes_min;
    }
    int k = 0;
    for (int i = 0; i < ncls && k < max_entries; ++i)
        if (agg[i].launches > 0) out[k++] = agg[i];
    return k;
}

int fnls_autotune(fnls_ctx* c, const fnls_c128* b, int precision, int reps, int best[4], double* best_ms) {
    const TraceRange trace("fnls.autotune");
    int rc = check_solve_ready(c);
    if (rc != FNLS_OK) return rc;
    if (!b) return set_err(c, FNLS_ERR_INVALID_ARG, "NULL vector");
    if (precision != FNLS_FP64 && precision != FNLS_FP32_IR)
        return set_err(c, FNLS_ERR_INVALID_ARG, "unknown precision");
    if (reps < 1 || reps > 1000) return set_err(c, FNLS_ERR_INVALID_ARG, "reps must lie in [1, 1000]");
    HIPCHK(c, hipSetDevice(c->device));
    fnls_opts o;
    fnls_default_opts(&o);
    o.precision = precision;
    o.restart = std::min(o.restart, c->restart_cap);
    fnls_c128* x = c->at<fnls_c128>(c->lay.adj);
    const int f = precision == FNLS_FP64 ? 1 : 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_err(c, FNLS_ERR_HIP, "hipEventCreate failed");
    }
    // time per solve of the current schedule: one untimed warm-up solve, then
    // the fastest of three timed runs of `reps` solves (run-to-run noise is a
    // few per cent)
    auto measure = [&](double* ms) -> int {
        int r = solve_impl(c, b, x, &o, nullptr);
        if (r < 0) return r;
        double best_t = 0.0;
        for (int trial = 0; trial < 3; ++trial) {
            if (hipEventRecord(e0, c->stream) != hipSuccess) return set_err(c, FNLS_ERR_HIP, "hipEventRecord");
            for (int k = 0; k < reps; ++k) {
                r = solve_impl(c, b, x, &o, nullptr);
                if (r < 0) return r;
            }
            if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return set_err(c, FNLS_ERR_HIP, "event timing failed");
            float t = 0.f;
            if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return set_err(c, FNLS_ERR_HIP, "hipEventElapsedTime");
            const double per = (double)t / reps;
            if (trial == 0 || per < best_t) best_t = per;
        }
        *ms = best_t;
        return FNLS_OK;
    };
    static const int kRmax[3] = {4, 8, 16};
    static const int kLines[3] = {1, 2, 4};
    double cur = 0.0;
    rc = measure(&cur);
    // coordinate descent: strided axes, then the contiguous axis
    for (int strided = 1; strided >= 0 && rc == FNLS_OK; --strided) {
        int br = c->pcfg.rmax[f][strided], bl = c->pcfg.lines[f][strided];
        for (int ir = 0; ir < 3 && rc == FNLS_OK; ++ir)
            for (int il = 0; il < 3 && rc == FNLS_OK; ++il) {
                const int rm = kRmax[ir], li = kLines[il];
                if (rm == br && li == bl) continue;
                if ((1024 / rm) * li > pass_threads_max(rm)) continue;
                c->pcfg.rmax[f][strided] = rm;
                c->pcfg.lines[f][strided] = li;
                double t = 0.0;
                rc = measure(&t);
                // a schedule replaces the current one only when clearly faster
                if (rc == FNLS_OK && t < 0.99 * cur) {
                    cur = t;
                    br = rm;
                    bl = li;
                }
            }
        c->pcfg.rmax[f][strided] = br;
        c->pcfg.lines[f][strided] = bl;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != FNLS_OK) return rc;
    tuned_put(c->m, f == 1, false, c->pcfg.rmax[f][0], c->pcfg.lines[f][0]);
    tuned_put(c->m, f == 1, true, c->pcfg.rmax[f][1], c->pcfg.lines[f][1]);
    if (best) {
        best[0] = c->pcfg.rmax[f][0];
        best[1] = c->pcfg.lines[f][0];
        best[2] = c->pcfg.rmax[f][1];
        best[3] = c->pcfg.lines[f][1];
    }
    if (best_ms) *best_ms = cur;
    return FNLS_OK;
}

int fnls_set_pass_config(fnls_ctx* c, int precision, int strided, int rmax, int lines) {
    if (!c) return FNLS_ERR_INVALID_ARG;
    if ((precision != FNLS_FP64 && precision != FNLS_FP32_IR) || (strided != 0 && strided != 1))
        return set_err(c, FNLS_ERR_INVALID_ARG, "precision / axis kind out of range");
    if (rmax != 4 && rmax != 8 && rmax != 16) return set_err(c, FNLS_ERR_INVALID_ARG, "rmax must be 4, 8 or 16");
    if (lines < 1 || lines > 64 || (lines & (lines - 1)) != 0)
        return set_err(c, FNLS_ERR_INVALID_ARG, "lines must be a power of two in [1, 64]");
    if ((1024 / rmax) * lines > pass_threads_max(rmax))
        return set_err(c, FNLS_ERR_INVALID_ARG, "too many threads per workgroup for rmax %d", rmax);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int f = precision == FNLS_FP64 ? 1 : 0;
    c->pcfg.rmax[f][strided] = rmax;
    c->pcfg.lines[f][strided] = lines;
    return FNLS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: many assembled contexts (any sizes, same d, device and stream)
// advanced together, one kernel launch per pass / update / decision for all
// of them.  Every instance's lines use radix 4 and 1024-thread workgroups
// (G = m / 4 threads per line, 1024 / G lines), so one launch shape serves
// all line lengths; the workgroups of instance i form one block range of the
// launch.  Per-launch argument arrays are staged through a pinned ring into
// the caller's batch workspace.  The launches of one Arnoldi iteration take
// the iteration index from each instance's GMRES state, so one argument
// table serves a whole cycle; in graph mode those launches are captured once
// into a hipGraph that is replayed for every iteration (and every later
// cycle or call with the same arguments).
// ---------------------------------------------------------------------------
constexpr int kBatchThreads = 1024;
constexpr int kMaxBatch = 4096;
constexpr size_t kBatchRingMin = (size_t)16 << 20;
constexpr int kGraphSlots = 4;        // cached iteration graphs per batch
constexpr int kMaxIterLaunches = 36;  // launches of one Arnoldi iteration (d <= 3, 4 line-length classes)

struct GraphSlot {
    std::vector<char> key;            // argument table + launch shapes it was captured with
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    unsigned long long used = 0;      // last use (LRU replacement)
};

struct fnls_batch {
    int count = 0;
    std::vector<fnls_ctx*> ctx;
    int device = 0;
    hipStream_t stream = nullptr;
    int d = 0;
    char* dring = nullptr;       // caller's workspace
    char* hring = nullptr;       // pinned staging
    size_t ring_bytes = 0;
    size_t off = 0;
    hipEvent_t ev[kEvents] = {};
    // graph mode: argument tables of the cached graphs (caller's workspace,
    // after the ring), a stream used only for capturing, the cache
    char* dgraph = nullptr;
    size_t slot_bytes = 0;
    hipStream_t cap = nullptr;
    GraphSlot gs[kGraphSlots];
    unsigned long long tick = 0;
    long long captures = 0, replays = 0;
    // side streams of an Arnoldi iteration: the pass launches of the line-length
    // classes other than the first run on them, forked from and joined back to
    // the batch stream (default priority, non-blocking)
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[kSide] = {};
    // transform schedules chosen by fnls_batch_autotune per line length,
    // precision and axis kind: key m * 4 + fp64 * 2 + strided -> (rmax, lines)
    std::map<long long, std::pair<int, int>> sched;
    std::string err;
};

namespace {

int berr(fnls_batch* B, int code, const char* fmt, ...) {
    if (B) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        B->err = buf;
    }
    return code;
}

#define BHIPCHK(B, expr)                                                                             \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return berr(B, FNLS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t batch_ring_bytes(int count) { return std::max(kBatchRingMin, (size_t)count * 64 * 1024); }
// Upper bound of one iteration's argument table (every launch: count argument
// blocks and count + 1 block offsets, each array 256-byte aligned).
size_t batch_slot_bytes(int count) {
    const size_t args = std::max(sizeof(PassArgs), sizeof(StreamArgs));
    return (size_t)kMaxIterLaunches * (align_up((size_t)count * args) + align_up((size_t)(count + 1) * sizeof(int)));
}
size_t batch_total_bytes(int count) { return batch_ring_bytes(count) + (size_t)kGraphSlots * batch_slot_bytes(count); }

int batch_lgm_class(int lgm);

// Geometry of a pass in a batched launch.  By default radix 4 and
// G * L = 1024 threads, one launch shape for every line length.  Line
// lengths with a compile-time plan (m = 256, 512, 1024) take the schedule
// fnls_batch_autotune chose for the batch (radix 4 or 8, lines per workgroup
// by the rule of the single-instance passes), if any.
Geo batch_geo(int d, int n, int axis, bool fp64, const fnls_batch* B = nullptr) {
    Geo g;
    const int m = n + 1;
    int lgm = 0;
    while ((1 << lgm) < m) ++lgm;
    int rmax = 4, lines = 0;
    bool tuned = false;
    if (B && batch_lgm_class(lgm) != 0) {
        // a class with a compile-time plan has one line length, so its launch
        // takes that length's own schedule: the one fnls_batch_autotune chose,
        // else the single-instance default (smaller workgroups than the
        // shared 1024-thread shape, so that several share a CU and overlap
        // their load, transform and store phases)
        auto it = B->sched.find((long long)m * 4 + (fp64 ? 2 : 0) + (axis != d - 1 ? 1 : 0));
        if (it != B->sched.end()) {
            rmax = it->second.first;
            lines = it->second.second;
        } else {
            const PassConfig cfg = default_pass_config(m);
            rmax = cfg.rmax[fp64 ? 1 : 0][axis != d - 1 ? 1 : 0];
            lines = cfg.lines[fp64 ? 1 : 0][axis != d - 1 ? 1 : 0];
        }
        tuned = (rmax == 4 || rmax == 8);
    }
    if (tuned) {
        g.rmax = rmax;
        g.G = std::max(1, m / rmax);
        const int tmax = std::min(kBatchThreads, pass_threads_max(rmax));
        int L = lines * std::max(1, (1024 / rmax) / g.G);
        L = std::max(1, std::min(L, tmax / g.G));
        while (g.G * L < 64) L *= 2;
        g.L = L;
    } else {
        g.rmax = 4;
        g.G = std::max(1, m / 4);
        g.L = std::max(1, kBatchThreads / g.G);
    }
    const size_t elem = fp64 ? 16 : 8;
    int pa = 0, ls = 0;
    line_layout(m, g.L, fp64, true, &pa, &ls);   // the larger (Toeplitz) layout
    g.lds = (size_t)g.L * ls * elem + (size_t)(m >= 4 ? m / 4 : 1) * elem + (size_t)g.L * (8 + elem / 2);
    g.stride = ipow(n, d - 1 - axis);
    g.nlines = ipow(n, d - 1);
    g.blocks = (int)((g.nlines + g.L - 1) / g.L);
    return g;
}

// Host-side image of the argument arrays of one or more launches.
struct Blob {
    std::vector<char> data;
    template <typename T> size_t add(const std::vector<T>& v) {
        const size_t o = align_up(data.size());
        data.resize(o + v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(data.data() + o, v.data(), v.size() * sizeof(T));
        return o;
    }
};

// Copy the blob into the device ring (stream-ordered); returns its device base.
int stage(fnls_batch* B, const Blob& blob, char** dbase) {
    const size_t n = align_up(blob.data.size());
    if (n > B->ring_bytes) return berr(B, FNLS_ERR_WORKSPACE, "argument arrays (%zu B) exceed the batch ring", n);
    if (B->off + n > B->ring_bytes) {
        // every earlier copy and launch must be done before the ring is reused
        BHIPCHK(B, hipStreamSynchronize(B->stream));
        B->off = 0;
    }
    std::memcpy(B->hring + B->off, blob.data.data(), blob.data.size());
    BHIPCHK(B, hipMemcpyAsync(B->dring + B->off, B->hring + B->off, blob.data.size(), hipMemcpyHostToDevice,
                              B->stream));
    *dbase = B->dring + B->off;
    B->off += n;
    return FNLS_OK;
}

// One launch of a batch: per-instance arguments and the block offsets.
// Line lengths with a compile-time plan in the batched pass kernel.
int batch_lgm_class(int lgm) { return (lgm == 8 || lgm == 9 || lgm == 10) ? lgm : 0; }

struct PassLaunch {
    PassVariant v;
    int fp64;
    int lgm = 0;                      // line-length class of every instance (batch_lgm_class)
    int threads = kBatchThreads;      // G * L of every instance of the launch
    std::vector<PassArgs> args;
    std::vector<int> offs{0};
    std::vector<size_t> ilds;         // LDS of each instance
    std::vector<int> irmax, ithreads; // schedule of each instance
    size_t lds = 0;
    size_t a_off = 0, o_off = 0;
    void add(PassArgs a, const Geo& g) {
        line_layout(a.m, g.L, fp64 != 0, (v.ops & P_TOEP) != 0, &a.pa, &a.ls);
        args.push_back(a);
        offs.push_back(offs.back() + g.blocks);
        ilds.push_back(pass_lds(g, a.m, fp64 != 0, (v.ops & P_TOEP) != 0));
        irmax.push_back(g.rmax);
        ithreads.push_back(g.G * g.L);
        lds = std::max(lds, ilds.back());
    }
};
struct StreamLaunch {
    int kind;   // 0 cgs (mode), 1 zupdate, 2 prepare, 3 precond_setup, 4 finish
    int fp64 = 1, mode = 0;
    std::vector<StreamArgs> args;
    std::vector<int> offs{0};
    size_t a_off = 0, o_off = 0;
    void add(const StreamArgs& a, int blocks) {
        args.push_back(a);
        offs.push_back(offs.back() + blocks);
    }
};

struct Step {
    std::vector<PassLaunch> passes;
    std::vector<StreamLaunch> streams;
    std::vector<int> order;   // >= 0: pass index, < 0: -(stream index) - 1
    // one launch per line-length class (compile-time plans for 2^8 .. 2^10)
    void pass(PassLaunch p) {
        std::vector<int> classes;
        for (const PassArgs& a : p.args) {
            const int cl = batch_lgm_class(a.lgm);
            if (std::find(classes.begin(), classes.end(), cl) == classes.end()) classes.push_back(cl);
        }
        for (int cl : classes) {
            PassLaunch q;
            q.v = p.v;
            q.fp64 = p.fp64;
            q.lgm = cl;
            for (size_t i = 0; i < p.args.size(); ++i) {
                if (batch_lgm_class(p.args[i].lgm) != cl) continue;
                // one line length per compile-time class, so one schedule
                q.v.rmax = p.irmax[i];
                q.threads = p.ithreads[i];
                q.args.push_back(p.args[i]);
                q.offs.push_back(q.offs.back() + (p.offs[i + 1] - p.offs[i]));
                q.ilds.push_back(p.ilds[i]);
                q.irmax.push_back(p.irmax[i]);
                q.ithreads.push_back(p.ithreads[i]);
                q.lds = std::max(q.lds, p.ilds[i]);
            }
            order.push_back((int)passes.size());
            passes.push_back(std::move(q));
        }
    }
    void strm(StreamLaunch s) {
        order.push_back(-(int)streams.size() - 1);
        streams.push_back(std::move(s));
    }
};

// Lay out the argument arrays of every launch of `st` in one blob.
void build_blob(Step& st, Blob& blob) {
    for (auto& p : st.passes) {
        p.a_off = blob.add(p.args);
        p.o_off = blob.add(p.offs);
    }
    for (auto& s : st.streams) {
        s.a_off = blob.add(s.args);
        s.o_off = blob.add(s.offs);
    }
}

// Enqueue the launches of `st` on stream `s`, argument arrays at device
// address `base` (laid out by build_blob).  attr_only: only raise the dynamic
// LDS limits of the pass kernels (no launch), as a graph capture needs.
// fork: a run of pass launches gives each line-length class its own stream
// (the first class stays on s_, the others on the batch's side streams,
// forked from s_ by an event); the classes touch disjoint instances, so their
// chains of passes are independent and run side by side.  Every side stream
// is joined back into s_ before the next streaming launch (which covers all
// instances) and at the end, so s_ orders everything that follows.
int launch_step(fnls_batch* B, const Step& st, char* base, hipStream_t s_, bool attr_only = false,
                bool fork = false) {
    fork = fork && !attr_only;
    int cls[fnls_batch::kSide + 1];   // class of s_ and of each side stream in use
    int ncls = 0;
    unsigned used = 0;                // side streams forked since the last join
    bool seg = false;                 // the fork event marks the start of the current run
    auto join = [&]() -> hipError_t {
        for (int k = 0; k < fnls_batch::kSide; ++k) {
            if (!(used & (1u << k))) continue;
            hipError_t e = hipEventRecord(B->ev_join[k], B->side[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s_, B->ev_join[k], 0);
            if (e != hipSuccess) return e;
        }
        used = 0;
        return hipSuccess;
    };
    for (int o : st.order) {
        hipError_t e = hipSuccess;
        if (o >= 0) {
            const PassLaunch& p = st.passes[o];
            const int count = (int)p.args.size();
            if (count == 0) continue;
            if (p.lds > B->ctx[0]->max_dyn_lds) return berr(B, FNLS_ERR_INVALID_ARG, "batch pass needs %zu B of LDS", p.lds);
            hipStream_t ps = s_;
            if (fork) {
                // the run's fork point precedes its first launch, so a side
                // stream waits only for what came before the run
                if (!seg) {
                    e = hipEventRecord(B->ev_fork, s_);
                    if (e != hipSuccess)
                        return berr(B, FNLS_ERR_HIP, "batched stream fork failed: %s", hipGetErrorString(e));
                    seg = true;
                }
                int k = 0;
                while (k < ncls && cls[k] != p.lgm) ++k;
                if (k == ncls && ncls <= fnls_batch::kSide) cls[ncls++] = p.lgm;
                if (k >= 1 && k <= fnls_batch::kSide) {
                    const int sk = k - 1;
                    if (!(used & (1u << sk))) {
                        e = hipStreamWaitEvent(B->side[sk], B->ev_fork, 0);
                        if (e != hipSuccess)
                            return berr(B, FNLS_ERR_HIP, "batched stream fork failed: %s", hipGetErrorString(e));
                        used |= 1u << sk;
                    }
                    ps = B->side[sk];
                }
            }
            e = launch_pass_batch(p.fp64, p.v, p.lgm, attr_only ? nullptr : reinterpret_cast<const PassArgs*>(base + p.a_off),
                                  reinterpret_cast<const int*>(base + p.o_off), count, p.offs.back(), p.lds,
                                  p.threads, ps);
        } else if (!attr_only) {
            seg = false;
            if (used) {
                e = join();
                if (e != hipSuccess) return berr(B, FNLS_ERR_HIP, "batched stream join failed: %s", hipGetErrorString(e));
            }
            const StreamLaunch& s = st.streams[-o - 1];
            const int count = (int)s.args.size();
            if (count == 0) continue;
            const StreamArgs* a = reinterpret_cast<const StreamArgs*>(base + s.a_off);
            const int* offs = reinterpret_cast<const int*>(base + s.o_off);
            switch (s.kind) {
                case 0: e = launch_cgs_batch(s.fp64, s.mode, a, offs, count, s.offs.back(), s_); break;
                case 1: e = launch_zupdate_batch(s.fp64, a, offs, count, s.offs.back(), s_); break;
                case 2: e = launch_prepare_batch(a, offs, count, s.offs.back(), s_); break;
                case 3: e = launch_precond_setup_batch(a, offs, count, s.offs.back(), s_); break;
                default: e = launch_finish_batch(a, count, s_); break;
            }
        }
        if (e != hipSuccess) return berr(B, FNLS_ERR_HIP, "batched launch failed: %s", hipGetErrorString(e));
    }
    if (used) {
        const hipError_t e = join();
        if (e != hipSuccess) return berr(B, FNLS_ERR_HIP, "batched stream join failed: %s", hipGetErrorString(e));
    }
    return FNLS_OK;
}

// Stage and enqueue the launches of `st` on the batch stream.
int run_step(fnls_batch* B, Step& st) {
    Blob blob;
    build_blob(st, blob);
    char* base = nullptr;
    int rc = stage(B, blob, &base);
    if (rc != FNLS_OK) return rc;
    return launch_step(B, st, base, B->stream);
}

// The launches of one Arnoldi iteration, ready to be enqueued once per
// iteration: either a staged argument table (eager launches) or a graph.
struct IterLaunch {
    Step st;
    char* base = nullptr;
    hipGraphExec_t ex = nullptr;
};

// Cache key of an iteration graph: the argument table and every launch shape.
std::vector<char> graph_key(const Step& st, const Blob& blob) {
    std::vector<int> sig;
    for (int o : st.order) {
        sig.push_back(o);
        if (o >= 0) {
            const PassLaunch& p = st.passes[o];
            sig.insert(sig.end(), {p.v.inm, p.v.ops, p.v.zm, p.v.outm, p.v.fin, p.v.rmax, p.fp64, p.lgm,
                                   (int)p.args.size(), p.offs.back(), (int)p.lds, p.threads});
        } else {
            const StreamLaunch& s = st.streams[-o - 1];
            sig.insert(sig.end(), {s.kind, s.fp64, s.mode, (int)s.args.size(), s.offs.back()});
        }
    }
    std::vector<char> key(blob.data);
    const char* sp = reinterpret_cast<const char*>(sig.data());
    key.insert(key.end(), sp, sp + sig.size() * sizeof(int));
    return key;
}

void drop_graph(GraphSlot& g) {
    if (g.ex) (void)hipGraphExecDestroy(g.ex);
    if (g.g) (void)hipGraphDestroy(g.g);
    g.ex = nullptr;
    g.g = nullptr;
    g.key.clear();
    g.used = 0;
}

// Prepare `it` (built by batch_arnoldi) for enqueueing.  Eager: stage its
// argument table in the ring.  Graph: find the cached graph of the same
// table and shapes, or copy the table into the least recently used slot and
// capture the launches (on the capture stream, which runs nothing) into a
// new graph.
int prepare_iteration(fnls_batch* B, IterLaunch& it, bool graph) {
    Blob blob;
    build_blob(it.st, blob);
    if (!graph) return stage(B, blob, &it.base);
    const size_t nbytes = align_up(blob.data.size());
    if (nbytes > B->slot_bytes)
        return berr(B, FNLS_ERR_WORKSPACE, "iteration argument table (%zu B) exceeds a graph slot", nbytes);
    std::vector<char> key = graph_key(it.st, blob);
    int slot = 0;
    for (int i = 0; i < kGraphSlots; ++i) {
        if (B->gs[i].ex && B->gs[i].key == key) {
            B->gs[i].used = ++B->tick;
            it.ex = B->gs[i].ex;
            return FNLS_OK;
        }
        if (B->gs[i].used < B->gs[slot].used) slot = i;
    }
    GraphSlot& g = B->gs[slot];
    drop_graph(g);
    char* dslot = B->dgraph + (size_t)slot * B->slot_bytes;
    // the table goes through the ring (stream-ordered after every earlier
    // launch, so no graph still reading this slot is overwritten)
    char* staged = nullptr;
    int rc = stage(B, blob, &staged);
    if (rc != FNLS_OK) return rc;
    BHIPCHK(B, hipMemcpyAsync(dslot, staged, blob.data.size(), hipMemcpyDeviceToDevice, B->stream));
    if ((rc = launch_step(B, it.st, dslot, B->cap, true)) != FNLS_OK) return rc;
    BHIPCHK(B, hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    rc = launch_step(B, it.st, dslot, B->cap, false, true);
    hipGraph_t graph_ = nullptr;
    const hipError_t e = hipStreamEndCapture(B->cap, &graph_);
    if (rc != FNLS_OK || e != hipSuccess) {
        if (graph_) (void)hipGraphDestroy(graph_);
        return rc != FNLS_OK ? rc : berr(B, FNLS_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, graph_, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph_);
        return berr(B, FNLS_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    g.g = graph_;
    g.ex = ex;
    g.key.swap(key);
    g.used = ++B->tick;
    ++B->captures;
    it.ex = ex;
    return FNLS_OK;
}

int launch_iteration(fnls_batch* B, IterLaunch& it) {
    if (it.ex) {
        BHIPCHK(B, hipGraphLaunch(it.ex, B->stream));
        ++B->replays;
        return FNLS_OK;
    }
    return launch_step(B, it.st, it.base, B->stream, false, true);
}

StreamArgs stream_base(fnls_ctx* c) {
    StreamArgs s;
    std::memset(&s, 0, sizeof s);
    s.N = c->N;
    s.pstride = c->lay.pstride;
    s.pin_stride = c->lay.pstride;
    s.st = c->st();
    s.hs = c->hs_dev;
    return s;
}

struct Inst {
    fnls_ctx* c;
    const double2* b;   // right-hand side (FP64)
    double2* x;
    Bufs bf;
};

// Toeplitz passes of y = (cD D + i ci I + cT T_d) x (FP64) into `fin` final mode on axis 0.
void add_matvec(const fnls_batch* B, Step& st, std::vector<Inst*>& live, const double2* const* xs, double cD,
                double ci, double cT,
                int fin, void* const* final_out, bool ir) {
    fnls_ctx* c0 = live[0]->c;
    const int d = c0->d;
    PassLaunch first;
    first.fp64 = 1;
    first.v = PassVariant{IN_PLAIN, P_TOEP, Z_NONE, OUT_ACC_FIRST, FIN_WRITE, 4};
    for (size_t k = 0; k < live.size(); ++k) {
        fnls_ctx* c = live[k]->c;
        Geo g = batch_geo(d, c->n, d - 1, true, B);
        PassArgs a = base_args(c, true, d - 1, g);
        a.in = xs[k];
        a.cD = cD;
        a.ci = ci;
        a.cT = cT;
        a.out = c->sc<char>(c->lay.acc);
        first.add(a, g);
    }
    st.pass(std::move(first));
    for (int ax = d - 2; ax >= 0; --ax) {
        const bool last = (ax == 0);
        PassLaunch p;
        p.fp64 = 1;
        p.v = PassVariant{IN_PLAIN, P_TOEP, Z_NONE, OUT_ACC_NEXT, last ? fin : FIN_WRITE, 4};
        for (size_t k = 0; k < live.size(); ++k) {
            fnls_ctx* c = live[k]->c;
            Geo g = batch_geo(d, c->n, ax, true, B);
            PassArgs a = base_args(c, true, ax, g);
            a.in = xs[k];
            a.acc_in = c->sc<char>(c->lay.acc);
            a.cT = cT;
            a.out = last ? final_out[k] : (void*)c->sc<char>(c->lay.acc);
            if (last && fin == FIN_RESID) {
                a.b64 = live[k]->b;
                a.r64 = c->sc<double2>(c->lay.r64);
                a.r32 = ir ? (void*)c->sc<float2>(c->lay.V) : nullptr;
                a.ir = ir ? 1 : 0;
                a.pout = c->sc<double2>(c->lay.pr);
                a.out = nullptr;
            }
            p.add(a, g);
        }
        st.pass(std::move(p));
    }
}

// The launches of one Arnoldi step of every live instance (the pass sequence
// of the single-instance path for d >= 2, with the basis scale in the first
// pass and a standalone Givens step).  The kernels read the iteration index j
// from each instance's state, so `st` serves every iteration of a cycle.
int batch_arnoldi(fnls_batch* B, std::vector<Inst*>& live, bool fp64, Step& st) {
    const int d = B->d;
    std::vector<void*> cur(live.size());
    int pp = 0;
    auto front = [&](int ax, int ops, bool first_pass) {
        PassLaunch p;
        p.fp64 = fp64 ? 1 : 0;
        p.v = PassVariant{first_pass ? IN_BASIS : IN_PLAIN, ops, Z_NONE, OUT_LINE, FIN_WRITE, 4};
        for (size_t k = 0; k < live.size(); ++k) {
            fnls_ctx* c = live[k]->c;
            Bufs& b = live[k]->bf;
            Geo g = batch_geo(d, c->n, ax, fp64, B);
            PassArgs a = base_args(c, fp64, ax, g);
            a.in = first_pass ? nullptr : cur[k];   // IN_BASIS: basis vector j
            a.v0 = b.v0;
            a.vbase = b.vbase;
            a.dev_j = 1;
            a.out = (pp == 0) ? b.t1 : b.t2;
            a.check_active = 1;
            cur[k] = a.out;
            p.add(a, g);
        }
        pp ^= 1;
        st.pass(std::move(p));
    };
    bool firstp = true;
    for (int ax = d - 1; ax >= 1; --ax) {
        front(ax, P_DST1, firstp);
        firstp = false;
    }
    front(0, P_DST1 | P_DIV | P_DST2, false);
    for (int ax = 1; ax <= d - 2; ++ax) front(ax, P_DST1, false);
    // last sine transform + scale (z_j kept) + first Toeplitz axis
    {
        PassLaunch p;
        p.fp64 = fp64 ? 1 : 0;
        p.v = PassVariant{IN_PLAIN, P_DST1 | P_SCALE | P_TOEP, Z_WRITE, OUT_ACC_FIRST, FIN_WRITE, 4};
        for (size_t k = 0; k < live.size(); ++k) {
            fnls_ctx* c = live[k]->c;
            Bufs& b = live[k]->bf;
            Geo g = batch_geo(d, c->n, d - 1, fp64, B);
            PassArgs a = base_args(c, fp64, d - 1, g);
            a.in = cur[k];
            a.zout = b.zbase;   // + j N
            a.jz = c->N;
            a.dev_j = 1;
            a.out = b.acc;
            a.cD = 1.0;
            a.ci = 1.0;
            a.cT = -1.0;
            a.check_active = 1;
            p.add(a, g);
        }
        st.pass(std::move(p));
    }
    for (int ax = d - 2; ax >= 0; --ax) {
        const bool last = (ax == 0);
        PassLaunch p;
        p.fp64 = fp64 ? 1 : 0;
        p.v = PassVariant{IN_PLAIN, P_TOEP, Z_NONE, OUT_ACC_NEXT, last ? FIN_WDOTS : FIN_WRITE, 4};
        for (size_t k = 0; k < live.size(); ++k) {
            fnls_ctx* c = live[k]->c;
            Bufs& b = live[k]->bf;
            Geo g = batch_geo(d, c->n, ax, fp64, B);
            PassArgs a = base_args(c, fp64, ax, g);
            a.in = b.zbase;   // z_j
            a.jin = c->N;
            a.acc_in = b.acc;
            a.cT = -1.0;
            a.check_active = 1;
            a.out = last ? b.vbase : b.acc;   // w = basis vector j + 1 at vbase + j N
            a.jout = last ? c->N : 0;
            a.v0 = b.v0;
            a.vbase = b.vbase;
            a.dev_j = 1;
            p.add(a, g);
        }
        st.pass(std::move(p));
    }
    // Gram-Schmidt updates and the Givens step
    StreamLaunch u0, u1, gv;
    u0.kind = 0;
    u0.mode = 0;
    u1.kind = 0;
    u1.mode = 1;
    u0.fp64 = u1.fp64 = fp64 ? 1 : 0;
    gv.kind = 4;
    for (size_t k = 0; k < live.size(); ++k) {
        fnls_ctx* c = live[k]->c;
        Bufs& b = live[k]->bf;
        StreamArgs s = stream_base(c);
        s.w = b.vbase;   // + j N
        s.jw = c->N;
        s.dev_j = 1;
        s.v0 = b.v0;
        s.vbase = b.vbase;
        s.check_active = 1;
        const int sb = stream_blocks(c->N);
        const int nb0 = batch_geo(d, c->n, 0, fp64, B).blocks;
        if (nb0 > kRedundantMax || sb > kRedundantMax)
            return berr(B, FNLS_ERR_INVALID_ARG, "instance too large for a batch (n = %d)", c->n);
        s.pin = c->sc<double2>(c->lay.p1);
        s.pin_nb = nb0;
        s.pout = c->sc<double2>(c->lay.p2);
        u0.add(s, sb);
        s.pin = c->sc<double2>(c->lay.p2);
        s.pin_nb = sb;
        s.pout = c->sc<double2>(c->lay.p3);
        u1.add(s, sb);
        StreamArgs f = stream_base(c);
        f.pin = c->sc<double2>(c->lay.p3);
        f.pin_nb = sb;
        f.check_active = 1;
        f.mode = 1;
        gv.add(f, 1);
    }
    st.strm(std::move(u0));
    st.strm(std::move(u1));
    st.strm(std::move(gv));
    return FNLS_OK;
}

// End of a cycle: x (+)= sum y_k z_k, FP64 residual and the decision.
int batch_cycle_final(fnls_batch* B, std::vector<Inst*>& live, bool fp64, int first) {
    const int d = B->d;
    Step st;
    StreamLaunch zu;
    zu.kind = 1;
    zu.fp64 = fp64 ? 1 : 0;
    std::vector<const double2*> xs(live.size());
    std::vector<void*> nulls(live.size(), nullptr);
    for (size_t k = 0; k < live.size(); ++k) {
        fnls_ctx* c = live[k]->c;
        StreamArgs s = stream_base(c);
        s.vbase = live[k]->bf.zbase;
        s.x64 = live[k]->x;
        s.mode = first;
        zu.add(s, stream_blocks(c->N));
        xs[k] = live[k]->x;
    }
    st.strm(std::move(zu));
    add_matvec(B, st, live, xs.data(), 1.0, 1.0, -1.0, FIN_RESID, nulls.data(), !fp64);
    StreamLaunch fr;
    fr.kind = 4;
    for (size_t k = 0; k < live.size(); ++k) {
        fnls_ctx* c = live[k]->c;
        StreamArgs s = stream_base(c);
        s.pin = c->sc<double2>(c->lay.pr);
        s.pin_nb = batch_geo(d, c->n, 0, true, B).blocks;
        s.mode = 2;
        s.ir = fp64 ? 0 : 1;
        fr.add(s, 1);
    }
    st.strm(std::move(fr));
    return run_step(B, st);
}

int batch_solve_impl(fnls_batch* B, std::vector<Inst>& inst, const fnls_opts* o, fnls_info* infos) {
    const bool fp64 = (o->precision == FNLS_FP64);
    const int n_inst = (int)inst.size();
    for (auto& I : inst)
        if (!I.c->have_D) return berr(B, FNLS_ERR_STATE, "an instance has no preconditioner setup");
    // configuration, ||b||, initial decision
    {
        Step st;
        StreamLaunch pr, fp;
        pr.kind = 2;
        fp.kind = 4;
        std::vector<StreamArgs> cfg;
        for (auto& I : inst) {
            fnls_ctx* c = I.c;
            StreamArgs s = stream_base(c);
            cfg.push_back(s);
            s.b64 = I.b;
            s.r32 = fp64 ? nullptr : (void*)c->sc<float2>(c->lay.V);
            s.pout = c->sc<double2>(c->lay.pr);
            const int sb = stream_blocks(c->N);
            if (sb > kRedundantMax) return berr(B, FNLS_ERR_INVALID_ARG, "instance too large for a batch");
            pr.add(s, sb);
            StreamArgs f = stream_base(c);
            f.pin = c->sc<double2>(c->lay.pr);
            f.pin_nb = sb;
            f.mode = 0;
            fp.add(f, 1);
        }
        Blob blob;
        const size_t cfg_off = blob.add(cfg);
        char* base = nullptr;
        int rc = stage(B, blob, &base);
        if (rc != FNLS_OK) return rc;
        hipError_t e = launch_config_batch(reinterpret_cast<const StreamArgs*>(base + cfg_off), n_inst,
                                           fp64 ? o->tol : o->inner_tol, o->tol, o->restart, o->maxit,
                                           fp64 ? o->fixed_iters : 0, fp64 ? (1 << 30) : o->max_outer, B->stream);
        if (e != hipSuccess) return berr(B, FNLS_ERR_HIP, "config launch failed: %s", hipGetErrorString(e));
        st.strm(std::move(pr));
        st.strm(std::move(fp));
        if ((rc = run_step(B, st)) != FNLS_OK) return rc;
    }
    BHIPCHK(B, hipStreamSynchronize(B->stream));
    std::vector<Inst*> live;
    int worst = FNLS_OK;
    for (int k = 0; k < n_inst; ++k) {
        const HostStatus& hs = *inst[k].c->hs;
        if (hs.done) {
            if (hs.nonfinite) {
                fill_info(inst[k].c, infos ? &infos[k] : nullptr, FNLS_ERR_NONFINITE);
                worst = FNLS_ERR_NONFINITE;
            } else {
                BHIPCHK(B, hipMemsetAsync(inst[k].x, 0, (size_t)inst[k].c->N * 16, B->stream));
                fill_info(inst[k].c, infos ? &infos[k] : nullptr, FNLS_OK);
                if (infos) infos[k].relres_true = 0.0;
            }
        } else {
            live.push_back(&inst[k]);
        }
    }
    int first = 1;
    const int lookahead = std::max(0, o->lookahead);
    while (!live.empty()) {
        for (Inst* I : live)
            I->bf = bufs(I->c, fp64, first ? (const void*)I->b : (const void*)I->c->sc<double2>(I->c->lay.r64));
        IterLaunch it;
        int rc = batch_arnoldi(B, live, fp64, it.st);
        if (rc == FNLS_OK) rc = prepare_iteration(B, it, o->graph != 0);
        if (rc != FNLS_OK) return rc;
        int issued = 0, waited = 0;
        while (true) {
            while (issued < o->restart && issued <= waited + lookahead) {
                rc = launch_iteration(B, it);
                if (rc != FNLS_OK) return rc;
                BHIPCHK(B, hipEventRecord(B->ev[issued % kEvents], B->stream));
                ++issued;
            }
            BHIPCHK(B, hipEventSynchronize(B->ev[waited % kEvents]));
            ++waited;
            bool all = true;
            for (Inst* I : live) {
                const HostStatus& hs = *I->c->hs;
                if (!(hs.stopped || hs.done)) all = false;
            }
            if (all || waited >= o->restart) break;
        }
        rc = batch_cycle_final(B, live, fp64, first);
        if (rc != FNLS_OK) return rc;
        first = 0;
        BHIPCHK(B, hipStreamSynchronize(B->stream));
        std::vector<Inst*> next;
        for (Inst* I : live) {
            const HostStatus& hs = *I->c->hs;
            const int k = (int)(I - inst.data());
            if (hs.nonfinite) {
                fill_info(I->c, infos ? &infos[k] : nullptr, FNLS_ERR_NONFINITE);
                worst = FNLS_ERR_NONFINITE;
            } else if (hs.done) {
                const int status = (fp64 && o->fixed_iters > 0) ? FNLS_OK
                                   : (hs.relres < o->tol ? FNLS_OK : FNLS_NOT_CONVERGED);
                fill_info(I->c, infos ? &infos[k] : nullptr, status);
                if (status == FNLS_NOT_CONVERGED && worst == FNLS_OK) worst = FNLS_NOT_CONVERGED;
            } else {
                next.push_back(I);
            }
        }
        live.swap(next);
    }
    return worst;
}

int batch_check(fnls_batch* B, const fnls_opts* opts, fnls_opts* o) {
    for (fnls_ctx* c : B->ctx) {
        int rc = resolve_opts(c, opts, o);
        if (rc != FNLS_OK) return berr(B, rc, "instance options: %s", c->err.c_str());
    }
    if (o->precision == FNLS_FP64 && o->fixed_iters > 0)
        return berr(B, FNLS_ERR_INVALID_ARG, "fixed_iters is not supported in batches");
    BHIPCHK(B, hipSetDevice(B->device));
    return FNLS_OK;
}

}  // namespace

extern "C" {

size_t fnls_batch_workspace_bytes(int count) {
    if (count < 1 || count > kMaxBatch) return 0;
    return batch_total_bytes(count);
}

int fnls_batch_create(fnls_batch** out, fnls_ctx* const* ctxs, int count, void* workspace, size_t bytes) {
    if (!out) return FNLS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!ctxs || count < 1 || count > kMaxBatch) return FNLS_ERR_INVALID_ARG;
    if (!workspace || bytes < batch_total_bytes(count) || ((uintptr_t)workspace % kAlign) != 0)
        return FNLS_ERR_WORKSPACE;
    for (int i = 0; i < count; ++i) {
        fnls_ctx* c = ctxs[i];
        if (!c || !c->assembled) return FNLS_ERR_STATE;
        if (c->device != ctxs[0]->device || c->stream != ctxs[0]->stream || c->d != ctxs[0]->d)
            return FNLS_ERR_INVALID_ARG;
        if (c->d < 2) return FNLS_ERR_INVALID_ARG;
        for (int a = 0; a < c->d; ++a)
            for (int p = 0; p < 2; ++p) {
                const Geo g = batch_geo(c->d, c->n, a, p == 1);
                if (g.G * g.L > kBatchThreads || (g.G * g.L) % 64 != 0 || g.lds > c->max_dyn_lds)
                    return FNLS_ERR_INVALID_ARG;
                if (g.blocks > kRedundantMax || stream_blocks(c->N) > kRedundantMax) return FNLS_ERR_INVALID_ARG;
            }
        for (int k = 0; k < i; ++k)
            if (ctxs[k] == c) return FNLS_ERR_INVALID_ARG;
    }
    fnls_batch* B = new (std::nothrow) fnls_batch();
    if (!B) return FNLS_ERR_HIP;
    B->count = count;
    B->ctx.assign(ctxs, ctxs + count);
    B->device = ctxs[0]->device;
    B->stream = ctxs[0]->stream;
    B->d = ctxs[0]->d;
    B->dring = reinterpret_cast<char*>(workspace);
    B->ring_bytes = batch_ring_bytes(count);
    B->dgraph = B->dring + B->ring_bytes;
    B->slot_bytes = batch_slot_bytes(count);
    if (hipSetDevice(B->device) != hipSuccess ||
        hipHostMalloc((void**)&B->hring, B->ring_bytes, hipHostMallocDefault) != hipSuccess) {
        delete B;
        return FNLS_ERR_HIP;
    }
    if (hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipHostFree(B->hring);
        delete B;
        return FNLS_ERR_HIP;
    }
    for (int i = 0; i < kEvents; ++i) {
        if (hipEventCreateWithFlags(&B->ev[i], hipEventDisableTiming) != hipSuccess) {
            for (int k = 0; k < i; ++k) (void)hipEventDestroy(B->ev[k]);
            (void)hipStreamDestroy(B->cap);
            (void)hipHostFree(B->hring);
            delete B;
            return FNLS_ERR_HIP;
        }
    }
    bool ok = hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < fnls_batch::kSide; ++k)
        ok = hipStreamCreateWithFlags(&B->side[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&B->ev_join[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        fnls_batch_destroy(B);
        return FNLS_ERR_HIP;
    }
    *out = B;
    return FNLS_OK;
}

void fnls_batch_destroy(fnls_batch* B) {
    if (!B) return;
    (void)hipSetDevice(B->device);
    (void)hipStreamSynchronize(B->stream);
    for (int i = 0; i < kEvents; ++i)
        if (B->ev[i]) (void)hipEventDestroy(B->ev[i]);
    for (int k = 0; k < fnls_batch::kSide; ++k) {
        if (B->side[k]) (void)hipStreamDestroy(B->side[k]);
        if (B->ev_join[k]) (void)hipEventDestroy(B->ev_join[k]);
    }
    if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
    for (int i = 0; i < kGraphSlots; ++i) drop_graph(B->gs[i]);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    if (B->hring) (void)hipHostFree(B->hring);
    delete B;
}

int fnls_batch_graph_stats(const fnls_batch* B, long long* captures, long long* replays) {
    if (!B) return FNLS_ERR_INVALID_ARG;
    if (captures) *captures = B->captures;
    if (replays) *replays = B->replays;
    return FNLS_OK;
}

int fnls_batch_solve(fnls_batch* B, const fnls_c128* const* bs, fnls_c128* const* xs, const fnls_opts* opts,
                     fnls_info* infos) {
    const TraceRange trace("fnls.batch_solve");
    if (!B) return FNLS_ERR_INVALID_ARG;
    if (!bs || !xs) return berr(B, FNLS_ERR_INVALID_ARG, "NULL pointer array");
    fnls_opts o;
    int rc = batch_check(B, opts, &o);
    if (rc != FNLS_OK) return rc;
    std::vector<Inst> inst(B->count);
    for (int k = 0; k < B->count; ++k) {
        if (!bs[k] || !xs[k] || (const void*)bs[k] == (const void*)xs[k])
            return berr(B, FNLS_ERR_INVALID_ARG, "instance %d: NULL or aliased vectors", k);
        inst[k].c = B->ctx[k];
        inst[k].b = reinterpret_cast<const double2*>(bs[k]);
        inst[k].x = reinterpret_cast<double2*>(xs[k]);
    }
    return batch_solve_impl(B, inst, &o, infos);
}

int fnls_batch_step(fnls_batch* B, const fnls_c128* const* u_prev, const fnls_c128* const* u_cur,
                    fnls_c128* const* u_next, const fnls_opts* opts, fnls_info* infos) {
    const TraceRange trace("fnls.batch_step");
    if (!B) return FNLS_ERR_INVALID_ARG;
    if (!u_prev || !u_cur || !u_next) return berr(B, FNLS_ERR_INVALID_ARG, "NULL pointer array");
    fnls_opts o;
    int rc = batch_check(B, opts, &o);
    if (rc != FNLS_OK) return rc;
    std::vector<Inst> inst(B->count);
    std::vector<Inst*> all;
    std::vector<const double2*> prev(B->count);
    std::vector<void*> bout(B->count);
    Step st;
    StreamLaunch ps;
    ps.kind = 3;
    for (int k = 0; k < B->count; ++k) {
        fnls_ctx* c = B->ctx[k];
        if (!u_prev[k] || !u_cur[k] || !u_next[k] || (const void*)u_next[k] == (const void*)u_prev[k] ||
            (const void*)u_next[k] == (const void*)u_cur[k])
            return berr(B, FNLS_ERR_INVALID_ARG, "instance %d: NULL or aliased vectors", k);
        c->tscale = 1.0;
        c->omega = c->omega > 0 ? c->omega : 1.0;
        StreamArgs s = stream_base(c);
        s.u = u_cur[k];
        s.V = c->Vpot;
        s.D64 = c->at<double>(c->lay.D64);
        s.D32 = c->at<float>(c->lay.D32);
        s.rho = c->rho;
        s.tau = c->tau;
        ps.add(s, (int)std::min<long long>(4096, (c->N + 255) / 256));
        c->have_D = 1;
        inst[k].c = c;
        inst[k].b = c->at<double2>(c->lay.bbuf);
        inst[k].x = reinterpret_cast<double2*>(u_next[k]);
        all.push_back(&inst[k]);
        prev[k] = reinterpret_cast<const double2*>(u_prev[k]);
        bout[k] = c->at<double2>(c->lay.bbuf);
    }
    st.strm(std::move(ps));
    // b = (iI + T_d - D) u_prev
    add_matvec(B, st, all, prev.data(), -1.0, 1.0, 1.0, FIN_WRITE, bout.data(), false);
    if ((rc = run_step(B, st)) != FNLS_OK) return rc;
    return batch_solve_impl(B, inst, &o, infos);
}

int fnls_batch_autotune(fnls_batch* B, const fnls_c128* const* b, int precision, int reps, int* classes) {
    const TraceRange trace("fnls.batch_autotune");
    if (!B) return FNLS_ERR_INVALID_ARG;
    if (classes) *classes = 0;
    if (!b) return berr(B, FNLS_ERR_INVALID_ARG, "NULL pointer array");
    if (precision != FNLS_FP64 && precision != FNLS_FP32_IR)
        return berr(B, FNLS_ERR_INVALID_ARG, "unknown precision");
    if (reps < 1 || reps > 1000) return berr(B, FNLS_ERR_INVALID_ARG, "reps must lie in [1, 1000]");
    fnls_opts in, o;
    fnls_default_opts(&in);
    in.precision = precision;
    for (fnls_ctx* c : B->ctx) in.restart = std::min(in.restart, c->restart_cap);
    int rc = batch_check(B, &in, &o);
    if (rc != FNLS_OK) return rc;
    // every instance solves its b into its adjoint buffer (not needed here)
    std::vector<Inst> inst(B->count);
    std::vector<int> ms_of;   // line lengths with a compile-time plan, in order of appearance
    for (int k = 0; k < B->count; ++k) {
        fnls_ctx* c = B->ctx[k];
        if (!b[k]) return berr(B, FNLS_ERR_INVALID_ARG, "instance %d: NULL vector", k);
        if (!c->have_D) return berr(B, FNLS_ERR_STATE, "instance %d has no preconditioner setup", k);
        inst[k].c = c;
        inst[k].b = reinterpret_cast<const double2*>(b[k]);
        inst[k].x = c->at<double2>(c->lay.adj);
        int lgm = 0;
        while ((1 << lgm) < c->m) ++lgm;
        if (batch_lgm_class(lgm) != 0 && std::find(ms_of.begin(), ms_of.end(), c->m) == ms_of.end())
            ms_of.push_back(c->m);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BHIPCHK(B, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return berr(B, FNLS_ERR_HIP, "hipEventCreate failed");
    }
    // time per batch solve: one untimed solve, then the fastest of two timed
    // runs of `reps` solves
    auto measure = [&](double* ms) -> int {
        int r = batch_solve_impl(B, inst, &o, nullptr);
        if (r < 0) return r;
        double best_t = 0.0;
        for (int trial = 0; trial < 2; ++trial) {
            if (hipEventRecord(e0, B->stream) != hipSuccess) return berr(B, FNLS_ERR_HIP, "hipEventRecord");
            for (int k = 0; k < reps; ++k) {
                r = batch_solve_impl(B, inst, &o, nullptr);
                if (r < 0) return r;
            }
            if (hipEventRecord(e1, B->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return berr(B, FNLS_ERR_HIP, "event timing failed");
            float t = 0.f;
            if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return berr(B, FNLS_ERR_HIP, "hipEventElapsedTime");
            const double per = (double)t / reps;
            if (trial == 0 || per < best_t) best_t = per;
        }
        *ms = best_t;
        return FNLS_OK;
    };
    const bool fp64 = precision == FNLS_FP64;
    double cur = 0.0;
    rc = measure(&cur);
    // coordinate descent: per line-length class, strided axes then the
    // contiguous axis, over radix {4, 8} x lines {1, 2, 4} (radix 4 with
    // lines 4 is the default shape of 1024 threads); a candidate replaces
    // the current schedule only when it is more than 1 % faster
    for (size_t ci = 0; ci < ms_of.size() && rc == FNLS_OK; ++ci) {
        for (int strided = 1; strided >= 0 && rc == FNLS_OK; --strided) {
            const long long key = (long long)ms_of[ci] * 4 + (fp64 ? 2 : 0) + strided;
            const auto had = B->sched.find(key);
            std::pair<int, int> best = had != B->sched.end() ? had->second : std::make_pair(4, 4);
            for (int rm : {4, 8}) {
                for (int li : {1, 2, 4}) {
                    if (rc != FNLS_OK || (rm == best.first && li == best.second)) continue;
                    B->sched[key] = std::make_pair(rm, li);
                    double t = 0.0;
                    rc = measure(&t);
                    if (rc == FNLS_OK && t < 0.99 * cur) {
                        cur = t;
                        best = std::make_pair(rm, li);
                    }
                }
            }
            B->sched[key] = best;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != FNLS_OK) return rc;
    if (classes) *classes = (int)ms_of.size();
    return FNLS_OK;
}

int fnls_batch_schedule(const fnls_batch* B, int n, int precision, int strided, int* rmax, int* lines) {
    if (!B || !rmax || !lines) return FNLS_ERR_INVALID_ARG;
    if (precision != FNLS_FP64 && precision != FNLS_FP32_IR) return FNLS_ERR_INVALID_ARG;
    const auto it = B->sched.find((long long)(n + 1) * 4 + (precision == FNLS_FP64 ? 2 : 0) + (strided ? 1 : 0));
    if (it == B->sched.end()) {
        *rmax = 0;
        *lines = 0;
    } else {
        *rmax = it->second.first;
        *lines = it->second.second;
    }
    return FNLS_OK;
}

const char* fnls_batch_last_error(const fnls_batch* B) { return B ? B->err.c_str() : "null batch"; }

}  // extern "C"
