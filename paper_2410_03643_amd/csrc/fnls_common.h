// Shared host/device definitions of libfnls: workspace-resident solver state,
// the host-visible status word, and the argument blocks of the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fnls {

// Largest restart length supported by the fixed-size Hessenberg state.
constexpr int kMaxRestart = 64;
// Elements per thread in the streaming (CGS update / setup) kernels.
constexpr int kEpt = 8;
constexpr int kStreamThreads = 512;

// GMRES state kept in device memory (inside the caller's workspace).  Only
// the last workgroup of a reduction kernel (and single-workgroup kernels)
// write it; everything else reads it.
struct GmresState {
    // rotated Hessenberg R (column j holds rows 0..j), Givens, rhs g
    double2 R[kMaxRestart][kMaxRestart];
    double cs[kMaxRestart];
    double2 sn[kMaxRestart];
    double2 g[kMaxRestart + 1];
    double2 hcol[kMaxRestart + 1];   // current column (h1 + h2)
    double2 coef[kMaxRestart + 1];   // coefficients for update / combination kernels
    double sigma[kMaxRestart + 1];   // raw basis vector i is stored as v_i / sigma_i
    double2 y[kMaxRestart];
    double hist[64];
    double refnorm;     // ||b|| (FP64) or ||r|| (IR inner): GMRES relative reference
    double bnorm;       // ||b||
    double wnorm0;      // ||A P^{-1} v_j|| before orthogonalisation
    double est;         // |g_{j+1}| / refnorm
    double relres;      // last recomputed ||b - A x|| / ||b||
    double tol;         // GMRES tolerance for the estimate
    double outer_tol;   // tolerance on the recomputed residual
    double inner_tol0;  // FP32-IR: requested inner tolerance (floor of the adaptive one)
    int j;              // current iteration within the cycle
    int k;              // basis size of the stopped cycle
    int total;          // total iterations
    int active;         // 1 while the current cycle is running
    int done;           // 1 when the whole solve has finished
    int breakdown;
    int restart, maxit, fixed_iters;
    int outer;          // completed cycles / refinement steps
    int max_outer;
    int nonfinite;
    unsigned counter;   // arrival counter for last-workgroup reductions
    unsigned seq;       // status sequence number
};

// Status mirrored into pinned host memory after every decision point.
struct HostStatus {
    unsigned seq;    // seqlock: odd while a report is written, else the last report's number
    int total;
    int stopped;     // 1: cycle stopped at this iteration
    int done;        // 1: whole solve finished
    int breakdown;
    int nonfinite;
    int outer;
    int pad;
    double est;
    double relres;
    double bnorm;
    double tol;      // the tolerance est is compared with (inner one in FP32-IR)
    double hist[64];
};

// IN_CGS: the second Gram-Schmidt update w -= sum_i h2_i v_i (h2 from the
// partials cgs_pin of the second-round dot products), w written back in
// place and its squared norm's per-workgroup partial to pout, then the line
// transforms of the next Arnoldi step's first pass run on w
enum InMode { IN_PLAIN = 0, IN_BASIS = 1, IN_COMBO = 2, IN_CGS = 3 };
enum OutMode { OUT_LINE = 0, OUT_ACC_FIRST = 1, OUT_ACC_NEXT = 2 };
enum FinalMode { FIN_WRITE = 0, FIN_WDOTS = 1, FIN_RESID = 2 };
enum ZMode { Z_NONE = 0, Z_WRITE = 1, Z_XSET = 2, Z_XADD = 3 };

// Arguments of the fused axis-pass kernel.  Element type of all "typed"
// vectors is complex<R> (R = float or double, the kernel's template type);
// x64 / b64 / r64 are always complex<double>.
struct PassArgs {
    // geometry
    int n, m, d, axis;
    int lgm;          // log2(m)
    int G;            // threads per line in the transform phases (power of two)
    int L;            // lines per workgroup (power of two)
    int lgG, lgL;     // log2 of G and L
    int pa, ls;       // LDS: slots of a line buffer (>= m) and line stride in slots
    unsigned magic_n; // ceil(2^32 / n) (n >= 2): e / n == umulhi(e, magic_n) for e < 2^16
    long long stride; // element stride along the axis
    long long nlines; // n^(d-1)
    long long N;      // n^d
    // input
    const void* in;       // IN_PLAIN / IN_BASIS source (typed)
    const void* v0;       // basis vector 0 (typed)
    void* vbase;          // basis vector i >= 1 at vbase + (i-1) * N (typed)
    int basis_j;          // IN_BASIS: index j; FIN_WDOTS: dots with 0..basis_j
    // tables
    const void* tw;       // W_{2m}^s, s < 2m (typed complex)
    const void* sym_e;    // circulant symbol, even frequencies, pre-scaled (typed real)
    const void* sym_o;    // odd frequencies
    const void* lam;      // lambda_k at index k (typed real)
    const void* D;        // diagonal (typed real)
    double tscale;        // multiplies symbol and lambda (0.5 for the starter)
    double omega;
    // outputs
    void* out;            // typed output (line data / acc / w / residual when typed)
    void* zout;           // Z_WRITE target (typed)
    double2* x64;         // Z_XSET / Z_XADD target
    const void* acc_in;   // OUT_ACC_NEXT accumulator (typed)
    const void* tin;      // Toeplitz input when it is not the line data (typed)
    const double2* b64;   // FIN_RESID: right-hand side
    double2* r64;         // FIN_RESID: residual (FP64)
    void* r32;            // FIN_RESID: optional complex64 copy of the residual
    double cD, ci, cT;    // OUT_ACC_FIRST coefficients
    // reductions
    double2* pout;        // per-workgroup partials written here, layout [i][pstride]
    int pstride;
    GmresState* st;
    HostStatus* hs;
    int check_active;     // 1: return at once if st->active == 0; 2: unless st->active == 0 and st->k == guard_k
    int guard_k;          // check_active 2: the stopped cycle's basis size the launch was enqueued for
    int first_cycle;      // Z_XADD: 1 = set x (first correction), 0 = accumulate
    int zsum, z32;        // IN_COMBO: 1 = sum_k y_k z_k with z_k at vbase + k N (z32: complex64)
    int ir;               // FIN_RESID: 1 = refinement step of FP32-IR
    // Givens step of the previous Arnoldi iteration in one extra workgroup
    // (logical block 0) of this launch: partials of ||w||^2 in gpin
    int gfuse;
    const double2* gpin;
    int gpin_nb, gpin_stride;
    // IN_CGS: partials of the second-round dot products (nv = basis_j + 1
    // values, layout [i][cgs_stride], cgs_nb producer workgroups)
    const double2* cgs_pin;
    int cgs_nb, cgs_stride;
    // batched launches: with dev_j set the iteration index j is read from
    // st->j when the kernel starts (one argument table serves every Arnoldi
    // iteration of a cycle).  Then basis_j = j; IN_BASIS reads basis vector j;
    // in / out / zout are bases advanced by j * jin / jout / jz elements.
    int dev_j;
    long long jin, jout, jz;
};

struct StreamArgs {
    long long N;
    const void* u;        // precond_setup input (complex128)
    const double* V;      // optional potential
    double* D64;
    float* D32;
    double rho, tau;
    // CGS update
    void* w;              // typed vector being orthogonalised
    const void* v0;
    const void* vbase;
    int nv;               // number of basis vectors involved (j + 1)
    // norm / prepare
    const double2* b64;
    void* r32;            // optional complex64 copy
    const double2* pin;   // partials of the producer kernel, layout [i][pin_stride]
    int pin_nb;           // number of producer workgroups
    int pin_stride;       // distance between the partials of consecutive values
    double2* pout;        // this kernel's partials, layout [i][pstride]
    int pstride;
    GmresState* st;
    HostStatus* hs;
    int check_active;     // as PassArgs::check_active
    int guard_k;
    int mode;             // k_finish: FinishKind; k_zupdate: 1 = first correction (x = 0 before)
    int ir;               // k_finish residual decision: 1 = refinement step of FP32-IR
    double2* x64;         // k_zupdate: the iterate
    // k_finish prepare: the solve's limits (GMRES tolerance, outer tolerance,
    // restart, iteration cap, fixed iteration count, refinement steps) and
    // the first value of the status sequence
    double cfg_tol, cfg_outer_tol;
    int cfg_restart, cfg_maxit, cfg_fixed_iters, cfg_max_outer;
    unsigned cfg_seq0;
    // batched CGS launches: with dev_j set, j = st->j when the kernel starts,
    // nv = j + 1 and w is advanced by j * jw elements
    int dev_j;
    long long jw;
};

// Reverse mode of one step: gradient accumulation after the adjoint solve.
struct AdjointArgs {
    long long N;
    const double2* sol;      // A^{-1} conj(g_next) = conj(lam)
    const double2* w;        // B sol (so B^H lam = conj(w))
    const double2* u_prev;
    const double2* u_cur;
    const double2* u_next;
    double2* g_prev;         // += conj(w) (+ the u_cur term when g_cur is null)
    double2* g_cur;          // += 2 dt rho g_D u_cur (may be null: added to g_prev)
    double* g_V;             // += dt g_D (may be null)
    double dt, rho;          // time step of the system (dt/2 for the starter)
};

}  // namespace fnls
