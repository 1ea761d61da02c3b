// Host-side launch entry points of the kernels in fnls_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "fnls_common.h"

namespace fnls {

struct PassVariant {
    int inm, ops, zm, outm, fin;
    int rmax;   // largest FFT radix (4, 8, 16); threads per line G = m / rmax
};

enum PassOps { P_DST1 = 1, P_DIV = 2, P_DST2 = 4, P_SCALE = 8, P_TOEP = 16 };

// Optional pair of events that the runtime records at the start and at the end
// of one kernel's execution (hipExtLaunchKernel); nullptr: plain launch.
struct LaunchEvents {
    hipEvent_t start, stop;
};

hipError_t launch_pass(int fp64, const PassVariant& v, const PassArgs& a, int blocks, size_t lds, hipStream_t s,
                       const LaunchEvents* te = nullptr);
// per-precision halves of launch_pass / launch_pass_batch (fnls_pass64.hip, fnls_pass32.hip)
hipError_t launch_pass_f64(const PassVariant& v, const PassArgs& a, int blocks, size_t lds, hipStream_t s,
                           const LaunchEvents* te);
hipError_t launch_pass_f32(const PassVariant& v, const PassArgs& a, int blocks, size_t lds, hipStream_t s,
                           const LaunchEvents* te);
hipError_t launch_pass_batch_f64(const PassVariant& v, int lgm, const PassArgs* args, const int* offs, int count,
                                 int blocks, size_t lds, int threads, hipStream_t s);
hipError_t launch_pass_batch_f32(const PassVariant& v, int lgm, const PassArgs* args, const int* offs, int count,
                                 int blocks, size_t lds, int threads, hipStream_t s);
hipError_t launch_precond_setup(const StreamArgs& a, int blocks, hipStream_t s, const LaunchEvents* te = nullptr);
hipError_t launch_prepare(const StreamArgs& a, int blocks, hipStream_t s, const LaunchEvents* te = nullptr);
// one workgroup: StreamArgs::mode = 0 prepare (configures the solve from the cfg_ fields), 1 Givens,
// 2 residual
hipError_t launch_finish(const StreamArgs& a, hipStream_t s, const LaunchEvents* te = nullptr);
// `chunks` workgroups: workgroup c sums a contiguous chunk of the a.pin_nb producers of each of the
// a.nv values (a.pin, a.pin_stride) into a.pout[i * chunks + c]
hipError_t launch_reduce_chunks(const StreamArgs& a, int chunks, hipStream_t s, const LaunchEvents* te = nullptr);
hipError_t launch_cgs(int fp64, int mode, const StreamArgs& a, int blocks, hipStream_t s,
                      const LaunchEvents* te = nullptr);
// out = conj(in), complex128
hipError_t launch_conj(const double2* in, double2* out, long long N, hipStream_t s);
// gradient accumulation of one step's reverse mode
hipError_t launch_adjoint(const AdjointArgs& a, hipStream_t s, const LaunchEvents* te = nullptr);
// batched launches: instance i owns the blocks [offs[i], offs[i+1]); args / offs in device memory.
// lgm in {8, 9, 10}: every instance of the pass launch has lines of length 2^lgm (compile-time
// plan); anything else: the generic plan.  args == nullptr: only raise the kernel's LDS limit.
hipError_t launch_pass_batch(int fp64, const PassVariant& v, int lgm, const PassArgs* args, const int* offs,
                             int count, int blocks, size_t lds, int threads, hipStream_t s);
hipError_t launch_cgs_batch(int fp64, int mode, const StreamArgs* args, const int* offs, int count, int blocks,
                            hipStream_t s);
hipError_t launch_zupdate_batch(int fp64, const StreamArgs* args, const int* offs, int count, int blocks,
                                hipStream_t s);
hipError_t launch_prepare_batch(const StreamArgs* args, const int* offs, int count, int blocks, hipStream_t s);
hipError_t launch_precond_setup_batch(const StreamArgs* args, const int* offs, int count, int blocks,
                                      hipStream_t s);
hipError_t launch_finish_batch(const StreamArgs* args, int count, hipStream_t s);   // one workgroup per instance
hipError_t launch_config_batch(const StreamArgs* args, int count, double tol, double outer_tol, int restart,
                               int maxit, int fixed_iters, int max_outer, hipStream_t s);

}  // namespace fnls
