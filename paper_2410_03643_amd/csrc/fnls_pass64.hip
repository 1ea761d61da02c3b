// Axis-pass kernels of libfnls in FP64 (complex128 vectors).
#include "fnls_pass.hpp"

namespace fnls {

hipError_t launch_pass_f64(const PassVariant& v, const PassArgs& a, int blocks, size_t lds, hipStream_t s,
                          const LaunchEvents* te) {
    return dispatch_pass<double>(v, a, blocks, lds, s, te);
}

hipError_t launch_pass_batch_f64(const PassVariant& v, int lgm, const PassArgs* args, const int* offs, int count,
                                int blocks, size_t lds, int threads, hipStream_t s) {
    return dispatch_pass_batch<double>(v, lgm, args, offs, count, blocks, lds, threads, s);
}

}  // namespace fnls
