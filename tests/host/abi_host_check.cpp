// Host-only exercise of libfnls's C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of fnls_api.hip (see
// tests/test_host_sanitizers.py).  No GPU is used: the kernel launchers are
// replaced below by stubs that report "no device", so every path reached here
// is host code -- argument checking, workspace layout arithmetic, the status
// acceptance rule, option defaults, error strings and the NULL-context and
// no-device paths.  Prints "OK <checks>" on success, exits non-zero on the
// first failed check (or the sanitizers abort).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>

#include "../../include/fnls.h"
#include "../../paper_2410_03643_amd/csrc/fnls_launch.h"

// ---- launcher stubs: no kernels in this program ----
namespace fnls {
hipError_t launch_pass(int, const PassVariant&, const PassArgs&, int, size_t, hipStream_t, const LaunchEvents*) {
    return hipErrorNoDevice;
}
hipError_t launch_pass_f64(const PassVariant&, const PassArgs&, int, size_t, hipStream_t, const LaunchEvents*) {
    return hipErrorNoDevice;
}
hipError_t launch_pass_f32(const PassVariant&, const PassArgs&, int, size_t, hipStream_t, const LaunchEvents*) {
    return hipErrorNoDevice;
}
hipError_t launch_pass_batch_f64(const PassVariant&, int, const PassArgs*, const int*, int, int, size_t, int, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_pass_batch_f32(const PassVariant&, int, const PassArgs*, const int*, int, int, size_t, int, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_precond_setup(const StreamArgs&, int, hipStream_t, const LaunchEvents*) { return hipErrorNoDevice; }
hipError_t launch_prepare(const StreamArgs&, int, hipStream_t, const LaunchEvents*) { return hipErrorNoDevice; }
hipError_t launch_finish(const StreamArgs&, hipStream_t, const LaunchEvents*) { return hipErrorNoDevice; }
hipError_t launch_reduce_chunks(const StreamArgs&, int, hipStream_t, const LaunchEvents*) { return hipErrorNoDevice; }
hipError_t launch_cgs(int, int, const StreamArgs&, int, hipStream_t, const LaunchEvents*) { return hipErrorNoDevice; }
hipError_t launch_conj(const double2*, double2*, long long, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_adjoint(const AdjointArgs&, hipStream_t, const LaunchEvents*) { return hipErrorNoDevice; }
hipError_t launch_pass_batch(int, const PassVariant&, int, const PassArgs*, const int*, int, int, size_t, int,
                             hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_cgs_batch(int, int, const StreamArgs*, const int*, int, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_zupdate_batch(int, const StreamArgs*, const int*, int, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_prepare_batch(const StreamArgs*, const int*, int, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_precond_setup_batch(const StreamArgs*, const int*, int, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_finish_batch(const StreamArgs*, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_config_batch(const StreamArgs*, int, double, double, int, int, int, int, hipStream_t) {
    return hipErrorNoDevice;
}
}  // namespace fnls

static int checks = 0;
#define CHECK(cond)                                                                 \
    do {                                                                            \
        ++checks;                                                                   \
        if (!(cond)) {                                                              \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                               \
        }                                                                           \
    } while (0)

int main() {
    // option defaults and status strings
    fnls_opts o;
    std::memset(&o, 0xff, sizeof o);
    fnls_default_opts(&o);
    fnls_default_opts(nullptr);
    CHECK(o.tol == 1e-10 && o.restart == 30 && o.maxit == 2000 && o.precision == FNLS_FP64);
    CHECK(o.lookahead == 1 && o.poll_delay_us == 0 && o.fixed_iters == 0 && o.graph == 0);
    for (int code = -8; code <= 2; ++code) CHECK(std::strlen(fnls_status_string(code)) > 0);

    // workspace sizes: zero for invalid sizes, growing with the restart
    for (int d = 0; d <= 4; ++d)
        for (int n : {0, 1, 2, 3, 7, 62, 63, 255, 511, 1023, 1024, 2047, -5})
            for (int r : {-1, 0, 1, 2, 30, 64, 65}) {
                const size_t b = fnls_workspace_bytes(d, n, r);
                const bool ok = d >= 1 && d <= 3 && n >= 1 && n <= 1023 && ((n + 1) & n) == 0 && r >= 1 && r <= 64;
                CHECK((b != 0) == ok);
                // each restart slot adds two vectors (256-byte aligned, so
                // tiny grids may round to the same size)
                if (ok && r > 1) {
                    size_t N = 1;
                    for (int k = 0; k < d; ++k) N *= (size_t)n;
                    CHECK(b + 512 >= fnls_workspace_bytes(d, n, r - 1) + 2 * 16 * N);
                }
            }
    for (int cnt : {-1, 0, 1, 64, 4096, 4097}) CHECK((fnls_batch_workspace_bytes(cnt) != 0) == (cnt >= 1 && cnt <= 4096));

    // fnls_assemble's argument checks without a context
    const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
    void* ws = reinterpret_cast<void*>(static_cast<uintptr_t>(1) << 20);   // aligned, never dereferenced
    const size_t need = fnls_workspace_bytes(2, 63, 1);
    char msg[128];
    CHECK(fnls_check_assemble(1.5, 2.0, 2, 63, 0.3, 0.01, ws, need, msg, sizeof msg) == FNLS_OK && msg[0] == 0);
    struct Bad { double a, rho; int d, n; double h, tau; uintptr_t w; size_t bytes; int code; };
    const Bad bad[] = {
        {1.0, 2, 2, 63, 0.3, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG}, {nan, 2, 2, 63, 0.3, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG},
        {2.5, 2, 2, 63, 0.3, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG}, {1.5, -1, 2, 63, 0.3, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG},
        {1.5, inf, 2, 63, 0.3, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG}, {1.5, 2, 0, 63, 0.3, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG},
        {1.5, 2, 4, 63, 0.3, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG}, {1.5, 2, 2, 62, 0.3, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG},
        {1.5, 2, 2, 2047, 0.3, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG}, {1.5, 2, 2, 63, 0.0, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG},
        {1.5, 2, 2, 63, nan, 0.01, 1u << 20, need, FNLS_ERR_INVALID_ARG}, {1.5, 2, 2, 63, 0.3, -1.0, 1u << 20, need, FNLS_ERR_INVALID_ARG},
        {1.5, 2, 2, 63, 0.3, inf, 1u << 20, need, FNLS_ERR_INVALID_ARG}, {1.5, 2, 2, 63, 0.3, 0.01, 0, need, FNLS_ERR_WORKSPACE},
        {1.5, 2, 2, 63, 0.3, 0.01, (1u << 20) + 8, need, FNLS_ERR_WORKSPACE}, {1.5, 2, 2, 63, 0.3, 0.01, 1u << 20, need - 1, FNLS_ERR_WORKSPACE},
    };
    for (const Bad& b : bad) {
        msg[0] = 'x';
        CHECK(fnls_check_assemble(b.a, b.rho, b.d, b.n, b.h, b.tau, reinterpret_cast<void*>(b.w), b.bytes, msg,
                                  sizeof msg) == b.code);
        CHECK(std::strlen(msg) > 0 && std::strlen(msg) < sizeof msg);
        char tiny[4];   // truncated messages stay terminated
        CHECK(fnls_check_assemble(b.a, b.rho, b.d, b.n, b.h, b.tau, reinterpret_cast<void*>(b.w), b.bytes, tiny,
                                  sizeof tiny) == b.code && std::strlen(tiny) < sizeof tiny);
        CHECK(fnls_check_assemble(b.a, b.rho, b.d, b.n, b.h, b.tau, reinterpret_cast<void*>(b.w), b.bytes, nullptr,
                                  0) == b.code);
    }

    // the status acceptance rule over the 32-bit wrap
    const unsigned stride = 1u << 24;
    for (unsigned solve : {1u, 2u, 255u, 256u, 257u, 1000u}) {
        const unsigned base = solve * stride, prev = (solve - 1) * stride;
        CHECK(!fnls_status_report_accepted(base, base, base, 5, 0, 5));
        for (unsigned k : {1u, 2u, 3u, 1000u, (1u << 21) + 64u}) {
            CHECK(fnls_status_report_accepted(base, base + 2 * k, base + 2 * k, 5, 0, 5));
            CHECK(!fnls_status_report_accepted(base, base + 2 * k - 1, base + 2 * k - 1, 5, 0, 5));
            CHECK(!fnls_status_report_accepted(base, prev + 2 * k, prev + 2 * k, 5, 0, 5));
            CHECK(!fnls_status_report_accepted(base, base + 2 * k, base + 2 * k + 2, 5, 0, 5));
            CHECK(!fnls_status_report_accepted(base, base + 2 * k, base + 2 * k, 4, 0, 5));
            CHECK(fnls_status_report_accepted(base, base + 2 * k, base + 2 * k, 0, 1, 5));
        }
    }

    // NULL contexts and batches
    CHECK(fnls_assemble(nullptr, 1.5, 2, 2, 63, 0.3, 0.01, ws, need) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_precond_setup(nullptr, nullptr, nullptr, 1.0) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_apply_A(nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_apply_A_c64(nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_apply_precond(nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_apply_precond_c64(nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_rhs(nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_solve(nullptr, nullptr, nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_solve_noalloc(nullptr, nullptr, nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_step(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_first_step(nullptr, nullptr, nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_set_potential(nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_step_backward(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                             nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_first_step_backward(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
          FNLS_ERR_INVALID_ARG);
    CHECK(fnls_timing(nullptr, 1) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_timing_report(nullptr, nullptr, 0) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_set_pass_config(nullptr, 0, 0, 4, 1) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_autotune(nullptr, nullptr, 0, 1, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_get_host_stats(nullptr, nullptr, 1) == FNLS_ERR_INVALID_ARG);
    CHECK(std::strcmp(fnls_last_error(nullptr), "null context") == 0);
    fnls_destroy(nullptr);
    CHECK(fnls_batch_create(nullptr, nullptr, 0, nullptr, 0) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_batch_solve(nullptr, nullptr, nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_batch_step(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(fnls_batch_autotune(nullptr, nullptr, 0, 1, nullptr) == FNLS_ERR_INVALID_ARG);
    int rm = -1, li = -1;
    CHECK(fnls_batch_schedule(nullptr, 1023, 0, 1, &rm, &li) == FNLS_ERR_INVALID_ARG && rm == -1 && li == -1);
    CHECK(fnls_batch_graph_stats(nullptr, nullptr, nullptr) == FNLS_ERR_INVALID_ARG);
    CHECK(std::strcmp(fnls_batch_last_error(nullptr), "null batch") == 0);
    fnls_batch_destroy(nullptr);

    // no device: creation fails cleanly
    fnls_ctx* c = reinterpret_cast<fnls_ctx*>(0x1);
    CHECK(fnls_create(nullptr, 0, nullptr) == FNLS_ERR_INVALID_ARG);
    const int rc = fnls_create(&c, 0, nullptr);
    CHECK(rc == FNLS_ERR_NO_DEVICE && c == nullptr);
    CHECK(fnls_create(&c, -1, nullptr) == FNLS_ERR_NO_DEVICE && c == nullptr);

    std::printf("OK %d\n", checks);
    return 0;
}
