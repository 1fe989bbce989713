// Allocation-free direct history row: cq_history_noalloc (include/cqfp.h).
//
// The same sum as cq_history, S = sum_{i=1}^{n-1} d_i G^{n-i} ((3.8)/(3.17)),
// for callers that cannot allocate device memory. Its workspace (the weights
// and the slices' partial sums) is a file-scope device array, `scratch`, that
// every GPU the library runs on holds until the process ends. Host code never
// passes the array's name to a kernel: that name is a host-side stand-in. The
// array's device address is looked up once per device with
// hipGetSymbolAddress and kept in a per-device table.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "internal.h"
#include "kernels.h"

namespace {

// Workspace layout (doubles): weights d_0 .. d_{n-1} in the first
// kMaxLevels, partial sums [ks][M] in the next kMaxPart.
constexpr int64_t kMaxLevels = int64_t(1) << 20;
constexpr int64_t kMaxPart = int64_t(1) << 20;
constexpr int64_t kScratchDoubles = kMaxLevels + kMaxPart;  // 16 MiB

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
int scratch_ptr(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return cqfp::fail(CQ_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return cqfp::fail(CQ_EHIP, "device %d beyond the table of %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return cqfp::fail(CQ_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_ptr[dev];
    return CQ_OK;
}

// Weights d_i = tau^-beta g_i, i = 0..cnt-1, of (3.4) (scheme 1) or (3.12)
// (scheme 2) on the device, by the first-order recurrences of the host
// set-up: g_i = g_{i-1} (1 - (1+beta)/i) for (1-z)^beta, and for
// (3/2 - 2z + z^2/2)^beta, from p f' = beta p' f,
//   c_i = A_i c_{i-1} + B_i c_{i-2},  A_i = (beta-(i-1)) p1 / (p0 i),
//   B_i = (2 beta-(i-2)) p2 / (p0 i),  c_0 = p0^beta.
// Both recurrences are stable (the second one's parasitic solution decays
// like 3^-i). One lane runs the recurrence; its coefficients do not depend
// on earlier terms, so only one multiply (BE) or multiply-add (BDF2) per
// term sits on the dependency chain.
__global__ __launch_bounds__(64) void k_cq_weights(int scheme, double beta, double tau, int64_t cnt,
                                                   double* __restrict__ d) {
    if (threadIdx.x != 0) return;
    const double s = pow(tau, -beta);
    if (scheme == 1) {
        double g = 1.0;
        d[0] = s;
#pragma unroll 8
        for (int64_t i = 1; i < cnt; ++i) {
            g *= 1.0 - (1.0 + beta) / double(i);
            d[i] = s * g;
        }
        return;
    }
    const double p0 = 1.5, p1 = -2.0, p2 = 0.5;
    double cm2 = 0.0, cm1 = pow(p0, beta);
    d[0] = s * cm1;
#pragma unroll 8
    for (int64_t i = 1; i < cnt; ++i) {
        const double di = double(i);
        const double inv = 1.0 / (p0 * di);
        const double A = (beta - (di - 1.0)) * p1 * inv;
        const double B = (2.0 * beta - (di - 2.0)) * p2 * inv;
        const double c = fma(A, cm1, B * cm2);
        d[i] = s * c;
        cm2 = cm1;
        cm1 = c;
    }
}

}  // namespace

extern "C" int cq_history_noalloc(int32_t scheme, double beta, double tau, const double* G_hist, int64_t n,
                                  int64_t M, double* S_out, void* hip_stream) {
    using namespace cqfp;
    clear_error();
    if (scheme != 1 && scheme != 2) return fail(CQ_EINVAL, "scheme must be 1 or 2");
    if (!(beta > 0 && beta < 1)) return fail(CQ_EINVAL, "beta must lie in (0,1)");
    if (!(tau > 0) || !std::isfinite(tau)) return fail(CQ_EINVAL, "tau must be > 0");
    if (n < 1 || M < 1) return fail(CQ_EINVAL, "n and M must be >= 1");
    if (n > kMaxLevels)
        return fail(CQ_EINVAL, "n = %lld exceeds the static workspace of cq_history_noalloc (at most %lld levels)",
                    (long long)n, (long long)kMaxLevels);
    if (!G_hist || !S_out) return fail(CQ_EINVAL, "NULL array");
    double* ws = nullptr;
    int rc = scratch_ptr(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int ks = hist_row_slices(n, M, kMaxPart);
    if (n > 1) hipLaunchKernelGGL(k_cq_weights, dim3(1), dim3(64), 0, st, scheme, beta, tau, n, ws);
    launch_hist_row(G_hist, n, M, ws, ks, ws + kMaxLevels, S_out, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CQ_EHIP, "launch: %s", hipGetErrorString(e));
    return CQ_OK;
}
