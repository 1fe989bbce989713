// Device helpers shared by the kernel sources (gfx950): the FP64 MFMA tile,
// DPP lane moves and lane reads.
#pragma once

#include <hip/hip_runtime.h>

namespace cqfp {

typedef double d4 __attribute__((ext_vector_type(4)));
// read-only data that a wave reads at uniform addresses (scalar loads)
typedef __attribute__((address_space(4))) const double cdouble;

__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Cross-lane sums with DPP (no LDS round trip): a double moved by a DPP
// pattern on each 32-bit half; lanes a pattern does not write (rows outside
// row_mask) read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffll), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// DPP move with out-of-range source lanes reading zero (bound_ctrl)
template <int CTRL>
__device__ __forceinline__ double dpp_zero(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp(int(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

}  // namespace cqfp
