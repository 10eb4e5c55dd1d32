// Fixed-order FP64 reductions across a wavefront with DPP row operations
// (no LDS round trips): an inclusive scan, whose last lane holds the
// wavefront's sum.
#pragma once

#include <hip/hip_runtime.h>

namespace wnnc {

// One DPP step on an FP64 value: each lane receives the value of the lane
// selected by CTRL (as its two 32-bit halves), 0 where that lane is outside
// the row or the lane's row is not in ROW_MASK.
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_f64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Inclusive scan over the 64 lanes: within rows of 16 (row shifts 1, 2, 4,
// 8), then lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31 into rows
// 2 and 3.  Fixed order: reproducible.
__device__ inline double wave_scan(double x) {
    x += dpp_f64<0x111, 0xf>(x);
    x += dpp_f64<0x112, 0xf>(x);
    x += dpp_f64<0x114, 0xf>(x);
    x += dpp_f64<0x118, 0xf>(x);
    x += dpp_f64<0x142, 0xa>(x);
    x += dpp_f64<0x143, 0xc>(x);
    return x;
}

}  // namespace wnnc
