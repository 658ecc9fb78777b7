// Device arithmetic shared by the solver kernels: error-free transformations
// for the double-double residual and a deterministic 64-lane wave sum.
#pragma once

#include <hip/hip_runtime.h>

namespace spai {

// ---------------------------------------------------------------------------
// double-double helpers (error-free transformations)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    e = b - (s - a);
}

// (xh, xl) + (yh, yl), accurate double-word addition (Joldes, Muller, Popescu 2017)
__device__ __forceinline__ void dd_add(double xh, double xl, double yh, double yl, double& zh, double& zl) {
    double sh, sl, th, tl;
    two_sum(xh, yh, sh, sl);
    two_sum(xl, yl, th, tl);
    sl = sl + th;
    fast_two_sum(sh, sl, sh, sl);
    sl = sl + tl;
    fast_two_sum(sh, sl, zh, zl);
}

// Sum of one double over the 64 lanes of a wave (all lanes active), the same
// bits in every lane: row sums of 16 lanes by DPP moves (quad_perm xor 1, xor 2,
// row_ror 4, row_ror 8; no LDS round trip), then the four row sums read with
// readlane and added in a fixed order.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_mov<0xB1>(v);     // quad_perm(1, 0, 3, 2)
    v += dpp_mov<0x4E>(v);     // quad_perm(2, 3, 0, 1)
    v += dpp_mov<0x124>(v);    // row_ror:4
    v += dpp_mov<0x128>(v);    // row_ror:8
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float read_lane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// the same reduction tree for binary32
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x124>(v);
    v += dpp_mov<0x128>(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

}  // namespace spai
