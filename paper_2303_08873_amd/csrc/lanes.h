// Wave-level lane moves shared by the stencil kernels (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace ao {

// Cross-lane moves of a double by one lane with DPP wave shifts (plain VALU
// moves, no LDS traffic): from_left gives lane L the value of lane L-1,
// from_right the value of lane L+1; lanes 0 / 63 keep their own value and
// are overwritten by the strip-edge loads.  The whole wave must execute them.
__device__ __forceinline__ double from_left(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_right(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false));
}

}  // namespace ao
