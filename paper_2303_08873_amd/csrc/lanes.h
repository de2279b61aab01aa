// Wave-level lane moves shared by the stencil kernels (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace ao {

// Cross-lane moves of a double by one lane with DPP wave shifts (plain VALU
// moves, no LDS traffic): from_left gives lane L the value of lane L-1,
// from_right the value of lane L+1.  Lanes 0 / 63 have no source and
// receive 0 (bound_ctrl); every caller overwrites them with its strip-edge
// loads or never uses them.  The whole wave must execute these.
__device__ __forceinline__ double from_left(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_right(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true));
}

// The same moves with a fill: lane 0 (from_left_or) or lane 63
// (from_right_or) receives its own `fill` instead of 0 -- the DPP move
// leaves a lane with no source unwritten (bound_ctrl off), so the strip
// edge costs a copy of `fill` instead of a select per half.
__device__ __forceinline__ double from_left_or(double v, double fill) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(
        __builtin_amdgcn_update_dpp(__double2hiint(fill), hi, 0x138, 0xf, 0xf, false),
        __builtin_amdgcn_update_dpp(__double2loint(fill), lo, 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_right_or(double v, double fill) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(
        __builtin_amdgcn_update_dpp(__double2hiint(fill), hi, 0x130, 0xf, 0xf, false),
        __builtin_amdgcn_update_dpp(__double2loint(fill), lo, 0x130, 0xf, 0xf, false));
}

// The wave's index within its block, as a wave-uniform value: the compiler
// then keeps what derives from it (row indices, row base addresses, row
// bounds tests) in scalar registers instead of one copy per lane.
__device__ __forceinline__ int wave_index() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

}  // namespace ao
