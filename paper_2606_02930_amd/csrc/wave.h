// Wavefront-wide reductions of doubles by DPP lane permutations (sums within
// quads, half rows and rows, then the row broadcasts across the four rows),
// which stay in the vector register file instead of passing through LDS as
// cross-lane shuffles do.
#pragma once

#include <hip/hip_runtime.h>

namespace ite {

// One DPP data movement on both halves of a double; lanes of rows outside
// ROWS receive 0.
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double v) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Value of v in lane `lane` (uniform), returned to every lane.
__device__ inline double lane_value(double v, int lane) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, lane);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes, returned to every lane (lane 63 ends with the total).
__device__ inline double wave_sum(double v) {
    v += dpp_move<0xB1, 0xf>(v);     // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E, 0xf>(v);     // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141, 0xf>(v);    // row_half_mirror
    v += dpp_move<0x140, 0xf>(v);    // row_mirror
    v += dpp_move<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    return lane_value(v, 63);
}

// Largest value over the 64 lanes of non-negative v, returned to every lane
// (the zeros moved into the rows outside a broadcast's mask leave it as is).
__device__ inline double wave_max_nonneg(double v) {
    v = fmax(v, dpp_move<0xB1, 0xf>(v));
    v = fmax(v, dpp_move<0x4E, 0xf>(v));
    v = fmax(v, dpp_move<0x141, 0xf>(v));
    v = fmax(v, dpp_move<0x140, 0xf>(v));
    v = fmax(v, dpp_move<0x142, 0xa>(v));
    v = fmax(v, dpp_move<0x143, 0xc>(v));
    return lane_value(v, 63);
}

}  // namespace ite
