// Exact multiword sums across lanes by DPP register moves (no LDS permutes): inclusive
// scans within 16-lane rows and across the four rows of a wave.
#pragma once
#include <hip/hip_runtime.h>

#include "mw.h"

namespace dpm {

// s += s moved by the DPP control CTRL, on the rows in ROWS; lanes with no source (or
// in other rows) add zero.
template <int CTRL, int ROWS, int N>
__device__ __forceinline__ void add_dpp(mw::Int<N> &s) {
    mw::Int<N> o;
#pragma unroll
    for (int l = 0; l < N; ++l) o.w[l] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s.w[l], CTRL, ROWS, 0xF, false);
    mw::add(s, o);
}

// The sum of the 16 lanes of every aligned 16-lane group (DPP row) ends in the row's last
// lane: shifts of 1, 2, 4 and 8 lanes.
template <int N>
__device__ __forceinline__ void row16_sum_last(mw::Int<N> &s) {
    add_dpp<0x111, 0xF>(s);  // row_shr:1
    add_dpp<0x112, 0xF>(s);  // row_shr:2
    add_dpp<0x114, 0xF>(s);  // row_shr:4
    add_dpp<0x118, 0xF>(s);  // row_shr:8
}

// The sum of all 64 lanes ends in lane 63: row sums, then lane 15 of rows 0 and 2 added
// into rows 1 and 3 (row_bcast:15), then lane 31 into rows 2 and 3 (row_bcast:31).
template <int N>
__device__ __forceinline__ void wave_sum_last(mw::Int<N> &s) {
    row16_sum_last(s);
    add_dpp<0x142, 0xA>(s);
    add_dpp<0x143, 0xC>(s);
}

}  // namespace dpm
