// Internal interface of the served loop's resident 2D moments (not part of the C ABI).
//
// A completed request may keep, on the device, the 2D moments of each side of each of its
// projection images (Section 3.1's images, their eq. 1 moments): one "tile" per image side
// (slot s = 2 d + side), part[s][k][q][nlr] for k, q <= K -- the layout the recombination
// kernel reads, with tile s holding slot s.  A later query recombines them (Section 3.2)
// for any order <= K without reading the volume again.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace dpm {

// Sum the power-sum tiles of every slot s < 2 (K + 1) of one volume into out[s][k][q].
//   single volume: the tiles of slot s are [tile0[s], tile0[s + 1]) (roi == null);
//   batched ROI:   the tiles of the ROI's non-empty slots follow rd->tile0 in slot order,
//                  ceil(M / 16) per slot (the layout of the batched power sums).
struct CollapseArgs {
    const uint32_t *part;   // tile partials, [tile][K + 1][K + 1][nlr]
    const RoiDesc *roi;     // device descriptor of the ROI, or null
    int32_t tile0[NSLOT + 1];
    int32_t K, nlr;
    uint32_t *out;          // [2 (K + 1)][K + 1][K + 1][nlr]
};
hipError_t launch_collapse(const CollapseArgs &a, hipStream_t st);

// out[s][k][q] (order Ko) = in[s][k][q] (order Ki >= Ko) for s < 2 (Ko + 1).
hipError_t launch_restride(const uint32_t *in, int Ki, uint32_t *out, int Ko, int nlr, hipStream_t st);

}  // namespace dpm
