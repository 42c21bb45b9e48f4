// Instantiations of the fused batched kernel for uint16 ROIs (row values held as uint32).
#include "slice_block.h"

namespace dpm {
hipError_t launch_slice_block_u16(int nd, const BlockArgs &a, int items, size_t lds, hipStream_t st) {
    return launch_block_nd<uint16_t, uint32_t>(nd, a, items, lds, st);
}
}  // namespace dpm
