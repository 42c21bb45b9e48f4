// Instantiations of the fused batched kernel for uint8 ROIs (row values held as uint16
// when every line sum fits, else as uint32).
#include "slice_block.h"

namespace dpm {
hipError_t launch_slice_block_u8(int rowbytes, int nd, const BlockArgs &a, int items, size_t lds, hipStream_t st) {
    return rowbytes == 2 ? launch_block_nd<uint8_t, uint16_t>(nd, a, items, lds, st)
                         : launch_block_nd<uint8_t, uint32_t>(nd, a, items, lds, st);
}
}  // namespace dpm
