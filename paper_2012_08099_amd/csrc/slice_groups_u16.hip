// Instantiations of the one-launch projection for orders 7-16 (split across files for
// parallel builds).
#include "slice_impl.h"

namespace dpm {
hipError_t launch_slice_groups_u16(int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    return launch_groups_nd<uint16_t>(nd, a, items, lds, st);
}
}  // namespace dpm
