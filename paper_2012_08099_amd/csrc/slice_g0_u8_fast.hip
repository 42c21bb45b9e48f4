// Instantiations of the projection kernel (split across files for parallel builds).
#include "slice_impl.h"

namespace dpm {

hipError_t launch_slice_g0_u8_fast(int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    if (a.waves == 8) return launch_nd<uint8_t, 0, true, false, 8>(nd, a, items, lds, st);
    return launch_nd<uint8_t, 0, true>(nd, a, items, lds, st);
}
}  // namespace dpm
