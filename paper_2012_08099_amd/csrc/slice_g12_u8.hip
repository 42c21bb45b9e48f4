// Instantiations of the projection kernel (split across files for parallel builds).
#include "slice_impl.h"

namespace dpm {

hipError_t launch_slice_g12_u8(int g, bool fast, int nd, const SliceArgs &a, int items, size_t lds,
                               hipStream_t st) {
    if (g == 1) return fast ? launch_nd<uint8_t, 7, true>(nd, a, items, lds, st)
                            : launch_nd<uint8_t, 7, false>(nd, a, items, lds, st);
    return fast ? launch_nd<uint8_t, 12, true>(nd, a, items, lds, st)
                : launch_nd<uint8_t, 12, false>(nd, a, items, lds, st);
}
}  // namespace dpm
