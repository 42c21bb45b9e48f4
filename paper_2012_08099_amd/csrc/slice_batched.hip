// Instantiations of the projection kernel (split across files for parallel builds).
#include "slice_impl.h"

namespace dpm {

template <typename VT>
static hipError_t launch_b_nd(int nd, const BatchSliceArgs &a, int items, size_t lds, hipStream_t st) {
    switch (nd) {
        case 1: return launch_b_one<VT, 0, 1>(a, items, lds, st);
        case 2: return launch_b_one<VT, 0, 2>(a, items, lds, st);
        case 3: return launch_b_one<VT, 0, 3>(a, items, lds, st);
        case 4: return launch_b_one<VT, 0, 4>(a, items, lds, st);
        case 5: return launch_b_one<VT, 0, 5>(a, items, lds, st);
        case 6: return launch_b_one<VT, 0, 6>(a, items, lds, st);
        case 7: return launch_b_one<VT, 0, 7>(a, items, lds, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_slice_batched(int elem, int g, int nd, const BatchSliceArgs &a, int items, size_t lds,
                                hipStream_t st) {
    if (g != 0) return hipErrorInvalidValue;  // batched ROIs: orders <= 6
    if (elem == 2) return launch_b_nd<uint16_t>(nd, a, items, lds, st);
    return launch_b_nd<uint8_t>(nd, a, items, lds, st);
}
}  // namespace dpm
