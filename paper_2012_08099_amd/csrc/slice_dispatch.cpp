// Dispatch of the projection kernel instantiations by dtype, group and width.
#include "kernels.h"

namespace dpm {
#define DECL(name) \
    hipError_t name(bool fast, int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st);
DECL(launch_slice_g0_u16_n4)
DECL(launch_slice_g0_u16_n8)
DECL(launch_slice_g0_u8_n4)
DECL(launch_slice_g0_u8_n8)
#undef DECL
hipError_t launch_slice_g12_u16(int g, bool fast, int nd, const SliceArgs &a, int items, size_t lds,
                                hipStream_t st);
hipError_t launch_slice_g12_u8(int g, bool fast, int nd, const SliceArgs &a, int items, size_t lds,
                               hipStream_t st);

hipError_t launch_slice(int elem, int nls, bool fast, int g, int nd, const SliceArgs &a, int items,
                        size_t lds, hipStream_t st) {
    if (nls != 4 && nls != 8) return hipErrorInvalidValue;
    if (g == 0) {
        if (elem == 2) return nls == 4 ? launch_slice_g0_u16_n4(fast, nd, a, items, lds, st)
                                       : launch_slice_g0_u16_n8(fast, nd, a, items, lds, st);
        return nls == 4 ? launch_slice_g0_u8_n4(fast, nd, a, items, lds, st)
                        : launch_slice_g0_u8_n8(fast, nd, a, items, lds, st);
    }
    if (nls != 8) return hipErrorInvalidValue;  // orders >= 7 always use 256-bit partials
    return elem == 2 ? launch_slice_g12_u16(g, fast, nd, a, items, lds, st)
                     : launch_slice_g12_u8(g, fast, nd, a, items, lds, st);
}
}  // namespace dpm
