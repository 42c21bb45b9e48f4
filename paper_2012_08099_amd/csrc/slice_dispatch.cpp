// Dispatch of the projection kernel instantiations by dtype, group and load path.
#include "kernels.h"

namespace dpm {
#define DECL(name) hipError_t name(int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st);
DECL(launch_slice_g0_u16_fast)
DECL(launch_slice_g0_u16_chain)
DECL(launch_slice_g0_u16_gen)
DECL(launch_slice_g0_u8_fast)
DECL(launch_slice_g0_u8_gen)
#undef DECL
hipError_t launch_slice_g12_u16(int g, bool fast, int nd, const SliceArgs &a, int items, size_t lds,
                                hipStream_t st);
hipError_t launch_slice_g12_u8(int g, bool fast, int nd, const SliceArgs &a, int items, size_t lds,
                               hipStream_t st);
hipError_t launch_slice_groups_u16(int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st);
hipError_t launch_slice_groups_u8(int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st);

hipError_t launch_slice_block_u8(int rowbytes, int nd, const BlockArgs &a, int items, size_t lds, hipStream_t st);
hipError_t launch_slice_block_u16(int nd, const BlockArgs &a, int items, size_t lds, hipStream_t st);

hipError_t launch_slice_block(int elem, int rowbytes, int nd, const BlockArgs &a, int items, size_t lds,
                              hipStream_t st) {
    if (elem == 2) return rowbytes == 4 ? launch_slice_block_u16(nd, a, items, lds, st) : hipErrorInvalidValue;
    return launch_slice_block_u8(rowbytes, nd, a, items, lds, st);
}

hipError_t launch_slice_groups(int elem, int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    return elem == 2 ? launch_slice_groups_u16(nd, a, items, lds, st) : launch_slice_groups_u8(nd, a, items, lds, st);
}

hipError_t launch_slice(int elem, bool fast, bool chain, int g, int nd, const SliceArgs &a, int items, size_t lds,
                        hipStream_t st) {
    if (g == 0) {
        if (elem == 2 && chain) return launch_slice_g0_u16_chain(nd, a, items, lds, st);
        if (elem == 2) return fast ? launch_slice_g0_u16_fast(nd, a, items, lds, st)
                                   : launch_slice_g0_u16_gen(nd, a, items, lds, st);
        return fast ? launch_slice_g0_u8_fast(nd, a, items, lds, st) : launch_slice_g0_u8_gen(nd, a, items, lds, st);
    }
    return elem == 2 ? launch_slice_g12_u16(g, fast, nd, a, items, lds, st)
                     : launch_slice_g12_u8(g, fast, nd, a, items, lds, st);
}
}  // namespace dpm
