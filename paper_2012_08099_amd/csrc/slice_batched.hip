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

__global__ void __launch_bounds__(64) batched_prep_kernel(BatchSliceArgs a, int nd) {
    const int roi = blockIdx.x;
    const RoiDesc &rd = a.rois[roi];
    if (threadIdx.x == 0) {
        ItemGeom g;
        item_geometry(0, nd, lane_voxels(rd.elem), rd.L, rd.N, 0, rd.N, g);
        a.geom[roi] = g;
    }
    for (int32_t y = threadIdx.x; y < rd.nitems; y += 64) a.items[rd.item_pos + y] = BatchItem{roi, y};
    for (int64_t j = threadIdx.x; j < rd.ntiles; j += 64) a.tile_roi[rd.tile0 + j] = roi;
}

hipError_t launch_batched_prep(int nd, const BatchSliceArgs &a, int nrois, hipStream_t st) {
    if (nrois <= 0) return hipSuccess;
    hipLaunchKernelGGL(batched_prep_kernel, dim3(nrois), dim3(64), 0, st, a, nd);
    return hipGetLastError();
}

hipError_t launch_slice_batched(int elem, int g, int nd, const BatchSliceArgs &a, int items, size_t lds,
                                hipStream_t st) {
    if (g != 0) return hipErrorInvalidValue;  // batched ROIs: orders <= 6
    if (elem == 2) return launch_b_nd<uint16_t>(nd, a, items, lds, st);
    return launch_b_nd<uint8_t>(nd, a, items, lds, st);
}
}  // namespace dpm
