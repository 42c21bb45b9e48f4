// Moments from supplied projection images (the tomography use of the method noted in
// Section 3.2: measured projections replace step 1).  Each image row y of direction d is
// split at the image's origin into the two row slots the power sums read: slot 2d holds
// a = o - i (columns left of the origin, a >= 1), slot 2d+1 holds a = i - o.
#include "dpm_common.h"
#include "kernels.h"

namespace dpm {

__global__ void __launch_bounds__(256) images_to_rows_kernel(ImgArgs a) {
    const int y = blockIdx.x;
    int32_t *row = a.rows + (int64_t)y * a.rl.row_stride;
    for (int d = 0; d < a.nd; ++d) {
        const int32_t *img = a.images + a.off[d] + (int64_t)y * a.width[d];
        const int32_t o = a.origin[d], w = a.width[d];
        for (int side = 0; side < 2; ++side) {
            const int s = 2 * d + side;
            const int32_t len = a.rl.slot_len[s];
            int32_t *dst = row + a.rl.slot_off[s];
            for (int32_t t = threadIdx.x; t < len; t += 256) {
                const int64_t i = side ? (int64_t)o + t : (int64_t)o - t;
                const bool in = side ? (i < w) : (t >= 1 && i >= 0);
                int32_t v = in ? img[i] : 0;
                if (v < 0 || (int64_t)v > a.bound) {
                    atomicOr(a.bad, 1u);
                    v = 0;
                }
                dst[t] = v;
            }
        }
    }
}

hipError_t launch_images_to_rows(const ImgArgs &a, hipStream_t st) {
    if (a.M <= 0) return hipSuccess;
    hipLaunchKernelGGL(images_to_rows_kernel, dim3(a.M), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace dpm
