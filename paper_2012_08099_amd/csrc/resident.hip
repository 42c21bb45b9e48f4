// Kernels of the served loop's resident 2D moments: collapse a volume's power-sum tiles
// into one tile per image side, and re-stride them for a query of lower order.  The
// values are exact multiword integers (nlr 32-bit limbs), summed exactly.
#include <hip/hip_runtime.h>

#include "mw.h"
#include "resident.h"

namespace dpm {

namespace {

template <int NLR>
__global__ void __launch_bounds__(64) collapse_kernel(CollapseArgs a) {
    const int s = blockIdx.x, kq = blockIdx.y, lane = threadIdx.x;
    const int K1 = a.K + 1;
    int32_t t0 = 0, nt = 0;
    if (a.roi) {
        const RoiDesc &rd = *a.roi;
        if (rd.slot_len[s]) {
            int rank = 0;
            for (int i = 0; i < s; ++i) rank += rd.slot_len[i] != 0;
            nt = (int32_t)((rd.M + 15) / 16);
            t0 = rd.tile0 + rank * nt;
        }
    } else {
        t0 = a.tile0[s];
        nt = a.tile0[s + 1] - a.tile0[s];
    }
    mw::Int<NLR> acc;
    mw::set_zero(acc);
    for (int t = lane; t < nt; t += 64) {
        const uint32_t *src = a.part + ((size_t)(t0 + t) * K1 * K1 + kq) * NLR;
        mw::Int<NLR> v;
#pragma unroll
        for (int l = 0; l < NLR; ++l) v.w[l] = src[l];
        mw::add(acc, v);
    }
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) {
        mw::Int<NLR> o;
#pragma unroll
        for (int l = 0; l < NLR; ++l) o.w[l] = (uint32_t)__shfl_xor((int)acc.w[l], sh, 64);
        mw::add(acc, o);
    }
    if (lane < NLR) a.out[((size_t)s * K1 * K1 + kq) * NLR + lane] = acc.w[lane];
}

__global__ void __launch_bounds__(256) restride_kernel(const uint32_t *in, int Ki, uint32_t *out, int Ko, int nlr) {
    const int Ki1 = Ki + 1, Ko1 = Ko + 1;
    const int n = 2 * Ko1 * Ko1 * Ko1 * nlr;
    for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
        const int l = v % nlr, q = (v / nlr) % Ko1, k = (v / nlr / Ko1) % Ko1, s = v / nlr / Ko1 / Ko1;
        out[v] = in[(((size_t)s * Ki1 + k) * Ki1 + q) * nlr + l];
    }
}

}  // namespace

hipError_t launch_collapse(const CollapseArgs &a, hipStream_t st) {
    const dim3 grid(2 * (a.K + 1), (a.K + 1) * (a.K + 1));
    if (a.nlr == 4) hipLaunchKernelGGL(collapse_kernel<4>, grid, dim3(64), 0, st, a);
    else if (a.nlr == 8) hipLaunchKernelGGL(collapse_kernel<8>, grid, dim3(64), 0, st, a);
    else if (a.nlr == 12) hipLaunchKernelGGL(collapse_kernel<12>, grid, dim3(64), 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_restride(const uint32_t *in, int Ki, uint32_t *out, int Ko, int nlr, hipStream_t st) {
    if (Ko > Ki) return hipErrorInvalidValue;
    const int n = 2 * (Ko + 1) * (Ko + 1) * (Ko + 1) * nlr;
    hipLaunchKernelGGL(restride_kernel, dim3((n + 255) / 256), dim3(256), 0, st, in, Ki, out, Ko, nlr);
    return hipGetLastError();
}

}  // namespace dpm
