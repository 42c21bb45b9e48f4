// Power sums of the image rows written by the projection kernel:
//
//     part[item][slot][k] = sum_a a^k row(item, slot, a),   d <= k <= K,  slot = 2d + side,
//
// exact, in multiword integers.  These are the x-z parts of the 2D moments (eq. 1) of
// each image row about the image's true origin (Section 3.2; the negative side enters
// the y reduction with the sign (-1)^k).
//
// Matrix-core path: a wave takes 16 items of one slot.  With a the contraction index,
// the 16 rows (items) are the A operand and the limbs of a^k (precomputed table) the B
// operand of v_mfma_i32_16x16x64_i8.  Row values (< 2^28) and powers are split into
// 7-bit limbs, so every product and the int32 accumulation over a are exact; the 4 x L
// limb-pair sums are reassembled into the exact sum with shifts.
// VALU path (row values >= 2^28): multiword products and an exact lane reduction.
#include "dpm_common.h"
#include "kernels.h"
#include "mw.h"

namespace dpm {

constexpr int PW_WAVES = 4;

struct TileInfo {
    int slot;
    int nitems;         // items of the tile (<= 16)
    int32_t len;        // values per row (multiple of 64)
    int64_t stride;     // int32 values between consecutive items' rows
    const int32_t *base;  // row of the tile's first item, this slot
    int64_t pidx0;      // part index of the tile's first item
};

__device__ bool decode_tile(const PowerArgs &a, int tile, TileInfo &ti) {
    if (!a.rois) {
        const int ipt = (a.nitems + 15) / 16;
        int cnt = 0;
        for (int s = 2 * a.d_first; s <= 2 * a.d_last + 1; ++s) {
            if (a.rl.slot_len[s] == 0) continue;
            if (tile < cnt + ipt) {
                const int item0 = (tile - cnt) * 16;
                ti.slot = s;
                ti.nitems = a.nitems - item0 < 16 ? a.nitems - item0 : 16;
                ti.len = a.rl.slot_len[s];
                ti.stride = a.rl.row_stride;
                ti.base = a.rows + (int64_t)item0 * a.rl.row_stride + a.rl.slot_off[s];
                ti.pidx0 = item0;
                return true;
            }
            cnt += ipt;
        }
        return false;
    }
    int lo = 0, hi = a.nrois - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (a.rois[mid].tile0 <= tile) lo = mid;
        else hi = mid - 1;
    }
    const RoiDesc &rd = a.rois[lo];
    const int ipt = (int)((rd.M + 15) / 16);
    int local = tile - rd.tile0, cnt = 0;
    for (int s = 0; s < 14 && s <= 2 * a.K + 1; ++s) {
        if (rd.slot_len[s] == 0) continue;
        if (local < cnt + ipt) {
            const int item0 = (local - cnt) * 16;
            ti.slot = s;
            ti.nitems = (int)rd.M - item0 < 16 ? (int)rd.M - item0 : 16;
            ti.len = rd.slot_len[s];
            ti.stride = rd.row_stride;
            ti.base = a.rows + rd.row_base + (int64_t)item0 * rd.row_stride + rd.slot_off[s];
            ti.pidx0 = rd.item0 + item0;
            return true;
        }
        cnt += ipt;
    }
    return false;
}

// acc += v * 2^shift (v < 2^32)
template <int N>
__device__ __forceinline__ void add_shifted(mw::Int<N> &acc, uint32_t v, int shift) {
    const int wi = shift >> 5, bi = shift & 31;
    const uint64_t x = (uint64_t)v << bi;
    uint64_t c = 0;
#pragma unroll
    for (int l = 0; l < N; ++l) {
        uint64_t add = 0;
        if (l == wi) add = (uint32_t)x;
        else if (l == wi + 1) add = (uint32_t)(x >> 32);
        const uint64_t t = (uint64_t)acc.w[l] + add + c;
        acc.w[l] = (uint32_t)t;
        c = t >> 32;
    }
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One workgroup per tile (16 items x one slot).  The four waves split the K-steps of
// 64 coordinates; their int32 limb-pair sums meet in LDS; then every thread
// reassembles one (item, k) sum.
constexpr int PW_NTP = 4;  // 16-column tiles per pass (4 P-limbs x 4 tiles x 4 = 64 VGPRs)

template <int NLS>
__global__ void __launch_bounds__(PW_WAVES * 64) power_mfma_kernel(PowerArgs a) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    __shared__ int32_t ctab[4][PW_NTP][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    TileInfo ti;
    if (!decode_tile(a, blockIdx.x, ti)) return;  // uniform over the workgroup
    const int K = a.K;
    const int d = ti.slot >> 1;
    const int il = lane & 15;
    const bool iv = il < ti.nitems;
    const int32_t *rp = ti.base + (iv ? (int64_t)il * ti.stride : 0) + (lane >> 4) * 16;
    const int nks = ti.len / 64;
    const int nt = a.pow.nt;
    const uint4 *bt = a.pow.b + lane;

    // reassembly work of this thread: (item, k) = (tid & 15, d + (tid >> 4) + 16 j)
    const int ei = tid & 15;
    constexpr int NJ = (KMAX + 16) / 16;
    mw::Int<NLS> R[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) mw::set_zero(R[j]);

    auto load_rows = [&](int ks, uint4 (&q)[4]) {
        if (iv && ks < nks) {
            const uint4 *p = reinterpret_cast<const uint4 *>(rp + ks * 64);
#pragma unroll
            for (int i = 0; i < 4; ++i) q[i] = p[i];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) q[i] = make_uint4(0u, 0u, 0u, 0u);
        }
    };

    for (int t0 = 0; t0 < nt; t0 += PW_NTP) {
        for (int i = tid; i < 4 * PW_NTP * 256; i += PW_WAVES * 64) (&ctab[0][0][0])[i] = 0;
        __syncthreads();
        v4i acc[4][PW_NTP];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int tp = 0; tp < PW_NTP; ++tp) acc[c][tp] = v4i{0, 0, 0, 0};
        uint4 cur[4], nxt[4];
        load_rows(wave, cur);
        for (int ks = wave; ks < nks; ks += PW_WAVES) {
            load_rows(ks + PW_WAVES, nxt);  // next K-step of this wave in flight
            uint4 bq[PW_NTP];
#pragma unroll
            for (int tp = 0; tp < PW_NTP; ++tp)
                if (t0 + tp < nt) bq[tp] = bt[((size_t)ks * nt + t0 + tp) * 64];
            const uint32_t v[16] = {cur[0].x, cur[0].y, cur[0].z, cur[0].w, cur[1].x, cur[1].y, cur[1].z, cur[1].w,
                                    cur[2].x, cur[2].y, cur[2].z, cur[2].w, cur[3].x, cur[3].y, cur[3].z, cur[3].w};
            v4i A[4];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint32_t w = 0;
#pragma unroll
                    for (int i = 0; i < 4; ++i) w |= ((v[4 * e + i] >> (7 * c)) & 0x7fu) << (8 * i);
                    A[c][e] = (int)w;
                }
#pragma unroll
            for (int tp = 0; tp < PW_NTP; ++tp) {
                if (t0 + tp < nt) {
                    v4i B;
                    __builtin_memcpy(&B, &bq[tp], 16);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c][tp] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[c], B, acc[c][tp], 0, 0, 0);
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) cur[i] = nxt[i];
        }
        // partial limb-pair sums of the four waves -> ctab[c][tile][item][col]
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int tp = 0; tp < PW_NTP; ++tp)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (acc[c][tp][e]) atomicAdd(&ctab[c][tp][((lane >> 4) * 4 + e) * 16 + (lane & 15)], acc[c][tp][e]);
        __syncthreads();
        // R_k(item) += sum_u 2^(7u) sum_c 2^(7c) C_c[item][col(k, u)]
        const int colp0 = t0 * 16, colp1 = (t0 + PW_NTP) * 16;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int k = d + (tid >> 4) + 16 * j;
            if (k > K) break;
            const int cs0 = a.pow.colstart[k], cs1 = a.pow.colstart[k + 1];
            const int lo = cs0 > colp0 ? cs0 : colp0, hi = cs1 < colp1 ? cs1 : colp1;
            for (int col = lo; col < hi; ++col) {
                const int tp = (col >> 4) - t0, cc = col & 15;
                uint64_t vsum = 0;  // < 2^27 * 2^22: exact
#pragma unroll
                for (int c = 0; c < 4; ++c) vsum += (uint64_t)(uint32_t)ctab[c][tp][ei * 16 + cc] << (7 * c);
                if (!vsum) continue;
                const int sh = 7 * (col - cs0);
                add_shifted(R[j], (uint32_t)vsum, sh);
                add_shifted(R[j], (uint32_t)(vsum >> 32), sh + 32);
            }
        }
        __syncthreads();
    }
    if (ei >= ti.nitems) return;
    const int nslot = 2 * (K + 1);
    uint32_t *dst = a.part + (((size_t)(ti.pidx0 + ei) * nslot + ti.slot) * (K + 1)) * NLS;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int k = d + (tid >> 4) + 16 * j;
        if (k > K) break;
#pragma unroll
        for (int l = 0; l < NLS; ++l) dst[(size_t)k * NLS + l] = R[j].w[l];
    }
}

template <int NLS>
__global__ void __launch_bounds__(PW_WAVES * 64) power_valu_kernel(PowerArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tile = blockIdx.x * PW_WAVES + wave;
    TileInfo ti;
    if (tile >= a.ntiles || !decode_tile(a, tile, ti)) return;
    const int K = a.K;
    const int d = ti.slot >> 1;
    const int nslot = 2 * (K + 1);
    for (int il = 0; il < ti.nitems; ++il) {
        const int32_t *rp = ti.base + (int64_t)il * ti.stride;
        mw::Int<NLS> acc[KMAX + 1];
#pragma unroll
        for (int k = 0; k <= KMAX; ++k) mw::set_zero(acc[k]);
        for (int32_t aa = lane; aa < ti.len; aa += 64) {
            const uint32_t P = (uint32_t)rp[aa];
            if (P == 0u) continue;
            mw::Int<NLS> t;
            mw::set_u64(t, P);
#pragma unroll
            for (int k = 0; k <= KMAX; ++k) {
                if (k <= K) {
                    if (k >= d) mw::add(acc[k], t);
                    if (k < K) mw::mul_u32(t, (uint32_t)aa);
                }
            }
        }
        uint32_t *dst = a.part + (((size_t)(ti.pidx0 + il) * nslot + ti.slot) * (K + 1)) * NLS;
#pragma unroll
        for (int k = 0; k <= KMAX; ++k) {
            if (k >= d && k <= K) {
                mw::Int<NLS> &v = acc[k];
#pragma unroll
                for (int m = 1; m < 64; m <<= 1) {
                    mw::Int<NLS> o2;
#pragma unroll
                    for (int l = 0; l < NLS; ++l) o2.w[l] = (uint32_t)__shfl_xor((int)v.w[l], m, 64);
                    mw::add(v, o2);
                }
                if (lane == 0)
#pragma unroll
                    for (int l = 0; l < NLS; ++l) dst[(size_t)k * NLS + l] = v.w[l];
            }
        }
    }
}

template <int NLS>
static hipError_t power_go(const PowerArgs &a, hipStream_t st) {
    if (a.ntiles == 0) return hipSuccess;
    if (a.pow.b) {
        hipLaunchKernelGGL((power_mfma_kernel<NLS>), dim3(a.ntiles), dim3(PW_WAVES * 64), 0, st, a);
    } else {
        const int blocks = (a.ntiles + PW_WAVES - 1) / PW_WAVES;
        hipLaunchKernelGGL((power_valu_kernel<NLS>), dim3(blocks), dim3(PW_WAVES * 64), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_power(int nls, const PowerArgs &a, hipStream_t st) {
    if (nls == 4) return power_go<4>(a, st);
    if (nls == 8) return power_go<8>(a, st);
    return hipErrorInvalidValue;
}

}  // namespace dpm
