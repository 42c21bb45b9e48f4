// Fused batched kernel: projection and power sums of a block of y-slices of one ROI in
// one workgroup, with the image rows kept in LDS.
//
// Workgroup = (ROI, block of BK_YB = 16 consecutive y-slices), BK_WAVES = 4 waves.
//  1. Projection (Section 3.1, eq. 4): in rounds, wave w forms the image rows I_d(., y) of
//     a group of spw consecutive slices (spw = 1, 2 or 4 per ROI: small slices are
//     grouped so that the wave's sub-rows all have work) in its own LDS scratch (the row
//     projection of the single-volume kernel, one wave per group), then copies every row side, split at
//     the image's true origin (Section 5's offset for beta < 0), into the block store:
//     row y - y0 of slot s = 2 d + side, values a = 0 .. bk_plen(s) - 1, zero outside the
//     side's extent.  The waves run their rounds independently (wave-local ordering).
//  2. Power sums: every non-empty slot's 16 rows are one matrix-core tile, as in the
//     power-sum kernel: r(y, s, k) = sum_a a^k row(y, s, a) from 7-bit limbs of the row
//     values (A operand, read from LDS) and of a^k (B operand, the power table), the
//     limb-pair sums reassembled exactly; then T(tile, k, q) = sum_y y^q r(y, s, k).
//     Each slot goes to the least loaded wave, longest first.
// The tile partials land where the power-sum kernel puts them (tile = tile0 of the ROI +
// rank of the slot x blocks of the ROI + block), so recombination is unchanged; the rows
// never leave LDS.
#pragma once
#include "power_impl.h"
#include "slice_impl.h"

namespace dpm {

// Workgroups per CU the register budget is cut for (the block store and scratch of the
// batches this kernel takes leave room for about three), and 16-column tiles of powers
// per pass of the contraction.
constexpr int BK_MIN_BLOCKS = 3;
constexpr int BK_NTP = 2;

// Orders this wave's LDS accesses before and after (all lanes of the wave).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// A operand limbs of 16 row values held as uint16: 3 limbs of 7 bits (values < 2^16),
// byte i of A[c][e] = limb c of value 4 e + i; A[3] = 0.
__device__ __forceinline__ void split_limbs16(const uint32_t (&p)[8], v4i (&A)[4]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const uint32_t m = c < 2 ? 0x7f7f7f7fu : 0x03030303u;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // p[2e] = v[4e] | v[4e+1] << 16, p[2e+1] = v[4e+2] | v[4e+3] << 16; after the
            // shift the limbs sit in bytes 0 and 2 of each: gather them in value order
            const uint32_t lo = p[2 * e] >> (7 * c), hi = p[2 * e + 1] >> (7 * c);
            A[c][e] = (int)(__builtin_amdgcn_perm(hi, lo, 0x06040200u) & m);
        }
    }
    A[3] = v4i{0, 0, 0, 0};
}

template <typename VT, int ND, typename RV>
__global__ void __launch_bounds__(BK_WAVES * 64, BK_MIN_BLOCKS) slice_block_kernel(BlockArgs a) {
    extern __shared__ uint4 lds_raw[];
    __shared__ ItemGeom ig;
    __shared__ int32_t plen[MAXSEG], soff[MAXSEG], rstr[MAXSEG], tot_s;  // block store: values, first value, stride
    constexpr int G = VecOf<VT>::G;
    constexpr int NS = 2 * ND;
    const BatchItem it = a.b.items[blockIdx.x];
    const RoiDesc &rd = a.b.rois[it.roi];
    // the wave index as a scalar: what derives from it (scratch base, slice groups) stays
    // in scalar registers
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    {
        // (its loads overlap those of the descriptor)
        const int32_t *src = reinterpret_cast<const int32_t *>(a.b.geom + it.roi);
        int32_t *dst = reinterpret_cast<int32_t *>(&ig);
        for (int i = tid; i < (int)(sizeof(ItemGeom) / 4); i += BK_WAVES * 64) dst[i] = src[i];
    }
    if (rd.elem != (int)sizeof(VT) || rd.rowbytes != (int)sizeof(RV)) return;  // uniform
    __syncthreads();
    if (tid == 0) {
        // block store layout (the same arithmetic as bk_lds_bytes on the host)
        int32_t t = 0;
        for (int s = 0; s < NS; ++s) {
            plen[s] = bk_plen(ig, s);
            rstr[s] = bk_rstride(plen[s], (int)sizeof(RV));
            soff[s] = t;
            t += BK_YB * rstr[s];
        }
        tot_s = t;
    }
    __syncthreads();
    const int32_t tot = tot_s;
    RV *store = reinterpret_cast<RV *>(lds_raw);
    const int32_t sbytes = (tot * (int32_t)sizeof(RV) + 15) / 16 * 16;
    const int spw = rd.spw;
    if (spw < 1 || spw > 4) return;  // uniform; the planner takes 1, 2 or 4 (the row-side copy assumes <= 4)
    const int32_t SW = bk_slice_dwords(ig);  // one slice's accumulators
    uint32_t *const scr = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(lds_raw) + sbytes) +
                          wave * bk_scratch_dwords(ig, spw);

    const int64_t y0 = (int64_t)it.y * BK_YB;
    const int ny = (int)(rd.M - y0 < BK_YB ? rd.M - y0 : BK_YB);
    const VT *vol = reinterpret_cast<const VT *>(a.b.packed + rd.offset);
    const int64_t pitch_z = rd.L * rd.M;

    // 1. projection: wave w takes groups of spw consecutive slices, g = w, w + 4, ...
    for (int j0 = wave * spw; j0 < ny; j0 += BK_WAVES * spw) {
        const int nsl = ny - j0 < spw ? ny - j0 : spw;
        for (int i = lane; i < nsl * SW / 4; i += 64) reinterpret_cast<uint4 *>(scr)[i] = make_uint4(0u, 0u, 0u, 0u);
        wave_lds_sync();
        project_rows<VT, 0, ND, false, 1, true, 1>(vol + (y0 + j0) * rd.L, rd.L, pitch_z, 0, rd.N, rd.R, rd.CT, scr, ig,
                                                nsl, rd.L, SW, a.b.packed_end);
        wave_lds_sync();
        // row sides into the store, four values per lane, read together, one store.  The
        // chunks of both sides of all nsl slices of a direction are numbered together, so
        // that short rows still keep every lane busy: chunk c is slice c / cps, then side 0
        // or 1 (q0 chunks of side 0 first); nsl <= 4.
        StaticFor<0, ND>::run([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int pp = dir_pp(i, G);
            const int32_t q0 = plen[2 * i] >> 2, cps = q0 + (plen[2 * i + 1] >> 2);  // lens: multiples of 16
            const SegView v0 = seg_view(scr, ig, i, 0, i == 1, pp), v1 = seg_view(scr, ig, i, 1, i == 1, pp);
            const int32_t so0 = soff[2 * i], so1 = soff[2 * i + 1], rs0 = rstr[2 * i], rs1 = rstr[2 * i + 1];
            for (int32_t c = lane; c < cps * nsl; c += 64) {
                const int32_t sl = (c >= cps) + (c >= 2 * cps) + (c >= 3 * cps);
                const int32_t r = c - sl * cps;
                const bool s1 = r >= q0;
                const int32_t x0 = 4 * (s1 ? r - q0 : r);
                SegView v = s1 ? v1 : v0;
                v.row += sl * SW;
                RV *dst = store + (s1 ? so1 : so0) + (j0 + sl) * (s1 ? rs1 : rs0) + x0;
                uint32_t e[4];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    e[k] = (x0 + k >= v.alo && x0 + k <= v.ahi) ? seg_value(v, x0 + k) : 0u;
                if constexpr (sizeof(RV) == 2)
                    *reinterpret_cast<uint2 *>(dst) = make_uint2(e[0] | e[1] << 16, e[2] | e[3] << 16);
                else
                    *reinterpret_cast<uint4 *>(dst) = make_uint4(e[0], e[1], e[2], e[3]);
            }
        });
        wave_lds_sync();  // the next group clears this scratch
    }
    __syncthreads();  // every slice's rows are in the store

    // 2. power sums, one slot per wave at a time; the wave's scratch becomes its table
    const PowerArgs &pa = a.pw;
    const int nt = pa.pow.nt;
    const int ipt = (int)((rd.M + 15) / 16);
    int32_t(*ctab)[1][256] = reinterpret_cast<int32_t(*)[1][256]>(scr);
    const int il = lane & 15, g4 = lane >> 4;
    const bool iv = il < ny;
    const uint4 *bt = pa.pow.b + lane;
    constexpr int NJ = epi_nj<64>();
    // slots to waves, longest first onto the least loaded wave (the same arithmetic in every
    // wave): cost = (k, q) pairs of the y-weighting + 2 per K-step of the contraction
    int load[BK_WAVES] = {};
    int rank = 0;
    for (int s = 0; s < NS; ++s) {
        if (plen[s] == 0) continue;
        const int d = s >> 1;
        const int32_t len = plen[s];
        const int nks = (len + 63) / 64;
        int wl = 0;
#pragma unroll
        for (int w = 1; w < BK_WAVES; ++w)
            if (load[w] < load[wl]) wl = w;
        load[wl] += (pa.K + 1 - d) * (pa.K + 2 - d) / 2 + 2 * nks;
        const int tile = rd.tile0 + rank * ipt + it.y;
        ++rank;
        if (wl != wave) continue;
        const RV *rowp = store + soff[s] + il * rstr[s] + g4 * 16;
        mw::Int<4> R[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) mw::set_zero(R[jj]);
        for (int t0 = 0; t0 < nt; t0 += BK_NTP) {
            v4i acc[4][BK_NTP];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int tp = 0; tp < BK_NTP; ++tp) acc[c][tp] = v4i{0, 0, 0, 0};
            for (int ks = 0; ks < nks; ++ks) {
                const bool ok = iv && ks * 64 + g4 * 16 < len;  // 16 values, all inside the row
                v4i A[4];
                if constexpr (sizeof(RV) == 2) {
                    uint32_t p[8];
                    const uint4 *q = reinterpret_cast<const uint4 *>(rowp + ks * 64);
                    const uint4 q0 = ok ? q[0] : make_uint4(0u, 0u, 0u, 0u), q1 = ok ? q[1] : make_uint4(0u, 0u, 0u, 0u);
                    p[0] = q0.x; p[1] = q0.y; p[2] = q0.z; p[3] = q0.w;
                    p[4] = q1.x; p[5] = q1.y; p[6] = q1.z; p[7] = q1.w;
                    split_limbs16(p, A);
                } else {
                    uint32_t v[16];
                    const uint4 *q = reinterpret_cast<const uint4 *>(rowp + ks * 64);
#pragma unroll
                    for (int i4 = 0; i4 < 4; ++i4) {
                        const uint4 w = ok ? q[i4] : make_uint4(0u, 0u, 0u, 0u);
                        v[4 * i4] = w.x; v[4 * i4 + 1] = w.y; v[4 * i4 + 2] = w.z; v[4 * i4 + 3] = w.w;
                    }
                    split_limbs(v, A);
                }
                constexpr int NL = sizeof(RV) == 2 ? 3 : 4;
#pragma unroll
                for (int tp = 0; tp < BK_NTP; ++tp) {
                    if (t0 + tp < nt) {
                        const uint4 bq = bt[((size_t)ks * nt + t0 + tp) * 64];
                        v4i B;
                        __builtin_memcpy(&B, &bq, 16);
#pragma unroll
                        for (int c = 0; c < NL; ++c)
                            acc[c][tp] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[c], B, acc[c][tp], 0, 0, 0);
                    }
                }
            }
            // one column tile at a time through the wave's table
#pragma unroll
            for (int tp = 0; tp < BK_NTP; ++tp) {
                if (t0 + tp >= nt) break;
                wave_lds_sync();  // the previous reassembly has read the table
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int e = 0; e < 4; ++e) ctab[c][0][(g4 * 4 + e) * 16 + il] = acc[c][tp][e];
                wave_lds_sync();
                reassemble<64, 4, NJ, 1>(pa, d, t0 + tp, 1, ctab, R, lane);
            }
        }
        TileInfo ti{};
        ti.slot = s;
        ti.nitems = ny;
        ti.ybase = (int32_t)y0;
        ti.ydiv = 1;
        yweight_store<64, 4, 4, NJ>(pa, ti, tile, d, R, lane);  // 4-limb tile partials only
    }
}

template <typename VT, typename RV, int ND>
hipError_t launch_block_one(const BlockArgs &a, int items, size_t lds, hipStream_t st) {
    auto k = slice_block_kernel<VT, ND, RV>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(items), dim3(BK_WAVES * 64), lds, st, a);
    return hipGetLastError();
}

template <typename VT, typename RV>
hipError_t launch_block_nd(int nd, const BlockArgs &a, int items, size_t lds, hipStream_t st) {
    switch (nd) {
        case 1: return launch_block_one<VT, RV, 1>(a, items, lds, st);
        case 2: return launch_block_one<VT, RV, 2>(a, items, lds, st);
        case 3: return launch_block_one<VT, RV, 3>(a, items, lds, st);
        case 4: return launch_block_one<VT, RV, 4>(a, items, lds, st);
        case 5: return launch_block_one<VT, RV, 5>(a, items, lds, st);
        case 6: return launch_block_one<VT, RV, 6>(a, items, lds, st);
        case 7: return launch_block_one<VT, RV, 7>(a, items, lds, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dpm
