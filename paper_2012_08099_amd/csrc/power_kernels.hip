// Power sums of the image rows written by the projection kernel, weighted in y:
//
//     r(item, slot, k)   = sum_a a^k row(item, slot, a),        d <= k <= K,  slot = 2d + side
//     T(tile, k, q)      = sum_{items i of the tile} y_i^q r(i, slot, k),   q <= K - k
//
// exact, in multiword integers.  r is the x-z part of the 2D moments (eq. 1) of one
// image row about the image's true origin (Section 3.2; the negative side enters with
// the sign (-1)^k later); T is a tile's share of the y part, so the 2D moment of
// image d is the sum of T over the tiles of its two slots.
//
// A tile is 16 items (consecutive image rows) of one slot, one workgroup.
// Matrix-core path: with a the contraction index, the 16 rows are the A operand and the
// limbs of a^k (precomputed table) the B operand of v_mfma_i32_16x16x64_i8.  Row values
// (< 2^28) and powers are split into 7-bit limbs, so every product and the int32
// accumulation over a are exact; the four waves split the contraction, and the limb-pair
// sums are reassembled into the exact r with shifts.
// VALU path (row values >= 2^28): multiword products and an exact lane reduction.
#include <cstdlib>

#include "dpm_common.h"
#include "kernels.h"
#include "mw.h"
#include "power_impl.h"

namespace dpm {

constexpr int PW_WAVES = 4;

__device__ bool decode_tile(const PowerArgs &a, int tile, TileInfo &ti) {
    if (!a.rois) {
        if (tile >= a.rl.tile0[NSLOT]) return false;
        int s = 0;
        while (tile >= a.rl.tile0[s + 1]) ++s;  // empty slots own no tiles
        const int local = tile - a.rl.tile0[s], nck = a.rl.nck[s];
        const int blk = local / nck, ch = local - blk * nck;
        const int item0 = blk * 16;
        ti.slot = s;
        ti.nitems = a.nitems - item0 < 16 ? a.nitems - item0 : 16;
        ti.len = a.rl.slot_len[s];
        ti.stride = a.rl.row_stride;
        ti.base = a.rows + (int64_t)item0 * a.rl.row_stride + a.rl.slot_off[s];
        ti.ybase = item0;
        ti.ydiv = a.zsplits;
        ti.ks0 = ch * a.rl.kchunk;
        ti.ks1 = ti.ks0 + a.rl.kchunk < ti.len / 64 ? ti.ks0 + a.rl.kchunk : ti.len / 64;
        return true;
    }
    const RoiDesc &rd = a.rois[a.tile_roi[tile]];
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
            ti.ybase = item0;
            ti.ydiv = 1;
            ti.ks0 = 0;
            ti.ks1 = ti.len / 64;
            return true;
        }
        cnt += ipt;
    }
    return false;
}

// One workgroup per tile (16 items x one slot).  Matrix-core kernels, three ways to
// spread a tile over its waves:
//  * split contraction (MW = 4): the waves split the K-steps of 64 coordinates (wave w
//    takes steps w, w + 4, ...); their int32 limb-pair sums meet in LDS through atomics;
//    up to PW_NTP column tiles of powers per pass;
//  * one wave (MW = 1), for short rows: no LDS clearing or atomics, one column tile at a
//    time through LDS;
//  * split columns (power_mfma_cols_kernel), for more columns than one pass holds: wave w
//    owns column tiles 4w .. 4w+3 for the whole contraction, so up to 16 column tiles take
//    one pass, with plain LDS stores and one reassembly; the waves take turns loading and
//    limb-splitting the rows of a K-step and share the limbs through LDS.
// Loads of PW_PF K-steps are in flight together; then every thread reassembles one
// (item, k) sum.
// Loads of PF K-steps: the 16 rows' values (A) and the limbs of a^k (B) of column tiles
// t0 .. t0 + PW_NTP - 1; zero past ks_end or past the rows.
template <int PF>
struct StepBuf {
    uint4 rq[PF][4], bq[PF][PW_NTP];
};

template <int PF>
__device__ __forceinline__ void load_steps(StepBuf<PF> &b, const int32_t *rp, bool iv, const uint4 *bt, int nt,
                                           int t0, int ks0, int ks_end, int stride) {
#pragma unroll
    for (int f = 0; f < PF; ++f) {
        const int ks = ks0 + f * stride;
        const bool ok = ks < ks_end;
        const uint4 *p = reinterpret_cast<const uint4 *>(rp + ks * 64);
#pragma unroll
        for (int i = 0; i < 4; ++i) b.rq[f][i] = (ok && iv) ? p[i] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int tp = 0; tp < PW_NTP; ++tp)
            b.bq[f][tp] = (ok && t0 + tp < nt) ? bt[((size_t)ks * nt + t0 + tp) * 64] : make_uint4(0u, 0u, 0u, 0u);
    }
}

// acc[c][tp] += A_c(ks) x B(ks, t0 + tp) for the PF K-steps of b: A_c = 7-bit limb c of
// the rows' values.
template <int PF>
__device__ __forceinline__ void mma_steps(const StepBuf<PF> &b, int nt, int t0, int ks0, int ks_end, int stride,
                                          v4i (&acc)[4][PW_NTP]) {
#pragma unroll
    for (int f = 0; f < PF; ++f) {
        if (ks0 + f * stride >= ks_end) break;
        const uint32_t v[16] = {b.rq[f][0].x, b.rq[f][0].y, b.rq[f][0].z, b.rq[f][0].w,
                                b.rq[f][1].x, b.rq[f][1].y, b.rq[f][1].z, b.rq[f][1].w,
                                b.rq[f][2].x, b.rq[f][2].y, b.rq[f][2].z, b.rq[f][2].w,
                                b.rq[f][3].x, b.rq[f][3].y, b.rq[f][3].z, b.rq[f][3].w};
        v4i A[4];
        split_limbs(v, A);
#pragma unroll
        for (int tp = 0; tp < PW_NTP; ++tp) {
            if (t0 + tp < nt) {
                v4i B;
                __builtin_memcpy(&B, &b.bq[f][tp], 16);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[c][tp] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[c], B, acc[c][tp], 0, 0, 0);
            }
        }
    }
}

// acc[c][tp] += sum over K-steps ks = ks_first, ks_first + stride, ... < ks_end of
// A_c(ks) x B(ks, t0 + tp), PW_PF K-steps per batch of loads.
__device__ __forceinline__ void mfma_steps(const int32_t *rp, bool iv, const uint4 *bt, int nt, int t0,
                                           int ks_first, int ks_end, int stride, v4i (&acc)[4][PW_NTP]) {
    for (int ks0 = ks_first; ks0 < ks_end; ks0 += PW_PF * stride) {
        StepBuf<PW_PF> b;
        load_steps<PW_PF>(b, rp, iv, bt, nt, t0, ks0, ks_end, stride);
        mma_steps<PW_PF>(b, nt, t0, ks0, ks_end, stride, acc);
    }
}

template <int NLS, int NLR, int MW>
__global__ void __launch_bounds__(MW * 64) power_mfma_kernel(PowerArgs a) {
    constexpr int T = MW * 64;
    constexpr int NCT = MW == 1 ? 1 : PW_NTP;  // column tiles held in LDS at once
    __shared__ int32_t ctab[4][NCT][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    TileInfo ti;
    if (!decode_tile(a, blockIdx.x, ti)) return;  // uniform over the workgroup
    const int d = ti.slot >> 1;
    const int il = lane & 15;
    const bool iv = il < ti.nitems;
    const int32_t *rp = ti.base + (iv ? (int64_t)il * ti.stride : 0) + (lane >> 4) * 16;
    const int nt = a.pow.nt;
    const uint4 *bt = a.pow.b + lane;
    constexpr int NJ = epi_nj<T>();
    mw::Int<NLS> R[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) mw::set_zero(R[j]);

    for (int t0 = 0; t0 < nt; t0 += PW_NTP) {
        if (MW > 1) {
            for (int i = tid; i < 4 * NCT * 256; i += T) (&ctab[0][0][0])[i] = 0;
            __syncthreads();
        }
        v4i acc[4][PW_NTP];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int tp = 0; tp < PW_NTP; ++tp) acc[c][tp] = v4i{0, 0, 0, 0};
        mfma_steps(rp, iv, bt, nt, t0, ti.ks0 + wave, ti.ks1, MW, acc);
        if (MW > 1) {
            // partial limb-pair sums of the waves -> ctab[c][tile][item][col]
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int tp = 0; tp < PW_NTP; ++tp)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (acc[c][tp][e]) atomicAdd(&ctab[c][tp][((lane >> 4) * 4 + e) * 16 + (lane & 15)], acc[c][tp][e]);
            __syncthreads();
            reassemble<T, NLS, NJ, NCT>(a, d, t0, PW_NTP, ctab, R, threadIdx.x);
            __syncthreads();
        } else {
            // one wave holds the whole sums: one column tile at a time through LDS
#pragma unroll
            for (int tp = 0; tp < PW_NTP; ++tp) {
                if (t0 + tp >= nt) break;
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int e = 0; e < 4; ++e) ctab[c][0][((lane >> 4) * 4 + e) * 16 + (lane & 15)] = acc[c][tp][e];
                __syncthreads();
                reassemble<T, NLS, NJ, NCT>(a, d, t0 + tp, 1, ctab, R, threadIdx.x);
                __syncthreads();
            }
        }
    }
    if constexpr (MW > 1) {
        // the last reassembly is behind a barrier: its table takes the sums r(item, k)
        static_assert((KMAX + 1) * 16 * NLS <= 4 * NCT * 256, "r table exceeds the LDS table");
        uint32_t *rt = reinterpret_cast<uint32_t *>(&ctab[0][0][0]);
        stage_r<T, NLS, NJ>(d, a.K, R, rt, tid);
        __syncthreads();
        yweight_store_even<T, NLS, NLR>(a, ti, blockIdx.x, d, rt, tid);
    } else {
        yweight_store<T, NLS, NLR, NJ>(a, ti, blockIdx.x, d, R, threadIdx.x);
    }
}

template <int NLS, int NLR>
__global__ void __launch_bounds__(PW_MW * 64) power_mfma_cols_kernel(PowerArgs a) {
    constexpr int T = PW_MW * 64;
    // LDS: during the contraction, the limb-split rows of PW_MW K-steps (two buffers,
    // [buffer][step][limb][lane]); afterwards the limb-pair sums of every column tile
    __shared__ int32_t lds[4 * PW_CTILES * 256];
    static_assert(2 * PW_MW * 4 * 64 * 4 <= 4 * PW_CTILES * 256, "limb buffers exceed the LDS table");
    int32_t(*ctab)[PW_CTILES][256] = reinterpret_cast<int32_t(*)[PW_CTILES][256]>(lds);
    uint4 *abuf = reinterpret_cast<uint4 *>(lds);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    TileInfo ti;
    if (!decode_tile(a, blockIdx.x, ti)) return;  // uniform over the workgroup
    const int d = ti.slot >> 1;
    const int il = lane & 15;
    const bool iv = il < ti.nitems;
    const int32_t *rp = ti.base + (iv ? (int64_t)il * ti.stride : 0) + (lane >> 4) * 16;
    const int nt = a.pow.nt;  // <= PW_CTILES (checked at launch)
    const uint4 *bt = a.pow.b + lane;
    const int t0 = wave * PW_NTP;
    v4i acc[4][PW_NTP];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int tp = 0; tp < PW_NTP; ++tp) acc[c][tp] = v4i{0, 0, 0, 0};
    // Every wave needs the limbs of the same rows at every K-step: wave w loads and splits
    // step ks0 + w of each group of PW_MW steps and shares it through LDS, then every wave
    // multiplies the group's steps into its own column tiles.  The loop bounds are uniform
    // over the workgroup, so every wave reaches every barrier.
    int buf = 0;
    for (int ks0 = ti.ks0; ks0 < ti.ks1; ks0 += PW_MW, buf ^= 1) {
        const int ks = ks0 + wave;
        const bool oka = iv && ks < ti.ks1;
        const uint4 *p = reinterpret_cast<const uint4 *>(rp + ks * 64);
        uint4 rq[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) rq[i] = oka ? p[i] : make_uint4(0u, 0u, 0u, 0u);
        uint4 bq[PW_MW][PW_NTP];
#pragma unroll
        for (int f = 0; f < PW_MW; ++f)
#pragma unroll
            for (int tp = 0; tp < PW_NTP; ++tp)
                bq[f][tp] = (ks0 + f < ti.ks1 && t0 + tp < nt) ? bt[((size_t)(ks0 + f) * nt + t0 + tp) * 64]
                                                               : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t v[16] = {rq[0].x, rq[0].y, rq[0].z, rq[0].w, rq[1].x, rq[1].y, rq[1].z, rq[1].w,
                                rq[2].x, rq[2].y, rq[2].z, rq[2].w, rq[3].x, rq[3].y, rq[3].z, rq[3].w};
        v4i A[4];
        split_limbs(v, A);
        uint4 *aw = abuf + (size_t)((buf * PW_MW + wave) * 4) * 64 + lane;
#pragma unroll
        for (int c = 0; c < 4; ++c) __builtin_memcpy(&aw[c * 64], &A[c], 16);
        // one barrier per group: a buffer is written again only two groups later, after
        // every wave has passed the next group's barrier and so finished reading it
        __syncthreads();
#pragma unroll
        for (int f = 0; f < PW_MW; ++f) {
            if (ks0 + f >= ti.ks1) break;
            const uint4 *ar = abuf + (size_t)((buf * PW_MW + f) * 4) * 64 + lane;
            v4i Af[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) __builtin_memcpy(&Af[c], &ar[c * 64], 16);
#pragma unroll
            for (int tp = 0; tp < PW_NTP; ++tp) {
                if (t0 + tp < nt) {
                    v4i B;
                    __builtin_memcpy(&B, &bq[f][tp], 16);
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        acc[c][tp] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Af[c], B, acc[c][tp], 0, 0, 0);
                }
            }
        }
    }
    __syncthreads();  // the limb buffers share LDS with the sums table
    // every wave stores its own column tiles (tiles >= nt are never read)
#pragma unroll
    for (int tp = 0; tp < PW_NTP; ++tp)
        if (t0 + tp < nt)
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int e = 0; e < 4; ++e) ctab[c][t0 + tp][((lane >> 4) * 4 + e) * 16 + (lane & 15)] = acc[c][tp][e];
    __syncthreads();
    constexpr int NJ = epi_nj<T>();
    mw::Int<NLS> R[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) mw::set_zero(R[j]);
    reassemble<T, NLS, NJ, PW_CTILES>(a, d, 0, PW_CTILES, ctab, R, threadIdx.x);
    __syncthreads();  // every thread has read the table: it takes the sums r(item, k)
    static_assert((KMAX + 1) * 16 * NLS <= 4 * PW_CTILES * 256, "r table exceeds the LDS table");
    uint32_t *rt = reinterpret_cast<uint32_t *>(lds);
    stage_r<T, NLS, NJ>(d, a.K, R, rt, tid);
    __syncthreads();
    yweight_store_even<T, NLS, NLR>(a, ti, blockIdx.x, d, rt, tid);
}

template <int NLS, int NLR>
__global__ void __launch_bounds__(PW_WAVES * 64) power_valu_kernel(PowerArgs a) {
    __shared__ uint32_t rbuf[16][KMAX + 1][NLS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    TileInfo ti;
    if (!decode_tile(a, blockIdx.x, ti)) return;  // uniform over the workgroup
    const int K = a.K;
    const int d = ti.slot >> 1;
    for (int i = tid; i < 16 * (KMAX + 1) * NLS; i += PW_WAVES * 64) (&rbuf[0][0][0])[i] = 0u;
    __syncthreads();
    for (int il = wave; il < ti.nitems; il += PW_WAVES) {
        const int32_t *rp = ti.base + (int64_t)il * ti.stride;
        mw::Int<NLS> acc[KMAX + 1];
#pragma unroll
        for (int k = 0; k <= KMAX; ++k) mw::set_zero(acc[k]);
        for (int32_t aa = ti.ks0 * 64 + lane; aa < ti.ks1 * 64; aa += 64) {
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
                    for (int l = 0; l < NLS; ++l) rbuf[il][k][l] = v.w[l];
            }
        }
    }
    __syncthreads();
    constexpr int T = PW_WAVES * 64;
    constexpr int NJ = epi_nj<T>();
    mw::Int<NLS> R[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int k = d + (tid >> 4) + (T / 16) * j;
#pragma unroll
        for (int l = 0; l < NLS; ++l) R[j].w[l] = k <= K ? rbuf[tid & 15][k][l] : 0u;
    }
    yweight_store<T, NLS, NLR, NJ>(a, ti, blockIdx.x, d, R, threadIdx.x);
}

// DPM_PW_NO_COLS=1 keeps multi-pass column sets on the split-contraction kernel.
static bool power_cols_off() {
    const char *e = std::getenv("DPM_PW_NO_COLS");
    return e && atoi(e);
}

template <int NLS, int NLR>
static hipError_t power_go(const PowerArgs &a, hipStream_t st) {
    if (a.ntiles == 0) return hipSuccess;
    if (a.pow.b && a.max_len <= PW_SHORT)
        hipLaunchKernelGGL((power_mfma_kernel<NLS, NLR, 1>), dim3(a.ntiles), dim3(64), 0, st, a);
    else if (a.pow.b && a.pow.nt > PW_NTP && a.pow.nt <= PW_CTILES && !power_cols_off())
        hipLaunchKernelGGL((power_mfma_cols_kernel<NLS, NLR>), dim3(a.ntiles), dim3(PW_MW * 64), 0, st, a);
    else if (a.pow.b)
        hipLaunchKernelGGL((power_mfma_kernel<NLS, NLR, PW_MW>), dim3(a.ntiles), dim3(PW_MW * 64), 0, st, a);
    else hipLaunchKernelGGL((power_valu_kernel<NLS, NLR>), dim3(a.ntiles), dim3(PW_WAVES * 64), 0, st, a);
    return hipGetLastError();
}

// The power table of PowTab built on the device (same bytes as the host build): thread
// (ks, tile, lane) writes the 16 limb bytes of column 16 tile + lane % 16 for
// a = 64 ks + 16 (lane / 16) + i, i = 0..15; columns past colstart[K+1] are zero.
__global__ void __launch_bounds__(256) powtab_build_kernel(uint4 *tab, int32_t nt, int32_t ncells, int32_t K,
                                                          PowTab shape) {
    const int cell = blockIdx.x * 256 + threadIdx.x;
    if (cell >= ncells) return;
    const int lane = cell % 64, tile = (cell / 64) % nt, ks = cell / (64 * nt);
    const int col = tile * 16 + lane % 16, kq = lane / 16;
    int k = -1;
    for (int j = 0; j <= K; ++j)
        if (col >= shape.colstart[j] && col < shape.colstart[j + 1]) k = j;
    uint32_t bytes[4] = {0u, 0u, 0u, 0u};
    if (k >= 0) {
        const int bit = 7 * (col - shape.colstart[k]);
        for (int i = 0; i < 16; ++i) {
            const uint32_t a = (uint32_t)(64 * ks + 16 * kq + i);
            mw::Int<8> v;
            mw::set_u64(v, 1);
            for (int j = 0; j < k; ++j) mw::mul_u32(v, a);
            const int w0 = bit >> 5, sh = bit & 31;
            uint32_t lo = 0u, hi = 0u;
#pragma unroll
            for (int l = 0; l < 8; ++l) {
                if (l == w0) lo = v.w[l] >> sh;
                if (l == w0 + 1 && sh) hi = v.w[l] << (32 - sh);
            }
            bytes[i / 4] |= ((lo | hi) & 0x7fu) << (8 * (i % 4));
        }
    }
    tab[cell] = make_uint4(bytes[0], bytes[1], bytes[2], bytes[3]);
}

hipError_t launch_powtab_build(uint4 *tab, const PowTab &shape, int K, hipStream_t st) {
    const int ncells = shape.amax / 64 * shape.nt * 64;
    if (ncells <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(powtab_build_kernel, dim3((ncells + 255) / 256), dim3(256), 0, st, tab, shape.nt, ncells, K,
                       shape);
    return hipGetLastError();
}

hipError_t launch_power(int nls, int nlr, const PowerArgs &a, hipStream_t st) {
    if (nls == 4 && nlr == 4) return power_go<4, 4>(a, st);
    if (nls == 4 && nlr == 8) return power_go<4, 8>(a, st);
    if (nls == 4 && nlr == 12) return power_go<4, 12>(a, st);
    if (nls == 8 && nlr == 8) return power_go<8, 8>(a, st);
    if (nls == 8 && nlr == 12) return power_go<8, 12>(a, st);
    return hipErrorInvalidValue;
}

}  // namespace dpm
