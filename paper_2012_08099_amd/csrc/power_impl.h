// Device helpers of the matrix-core power sums shared by the power-sum kernels and the
// fused batched kernel: tile description, limb split of 16 row values, reassembly of
// limb-pair sums into exact multiword power sums, and the y-weighted tile epilogue.
#pragma once
#include "dpm_common.h"
#include "kernels.h"
#include "lane_sum.h"
#include "mw.h"

namespace dpm {

struct TileInfo {
    int slot;
    int nitems;         // items of the tile (<= 16)
    int32_t len;        // values per row (multiple of 64)
    int64_t stride;     // int32 values between consecutive items' rows
    const int32_t *base;  // row of the tile's first item, this slot
    int32_t ybase;      // y of item i of the tile: (ybase + i) / ydiv
    int32_t ydiv;
    int32_t ks0, ks1;   // steps of 64 values of a covered by the tile
};

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

// Epilogue shared by both paths, for T threads (tid: the thread's index among them).  Thread t holds
// R[j] = r(item t % 16, slot, k) for k = d + t / 16 + (T / 16) j; the 16 lanes of one k
// are one aligned lane group.  For every q <= K - k the group sums y^q R exactly and
// its last lane stores T(tile, k, q).
template <int T>
constexpr int epi_nj() { return (KMAX + 1 + T / 16 - 1) / (T / 16); }

template <int T, int NLS, int NLR, int NJ>
__device__ __forceinline__ void yweight_store(const PowerArgs &a, const TileInfo &ti, int tile, int d,
                                              const mw::Int<NLS> (&R)[NJ], int tid) {
    const int ei = tid & 15, K = a.K;
    const uint32_t y = (uint32_t)((ti.ybase + ei) / ti.ydiv);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int k = d + (tid >> 4) + (T / 16) * j;
        if (k > K) break;  // uniform over the lane group
        mw::Int<NLR> v = mw::resize<NLR, NLS>(R[j]);  // r >= 0
        uint32_t *dst = a.part + ((size_t)tile * (K + 1) + k) * (K + 1) * NLR;
        for (int q = 0; q <= K - k; ++q) {
            mw::Int<NLR> s = v;
            row16_sum_last(s);
            if (ei == 15)
#pragma unroll
                for (int l = 0; l < NLR; ++l) dst[(size_t)q * NLR + l] = s.w[l];
            mw::mul_u32(v, y);
        }
    }
}

// The same T(tile, k, q) with the (k, q) pairs spread evenly over the T / 16 lane groups
// (one k per group leaves the group of k = d with K - d + 1 pairs and the last with one).
// stage_r puts every thread's r(item, k) into rt[k - d][item] (LDS, NLS words each); after
// a barrier, group g takes pairs [g P / G, (g + 1) P / G) in (k, q) order,
// P = (K - d + 1)(K - d + 2) / 2: it reads r(item, k), raises it by y^q for the group's
// first q, then sums and stores as above.
template <int T, int NLS, int NJ>
__device__ __forceinline__ void stage_r(int d, int K, const mw::Int<NLS> (&R)[NJ], uint32_t *rt, int tid) {
    const int ei = tid & 15;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int k = d + (tid >> 4) + (T / 16) * j;
        if (k > K) break;
#pragma unroll
        for (int l = 0; l < NLS; ++l) rt[((k - d) * 16 + ei) * NLS + l] = R[j].w[l];
    }
}

template <int T, int NLS, int NLR>
__device__ __forceinline__ void yweight_store_even(const PowerArgs &a, const TileInfo &ti, int tile, int d,
                                                   const uint32_t *rt, int tid) {
    constexpr int NG = T / 16;
    const int ei = tid & 15, g = tid >> 4, K = a.K;
    const uint32_t y = (uint32_t)((ti.ybase + ei) / ti.ydiv);
    const int nk = K - d + 1;
    const int P = nk * (nk + 1) / 2;
    const int p0 = g * P / NG, p1 = (g + 1) * P / NG;
    if (p0 >= p1) return;  // uniform over the lane group
    int k = d, before = 0;  // pairs of the k below the current one
    while (before + (K - k + 1) <= p0) {
        before += K - k + 1;
        ++k;
    }
    int q = p0 - before;
    for (int pi = p0; pi < p1; ++k, q = 0) {
        mw::Int<NLS> r;
#pragma unroll
        for (int l = 0; l < NLS; ++l) r.w[l] = rt[((k - d) * 16 + ei) * NLS + l];
        mw::Int<NLR> v = mw::resize<NLR, NLS>(r);  // r >= 0
        for (int e = 0; e < q; ++e) mw::mul_u32(v, y);
        uint32_t *dst = a.part + ((size_t)tile * (K + 1) + k) * (K + 1) * NLR;
        const int qe = K - k < q + (p1 - pi) - 1 ? K - k : q + (p1 - pi) - 1;
        for (; q <= qe; ++q, ++pi) {
            mw::Int<NLR> s = v;
            row16_sum_last(s);
            if (ei == 15)
#pragma unroll
                for (int l = 0; l < NLR; ++l) dst[(size_t)q * NLR + l] = s.w[l];
            mw::mul_u32(v, y);
        }
    }
}

constexpr int PW_MW = 4;   // waves of the split-contraction kernel
constexpr int PW_PF = 3;   // K-steps per wave whose loads are in flight together
constexpr int PW_NTP = 4;  // 16-column tiles per wave and pass (4 P-limbs x 4 tiles x 4 = 64 VGPRs)
constexpr int PW_SHORT = 512;  // rows up to this many values take the one-wave kernel
constexpr int PW_CTILES = 4 * PW_NTP;  // column tiles of the split-columns kernel

typedef int v4i __attribute__((ext_vector_type(4)));

// A_c = 7-bit limb c of 16 row values, four values per int32 (one byte each), the
// byte order of the matrix cores' A operand.
__device__ __forceinline__ void split_limbs(const uint32_t (&v)[16], v4i (&A)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            uint32_t w = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) w |= ((v[4 * e + i] >> (7 * c)) & 0x7fu) << (8 * i);
            A[c][e] = (int)w;
        }
}

// R_k(item) += sum_u 2^(7u) sum_c 2^(7c) C_c[item][col(k, u)] over the columns of tiles
// [tb, tb + n), whose limb-pair sums sit in ctab[c][tile - tb] ([c][tile][item*16+col]).
// Thread tid (index among the T threads) holds (item, k) = (tid & 15, d + (tid >> 4) + (T / 16) j).
template <int T, int NLS, int NJ, int NCT>
__device__ __forceinline__ void reassemble(const PowerArgs &a, int d, int tb, int n, const int32_t (*ctab)[NCT][256],
                                           mw::Int<NLS> (&R)[NJ], int tid) {
    const int ei = tid & 15, K = a.K;
    const int colp0 = tb * 16, colp1 = (tb + n) * 16;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int k = d + (tid >> 4) + (T / 16) * j;
        if (k > K) break;
        const int cs0 = a.pow.colstart[k], cs1 = a.pow.colstart[k + 1];
        const int lo = cs0 > colp0 ? cs0 : colp0, hi = cs1 < colp1 ? cs1 : colp1;
        for (int col = lo; col < hi; ++col) {
            const int tp = (col >> 4) - tb, cc = col & 15;
            uint64_t vsum = 0;  // < 2^27 * 2^22: exact
#pragma unroll
            for (int c = 0; c < 4; ++c) vsum += (uint64_t)(uint32_t)ctab[c][tp][ei * 16 + cc] << (7 * c);
            if (!vsum) continue;
            const int sh = 7 * (col - cs0);
            add_shifted(R[j], (uint32_t)vsum, sh);
            add_shifted(R[j], (uint32_t)(vsum >> 32), sh + 32);
        }
    }
}

}  // namespace dpm
