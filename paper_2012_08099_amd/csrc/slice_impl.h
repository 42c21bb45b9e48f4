// Projection kernel: one workgroup per work item (one y-slice of one volume, rows
// [zs, ze)).  It forms the image rows I_d(., y) of every direction d of its group in
// one coalesced pass over the voxels (Section 3.1, eq. 4; the projection loop of
// Section 5), then takes exact power sums of each row about the image's true origin:
//
//     r_{d,k}(y) = sum_i (i - o_d)^k I_d(i, y),   d <= k <= K,
//
// which is the x-z part of the 2D moments of eq. (1).  The y part and the
// recombination run in later kernels.  o_d = |beta| (N-1) for beta < 0 places the
// moment origin of a negative-index image at column N-1 (the offset correction of
// Section 5, applied before the sums by splitting each row at o_d).
//
// Mapping (gfx950, wave64): a sub-row of R lanes covers one volume row, lane r owning
// the G = 8 consecutive voxels x0 = 64*G*ct + G*r .. x0+7 (one 16/8-byte load).  Each
// sub-row walks a contiguous range of row chunks (z).  Per voxel and direction there
// is exactly one integer add into a register window; windows are flushed to LDS row
// accumulators every T_d rows with ds_add at compile-time offsets (conflict-free by
// the padding of dir_pp).  The (0,1) direction needs a full-row sum per z: v_dot2 /
// v_dot4 then a DPP reduction over 8-lane groups.  No global atomics.
#pragma once
#include "dpm_common.h"
#include "mw.h"
#include "kernels.h"

namespace dpm {

// ------------------------------------------------------------ compile-time helpers
template <int B, int E>
struct StaticFor {
    template <typename F>
    __device__ __forceinline__ static void run(F &&f) {
        if constexpr (B < E) {
            f(std::integral_constant<int, B>{});
            StaticFor<B + 1, E>::run(f);
        }
    }
};

template <typename VT>
struct VecOf;
template <>
struct VecOf<uint16_t> {
    using type = uint4;  // 8 voxels
};
template <>
struct VecOf<uint8_t> {
    using type = uint2;  // 8 voxels
};

template <typename VT>
__device__ __forceinline__ uint32_t voxel(const typename VecOf<VT>::type &v, int j);
template <>
__device__ __forceinline__ uint32_t voxel<uint16_t>(const uint4 &v, int j) {
    const uint32_t w = j < 2 ? v.x : j < 4 ? v.y : j < 6 ? v.z : v.w;
    return (j & 1) ? (w >> 16) : (w & 0xffffu);
}
template <>
__device__ __forceinline__ uint32_t voxel<uint8_t>(const uint2 &v, int j) {
    const uint32_t w = j < 4 ? v.x : v.y;
    return (w >> (8 * (j & 3))) & 0xffu;
}

// sum of the 8 voxels of a lane
__device__ __forceinline__ uint32_t lane_sum(const uint4 &v) {
    typedef unsigned short us2 __attribute__((ext_vector_type(2)));
    const us2 one = {1, 1};
    uint32_t s = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v.x), one, 0u, false);
    s = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v.y), one, s, false);
    s = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v.z), one, s, false);
    s = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v.w), one, s, false);
    return s;
}
__device__ __forceinline__ uint32_t lane_sum(const uint2 &v) {
    uint32_t s = __builtin_amdgcn_udot4(v.x, 0x01010101u, 0u, false);
    return __builtin_amdgcn_udot4(v.y, 0x01010101u, s, false);
}

// Sum over each aligned group of 8 lanes; every lane of the group gets the total.
__device__ __forceinline__ uint32_t group8_sum(uint32_t s) {
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x141, 0xF, 0xF, false);  // row_half_mirror
    return s;
}

// Is (tt, j) the first touch of its window slot within a block (t outer, j inner)?
template <int D>
__device__ constexpr bool first_touch(int tt, int j) {
    const int A = dir_alpha(D), Bt = dir_beta(D), SH = dir_shift(D);
    const int s = A * j + Bt * tt + SH;
    for (int t2 = 0; t2 <= tt; ++t2)
        for (int j2 = 0; j2 < G; ++j2) {
            if (t2 == tt && j2 >= j) return true;
            if (A * j2 + Bt * t2 + SH == s) return false;
        }
    return true;
}

// Does any voxel of a block land in window slot s?  (alpha j + beta t hits every slot
// only when alpha or |beta| is 1; e.g. (3,2) never reaches slot 1.)
template <int D>
__device__ constexpr bool slot_used(int s) {
    const int A = dir_alpha(D), Bt = dir_beta(D), SH = dir_shift(D);
    for (int t2 = 0; t2 < dir_td(D); ++t2)
        for (int j2 = 0; j2 < G; ++j2)
            if (A * j2 + Bt * t2 + SH == s) return true;
    return false;
}

// ------------------------------------------------------------ per-item work
template <typename VT, bool FAST>
__device__ __forceinline__ typename VecOf<VT>::type load_lane(const VT *row, int64_t x0, int64_t L,
                                                              bool in) {
    using Vec = typename VecOf<VT>::type;
    Vec v{};
    if constexpr (FAST) {
        v = *reinterpret_cast<const Vec *>(row + x0);
    } else {
        if (in) {
            uint32_t w[sizeof(Vec) / 4] = {};
#pragma unroll
            for (int j = 0; j < G; ++j) {
                uint32_t e = (x0 + j < L) ? (uint32_t)row[x0 + j] : 0u;
                w[(j * sizeof(VT)) / 4] |= e << (8 * ((j * sizeof(VT)) & 3));
            }
            __builtin_memcpy(&v, w, sizeof(Vec));
        }
    }
    return v;
}

template <int D0, int ND>
struct GroupTraits {
    static constexpr int g = D0 == 0 ? 0 : D0 == 7 ? 1 : 2;
    static constexpr int T = group_rows(g);
    static constexpr bool has_xy = (D0 == 0);
    static constexpr bool has_yz = (D0 == 0 && ND >= 2);
    static constexpr int NK = KMAX + 1 - D0;  // accumulator slots for k = D0..KMAX
};

template <typename VT, int D0, int ND, int NLS, bool FAST>
__device__ void slice_item(const VT *__restrict__ vol, int64_t L, int64_t N, int64_t pitch_y,
                           int64_t pitch_z, int64_t y, int64_t zs, int64_t ze, int K, int R,
                           int CT, int jobbins, uint32_t *__restrict__ part_out,
                           int32_t *__restrict__ img, const int64_t *img_off, const int64_t *img_w,
                           uint32_t *lds, ItemGeom &ig) {
    using Tr = GroupTraits<D0, ND>;
    using Vec = typename VecOf<VT>::type;
    constexpr int T = Tr::T;
    constexpr int NW = SLICE_WAVES;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    if (tid == 0) item_geometry(Tr::g, ND, L, N, zs, ze, ig);
    __syncthreads();
    for (int i = tid; i < ig.lds_dwords; i += NW * 64) lds[i] = 0u;
    __syncthreads();

    // ---------------- step 1: projection rows in LDS
    {
        const int SR = 64 / R;
        const int sr = lane / R, r = lane % R;
        const int gsr = wave * SR + sr, NSR = NW * SR;
        const int64_t nch = ig.n_chunks;
        const int64_t U = (int64_t)CT * nch;
        const int64_t u_begin = (int64_t)gsr * U / NSR, u_end = (int64_t)(gsr + 1) * U / NSR;
        const VT *slice = vol + y * pitch_y;

        for (int64_t u = u_begin; u < u_end; ++u) {
            const int64_t ct = u / nch, ch = u % nch;
            const int64_t x0 = ct * 64 * G + (int64_t)r * G;
            const bool valid = x0 < L;
            const int64_t zc0 = zs + ch * T;

            // load the chunk's rows (all loads issued before use)
            Vec dat[T];
            StaticFor<0, T>::run([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                const int64_t z = zc0 + t;
                const bool in = FAST ? true : (valid && z < ze);
                dat[t] = load_lane<VT, FAST>(slice + (FAST ? z : (z < ze ? z : ze - 1)) * pitch_z, x0,
                                            L, in);
            });

            uint32_t xy[G];
            uint32_t yzs[T];
            StaticFor<0, T>::run([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                const Vec &v = dat[t];
                if constexpr (Tr::has_xy) {
                    StaticFor<0, G>::run([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        if constexpr (t == 0) xy[j] = voxel<VT>(v, j);
                        else xy[j] += voxel<VT>(v, j);
                    });
                }
                if constexpr (Tr::has_yz) yzs[t] = group8_sum(lane_sum(v));
            });

            // sheared directions: register windows, flushed every T_d rows
            StaticFor<0, ND>::run([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int d = D0 + i;
                if constexpr (d >= 2) {
                    constexpr int A = dir_alpha(d), Bt = dir_beta(d), TD = dir_td(d);
                    constexpr int S = dir_slots(d), SH = dir_shift(d), PP = dir_pp(d);
                    // lane base in bins relative to the LDS row origin (32-bit: bins < 2^31)
                    const int32_t rel0 = (int32_t)(A * x0 + Bt * zc0 + ig.dir[i].o - SH - ig.dir[i].lo);
                    const int32_t doff = ig.dir[i].lds_off;
                    uint32_t w[S];
                    StaticFor<0, T>::run([&](auto tc) {
                        constexpr int t = decltype(tc)::value;
                        constexpr int tt = t % TD;
                        const Vec &v = dat[t];
                        StaticFor<0, G>::run([&](auto jc) {
                            constexpr int j = decltype(jc)::value;
                            constexpr int s = A * j + Bt * tt + SH;
                            if constexpr (first_touch<d>(tt, j)) w[s] = voxel<VT>(v, j);
                            else w[s] += voxel<VT>(v, j);
                        });
                        if constexpr (tt == TD - 1) {
                            if (FAST || valid) {
                                const uint32_t lb = (uint32_t)(rel0 + Bt * (t - (TD - 1)));
                                uint32_t *base = lds + doff + (lb + lb / PP);
                                StaticFor<0, S>::run([&](auto sc) {
                                    constexpr int s = decltype(sc)::value;
                                    if constexpr (slot_used<d>(s)) atomicAdd(base + (s + s / PP), w[s]);
                                });
                            }
                        }
                    });
                }
            });

            if constexpr (Tr::has_xy) {
                if (FAST || valid) {
                    const uint32_t x0u = (uint32_t)x0;
                    uint32_t *base = lds + ig.dir[0].lds_off + (x0u + x0u / 8);
                    StaticFor<0, G>::run([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        atomicAdd(base + j, xy[j]);
                    });
                }
            }
            if constexpr (Tr::has_yz) {
                if ((lane & 7) == 0) {
                    uint32_t *base = lds + ig.yz_off + (lane >> 3) * ig.yz_stride + (uint32_t)(zc0 - zs);
                    StaticFor<0, T>::run([&](auto tc) {
                        constexpr int t = decltype(tc)::value;
                        atomicAdd(base + t, yzs[t]);
                    });
                }
            }
        }
    }
    __syncthreads();

    // value of image i at bin b (b inside the item's real range)
    auto pix = [&](int i, int d, int64_t b) -> uint32_t {
        if (d == 1) {
            const uint32_t *p = lds + ig.yz_off + (b - zs);
            uint32_t s = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c) s += p[c * ig.yz_stride];
            return s;
        }
        const int64_t u = b - ig.dir[i].lo;
        return lds[ig.dir[i].lds_off + u + u / dir_pp(d)];
    };

    // ---------------- optional: write the image rows (full-row items only)
    if (img) {
        for (int i = 0; i < ND; ++i) {
            const int64_t lo = ig.dir[i].rb_lo, hi = ig.dir[i].rb_hi;
            int32_t *row = img + img_off[i] + y * img_w[i];
            for (int64_t b = lo + tid; b <= hi; b += NW * 64) row[b] = (int32_t)pix(i, D0 + i, b);
        }
    }

    // ---------------- step 2: exact power sums of every row about its true origin
    uint32_t *jobres = lds + ig.lds_dwords;
    constexpr int NK = Tr::NK;
    const int njobs = count_jobs(ig, ND, jobbins);
    for (int j = wave; j < njobs; j += NW) {
        int ji = 0, jside = 0;
        int64_t jb0 = 0, jb1 = -1;
        {
            int cnt = 0;
            for (int i = 0; i < ND; ++i)
                for (int side = 0; side < 2; ++side) {
                    int64_t b0, b1;
                    if (!seg_range(ig.dir[i], side, b0, b1)) continue;
                    const int nj = (int)((b1 - b0 + jobbins) / jobbins);
                    if (j >= cnt && j < cnt + nj) {
                        ji = i;
                        jside = side;
                        jb0 = b0 + (int64_t)(j - cnt) * jobbins;
                        jb1 = jb0 + jobbins - 1 < b1 ? jb0 + jobbins - 1 : b1;
                    }
                    cnt += nj;
                }
        }
        const int d = D0 + ji;
        const int64_t o = ig.dir[ji].o;
        mw::Int<NLS> acc[NK];
        StaticFor<0, NK>::run([&](auto kc) { mw::set_zero(acc[decltype(kc)::value]); });
        for (int64_t b = jb0 + lane; b <= jb1; b += 64) {
            const uint32_t P = pix(ji, d, b);
            if (P == 0u) continue;
            const uint32_t a = (uint32_t)(jside == 0 ? (o - b) : (b - o));
            mw::Int<NLS> t;
            mw::set_u64(t, P);
            // t runs through P * a^k for k = 0 .. K
            StaticFor<0, KMAX + 1>::run([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                if (k <= K) {
                    if constexpr (k >= D0) {
                        if (k >= d) mw::add(acc[k - D0], t);
                    }
                    if (k < K) mw::mul_u32(t, a);
                }
            });
        }
        // wave reduction (butterfly over 64 lanes, exact with carries)
        StaticFor<0, NK>::run([&](auto kc) {
            constexpr int kk = decltype(kc)::value;
            const int k = kk + D0;
            if (k >= d && k <= K) {
                mw::Int<NLS> &v = acc[kk];
#pragma unroll
                for (int m = 1; m < 64; m <<= 1) {
                    mw::Int<NLS> o2;
#pragma unroll
                    for (int l = 0; l < NLS; ++l) o2.w[l] = (uint32_t)__shfl_xor((int)v.w[l], m, 64);
                    mw::add(v, o2);
                }
                if (lane == 0) {
                    uint32_t *dst = jobres + ((size_t)j * NK + kk) * NLS;
#pragma unroll
                    for (int l = 0; l < NLS; ++l) dst[l] = v.w[l];
                }
            }
        });
    }
    __syncthreads();

    // ---------------- step 3: per (d, k) totals; the negative side carries (-1)^k
    int npg = 0;  // pairs of this group
    for (int i = 0; i < ND; ++i) npg += (K >= D0 + i) ? (K + 1 - (D0 + i)) : 0;
    for (int pidx = tid; pidx < npg; pidx += NW * 64) {
        int i = 0, rem = pidx;
        while (rem >= K + 1 - (D0 + i)) {
            rem -= K + 1 - (D0 + i);
            ++i;
        }
        const int d = D0 + i, k = d + rem;
        mw::Int<NLS> tot;
        mw::set_zero(tot);
        int cnt = 0;
        for (int i2 = 0; i2 < ND; ++i2)
            for (int side = 0; side < 2; ++side) {
                int64_t b0, b1;
                if (!seg_range(ig.dir[i2], side, b0, b1)) continue;
                const int nj = (int)((b1 - b0 + jobbins) / jobbins);
                if (i2 == i) {
                    for (int q = 0; q < nj; ++q) {
                        mw::Int<NLS> v;
                        const uint32_t *src = jobres + ((size_t)(cnt + q) * NK + (k - D0)) * NLS;
#pragma unroll
                        for (int l = 0; l < NLS; ++l) v.w[l] = src[l];
                        if (side == 0 && (k & 1)) mw::sub(tot, v);
                        else mw::add(tot, v);
                    }
                }
                cnt += nj;
            }
        uint32_t *dst = part_out + (size_t)pair_index(K, d, k) * NLS;
#pragma unroll
        for (int l = 0; l < NLS; ++l) dst[l] = tot.w[l];
    }
}

// ------------------------------------------------------------ kernels
template <typename VT, int D0, int ND, int NLS, bool FAST>
__global__ void __launch_bounds__(SLICE_WAVES * 64)
slice_kernel(SliceArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ ItemGeom ig;
    const int64_t item = blockIdx.x;
    const int64_t y = item / a.zsplits;
    const int64_t zs = (item % a.zsplits) * a.zrows;
    const int64_t ze = zs + a.zrows < a.N ? zs + a.zrows : a.N;
    slice_item<VT, D0, ND, NLS, FAST>(reinterpret_cast<const VT *>(a.vol), a.L, a.N, a.pitch_y,
                                      a.pitch_z, y, zs, ze, a.K, a.R, a.CT, a.jobbins,
                                      a.part + (size_t)item * a.npairs * NLS, a.images, a.img_off,
                                      a.img_w, lds, ig);
}

template <typename VT, int D0, int ND, int NLS>
__global__ void __launch_bounds__(SLICE_WAVES * 64)
slice_batched_kernel(BatchSliceArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ ItemGeom ig;
    const BatchItem it = a.items[blockIdx.x];
    const RoiDesc rd = a.rois[it.roi];
    if (rd.elem != (int)sizeof(VT)) return;
    slice_item<VT, D0, ND, NLS, false>(reinterpret_cast<const VT *>(a.packed + rd.offset), rd.L,
                                       rd.N, rd.L, rd.L * rd.M, it.y, it.zs, it.ze, a.K, rd.R, rd.CT,
                                       a.jobbins, a.part + (size_t)it.slot * a.npairs * NLS, nullptr,
                                       nullptr, nullptr, lds, ig);
}

// ------------------------------------------------------------ launch helpers
template <typename VT, int D0, int ND, int NLS, bool FAST>
hipError_t launch_one(const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    auto k = slice_kernel<VT, D0, ND, NLS, FAST>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(items), dim3(SLICE_WAVES * 64), lds, st, a);
    return hipGetLastError();
}

template <typename VT, int D0, int NLS, bool FAST>
hipError_t launch_nd(int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    switch (nd) {
        case 1: return launch_one<VT, D0, 1, NLS, FAST>(a, items, lds, st);
        case 2: return launch_one<VT, D0, 2, NLS, FAST>(a, items, lds, st);
        case 3: return launch_one<VT, D0, 3, NLS, FAST>(a, items, lds, st);
        case 4: return launch_one<VT, D0, 4, NLS, FAST>(a, items, lds, st);
        case 5: return launch_one<VT, D0, 5, NLS, FAST>(a, items, lds, st);
        default:
            if constexpr (D0 == 0) {
                if (nd == 6) return launch_one<VT, D0, 6, NLS, FAST>(a, items, lds, st);
                if (nd == 7) return launch_one<VT, D0, 7, NLS, FAST>(a, items, lds, st);
            }
            return hipErrorInvalidValue;
    }
}

template <typename VT, int D0, int ND, int NLS>
hipError_t launch_b_one(const BatchSliceArgs &a, int items, size_t lds, hipStream_t st) {
    auto k = slice_batched_kernel<VT, D0, ND, NLS>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(items), dim3(SLICE_WAVES * 64), lds, st, a);
    return hipGetLastError();
}

}  // namespace dpm
