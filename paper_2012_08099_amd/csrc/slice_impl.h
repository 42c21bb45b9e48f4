// Projection kernel: one workgroup per work item (one y-slice of one volume, rows
// [zs, ze)).  It forms the image rows I_d(., y) of every direction d of its group in
// one coalesced pass over the voxels (Section 3.1, eq. 4; the projection loop of
// Section 5) and writes each row, split at the image's true origin o_d into a negative
// side (a = o_d - i) and a non-negative side (a = i - o_d), to the row buffer read by
// the power-sum kernel.  o_d = |beta| (N-1) for beta < 0 puts the moment origin of a
// negative-index image at column N-1 (the offset correction of Section 5).
//
// Projection mapping (gfx950, wave64): a sub-row of R lanes covers one volume row, lane
// r owning the G = 8 consecutive voxels x0 = 64*G*ct + G*r .. x0+G-1, one 16-byte
// (uint16) or 8-byte (uint8) non-temporal load.  Each sub-row walks a contiguous range of 8-row units (z), loads
// of the next unit in flight while the current one is summed.  Per voxel and direction
// there is one integer add into a register window; windows are flushed to LDS row
// accumulators every T_d rows with ds_add at compile-time offsets.  The (0,1) direction
// needs a full-row sum per z: v_dot2/v_dot4 then a DPP reduction over 8-lane groups.
//
// No global atomics anywhere.
#pragma once
#include "dpm_common.h"
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

// One lane's voxels of one row: G = lane_voxels(elem) voxels, one 16-byte (uint16) or
// 8-byte (uint8) load.
template <typename VT>
struct VecOf;
template <>
struct VecOf<uint16_t> {
    using type = uint4;
    typedef unsigned int raw __attribute__((ext_vector_type(4)));
    static constexpr int G = lane_voxels(2);
};
template <>
struct VecOf<uint8_t> {
    using type = uint2;
    typedef unsigned int raw __attribute__((ext_vector_type(2)));
    static constexpr int G = lane_voxels(1);
};

template <typename VT>
__device__ __forceinline__ uint32_t voxel(const typename VecOf<VT>::type &v, int j) {
    if constexpr (sizeof(VT) == 2) {
        const uint32_t w = j < 2 ? v.x : j < 4 ? v.y : j < 6 ? v.z : v.w;
        return (j & 1) ? (w >> 16) : (w & 0xffffu);
    } else {
        const uint32_t w = j < 4 ? v.x : v.y;
        return (w >> (8 * (j & 3))) & 0xffu;
    }
}

// sum of the voxels of a lane
template <typename VT>
__device__ __forceinline__ uint32_t lane_sum(const typename VecOf<VT>::type &v) {
    if constexpr (sizeof(VT) == 2) {
        typedef unsigned short us2 __attribute__((ext_vector_type(2)));
        const us2 one = {1, 1};
        uint32_t s = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v.x), one, 0u, false);
        s = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v.y), one, s, false);
        s = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v.z), one, s, false);
        return __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v.w), one, s, false);
    } else {
        const uint32_t s = __builtin_amdgcn_udot4(v.x, 0x01010101u, 0u, false);
        return __builtin_amdgcn_udot4(v.y, 0x01010101u, s, false);
    }
}

// Sum over each aligned group of 8 lanes; every lane of the group gets the total.
__device__ __forceinline__ uint32_t group8_sum(uint32_t s) {
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x141, 0xF, 0xF, false);  // row_half_mirror
    return s;
}

// Is (tt, j) the first touch of its window slot within a block (t outer, j inner)?
template <int D, int G>
__device__ constexpr bool first_touch(int tt, int j) {
    const int A = dir_alpha(D), Bt = dir_beta(D), SH = dir_shift(D, G);
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
template <int D, int G>
__device__ constexpr bool slot_used(int s) {
    const int A = dir_alpha(D), Bt = dir_beta(D), SH = dir_shift(D, G);
    for (int t2 = 0; t2 < dir_td(D, G); ++t2)
        for (int j2 = 0; j2 < G; ++j2)
            if (A * j2 + Bt * t2 + SH == s) return true;
    return false;
}

template <typename VT, bool FAST>
__device__ __forceinline__ typename VecOf<VT>::type load_lane(const VT *row, int64_t x0, int64_t L, bool in) {
    using Vec = typename VecOf<VT>::type;
    using Raw = typename VecOf<VT>::raw;
    constexpr int G = VecOf<VT>::G;
    Vec v{};
    if constexpr (FAST) {
        // streamed once: non-temporal, so it does not evict the small shared tables
        const Raw r = __builtin_nontemporal_load(reinterpret_cast<const Raw *>(row + x0));
        __builtin_memcpy(&v, &r, sizeof(Vec));
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
};

// ------------------------------------------------------------ step 1: projection
template <typename VT, int D0, int ND, bool FAST>
__device__ void project_rows(const VT *__restrict__ slice, int64_t L, int64_t pitch_z, int64_t zs,
                             int64_t ze, int R, int CT, uint32_t *lds, const ItemGeom &ig) {
    using Tr = GroupTraits<D0, ND>;
    using Vec = typename VecOf<VT>::type;
    constexpr int G = VecOf<VT>::G;
    constexpr int T = Tr::T;
    constexpr int NW = slice_waves((int)sizeof(VT));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int SR = 64 / R;
    const int sr = lane / R, r = lane % R;
    const int gsr = wave * SR + sr, NSR = NW * SR;
    const int64_t nch = ig.n_chunks;
    const int64_t U = (int64_t)CT * nch;
    const int64_t u_begin = (int64_t)gsr * U / NSR, u_end = (int64_t)(gsr + 1) * U / NSR;

    uint32_t xy[G];
#pragma unroll
    for (int j = 0; j < G; ++j) xy[j] = 0u;

    // geometry constants in registers (the geometry lives in LDS next to the atomics)
    int32_t cbase[ND], coff[ND];
    StaticFor<0, ND>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        cbase[i] = (int32_t)(ig.dir[i].o - dir_shift(D0 + i, G) - ig.dir[i].lo);
        coff[i] = ig.dir[i].lds_off;
    });
    const int32_t yz_off = ig.yz_off, yz_stride = ig.yz_stride;

    // unit u = ct * nch + ch: column tile ct, T-row chunk ch.  Positions advance by
    // counters (no divisions in the loop); a unit's first row pointer is kept per lane.
    struct Pos {
        int32_t ct, ch;
        const VT *p;  // row zs + ch * T of this lane's voxels
    };
    const int64_t chunk_step = (int64_t)T * pitch_z;
    auto pos_of = [&](int64_t u) {
        Pos q;
        q.ct = (int32_t)(u / nch);
        q.ch = (int32_t)(u - (int64_t)q.ct * nch);
        q.p = slice + (zs + (int64_t)q.ch * T) * pitch_z + ((int64_t)q.ct * 64 * G + (int64_t)r * G);
        return q;
    };
    auto next_pos = [&](Pos q) {
        ++q.ch;
        q.p += chunk_step;
        if (q.ch == nch) {
            q.ch = 0;
            ++q.ct;
            q.p = slice + zs * pitch_z + ((int64_t)q.ct * 64 * G + (int64_t)r * G);
        }
        return q;
    };

    auto load_unit = [&](Vec(&buf)[T], const Pos &q) {
        const int64_t x0 = (int64_t)q.ct * 64 * G + (int64_t)r * G;
        const bool valid = x0 < L;
        const int64_t zc0 = zs + (int64_t)q.ch * T;
        StaticFor<0, T>::run([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            if constexpr (FAST) {
                buf[t] = load_lane<VT, true>(q.p + t * pitch_z, 0, L, true);
            } else {
                const int64_t z = zc0 + t;
                const bool in = valid && z < ze;
                buf[t] = load_lane<VT, false>(slice + (z < ze ? z : ze - 1) * pitch_z, x0, L, in);
            }
        });
    };

    auto process_unit = [&](const Vec(&dat)[T], const Pos &q, bool last_in_tile) {
        const int32_t x0 = q.ct * 64 * G + r * G;
        const bool valid = x0 < L;
        const int32_t zc0 = (int32_t)zs + q.ch * T;
        uint32_t yzs[T];
        StaticFor<0, T>::run([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            const Vec &v = dat[t];
            if constexpr (Tr::has_xy) {
                StaticFor<0, G>::run([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    xy[j] += voxel<VT>(v, j);
                });
            }
            if constexpr (Tr::has_yz) yzs[t] = group8_sum(lane_sum<VT>(v));
        });

        // sheared directions: register windows, flushed every T_d rows
        StaticFor<0, ND>::run([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int d = D0 + i;
            if constexpr (d >= 2) {
                constexpr int A = dir_alpha(d), Bt = dir_beta(d), TD = dir_td(d, G);
                constexpr int S = dir_slots(d, G), SH = dir_shift(d, G), PP = dir_pp(d, G);
                // lane base in bins relative to the LDS row origin (32-bit: bins < 2^31)
                const int32_t rel0 = (int32_t)(A * x0 + Bt * zc0) + cbase[i];
                const int32_t doff = coff[i];
                uint32_t w[S];
                StaticFor<0, T>::run([&](auto tc) {
                    constexpr int t = decltype(tc)::value;
                    constexpr int tt = t % TD;
                    const Vec &v = dat[t];
                    StaticFor<0, G>::run([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        constexpr int s = A * j + Bt * tt + SH;
                        if constexpr (first_touch<d, G>(tt, j)) w[s] = voxel<VT>(v, j);
                        else w[s] += voxel<VT>(v, j);
                    });
                    if constexpr (tt == TD - 1) {
                        if (FAST || valid) {
                            const uint32_t lb = (uint32_t)(rel0 + Bt * (t - (TD - 1)));
                            uint32_t *base = lds + doff + (lb + lb / PP);
                            StaticFor<0, S>::run([&](auto sc) {
                                constexpr int s = decltype(sc)::value;
                                if constexpr (slot_used<d, G>(s)) atomicAdd(base + (s + s / PP), w[s]);
                            });
                        }
                    }
                });
            }
        });

        if constexpr (Tr::has_yz) {
            if ((lane & 7) == 0) {
                uint32_t *base = lds + yz_off + ((lane >> 3) & (YZ_COPIES - 1)) * yz_stride +
                                 (uint32_t)(zc0 - zs);
                StaticFor<0, T>::run([&](auto tc) {
                    constexpr int t = decltype(tc)::value;
                    atomicAdd(base + t, yzs[t]);
                });
            }
        }
        // XY: flush when the next unit of this sub-row is in another column tile
        if constexpr (Tr::has_xy) {
            if (last_in_tile) {
                if (FAST || valid) {
                    const uint32_t x0u = (uint32_t)x0;
                    uint32_t *base = lds + coff[0] + (x0u + x0u / (uint32_t)dir_pp(0, G));
                    StaticFor<0, G>::run([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        atomicAdd(base + j, xy[j]);
                    });
                }
#pragma unroll
                for (int j = 0; j < G; ++j) xy[j] = 0u;
            }
        }
    };

    // two units in flight: the loads of unit u+1 are issued before unit u is summed
    Vec bufA[T], bufB[T];
    if (u_begin >= u_end) return;
    const int32_t n = (int32_t)(u_end - u_begin);
    Pos pa = pos_of(u_begin), pb;
    load_unit(bufA, pa);
    for (int32_t k = 0; k < n; k += 2) {
        pb = next_pos(pa);
        if (k + 1 < n) load_unit(bufB, pb);
        process_unit(bufA, pa, k + 1 >= n || pb.ct != pa.ct);
        if (k + 1 >= n) break;
        pa = next_pos(pb);
        if (k + 2 < n) load_unit(bufA, pa);
        process_unit(bufB, pb, k + 2 >= n || pa.ct != pb.ct);
    }
}

// One row side (segment) with everything needed to read its values, in registers (the
// geometry itself lives in LDS).
struct SegView {
    const uint32_t *row;  // LDS row accumulator (or first (0,1) copy)
    int32_t lo;           // bin of row index 0
    int32_t o;            // image column of the origin
    int32_t alo, ahi;     // coordinate magnitudes held by the segment
    int32_t neg;          // 1: a = o - bin, 0: a = bin - o
    int32_t yz;           // 1: (0,1) image, sum of the copies
    int32_t yz_stride;
    int32_t pp;           // LDS padding period of the row
};

__device__ __forceinline__ SegView seg_view(const uint32_t *lds, const ItemGeom &ig, int i, int side, bool yz,
                                            int pp) {
    SegView v;
    v.pp = pp;
    v.neg = side == 0;
    v.alo = ig.seg_alo[2 * i + side];
    v.ahi = ig.seg_ahi[2 * i + side];
    v.o = ig.dir[i].o;
    v.lo = ig.dir[i].lo;
    v.yz = yz;
    v.yz_stride = ig.yz_stride;
    v.row = lds + ig.dir[i].lds_off;
    return v;
}

// row value at coordinate magnitude a (caller keeps a inside [alo, ahi])
__device__ __forceinline__ uint32_t seg_value(const SegView &v, int32_t a) {
    const int32_t b = v.neg ? v.o - a : v.o + a;
    const uint32_t u = (uint32_t)(b - v.lo);
    if (v.yz) {
        uint32_t s = 0;
#pragma unroll
        for (int c = 0; c < YZ_COPIES; ++c) s += v.row[u + c * v.yz_stride];
        return s;
    }
    return v.row[u + u / (uint32_t)v.pp];
}

// ------------------------------------------------------------ per-item driver
template <typename VT, int D0, int ND, bool FAST>
__device__ void slice_item(const VT *__restrict__ vol, int64_t L, int64_t N, int64_t pitch_y,
                           int64_t pitch_z, int64_t y, int64_t zs, int64_t ze, int R, int CT,
                           int32_t *__restrict__ rows_out, const int32_t *slot_off, const int32_t *slot_len,
                           int32_t *__restrict__ img, const int64_t *img_off, const int64_t *img_w,
                           uint32_t *lds, ItemGeom &ig) {
    using Tr = GroupTraits<D0, ND>;
    constexpr int NW = slice_waves((int)sizeof(VT));
    const int tid = threadIdx.x;

    // geometry: one thread per direction, then the LDS offsets
    if (tid < ND) {
        DirGeom dg;
        int32_t an, hn, ap, hp;
        dir_geometry(Tr::g, tid, VecOf<VT>::G, L, N, zs, ze, dg, an, hn, ap, hp);
        ig.dir[tid] = dg;
        ig.seg_alo[2 * tid] = an;
        ig.seg_ahi[2 * tid] = hn;
        ig.seg_alo[2 * tid + 1] = ap;
        ig.seg_ahi[2 * tid + 1] = hp;
    }
    __syncthreads();
    if (tid == 0) {
        int32_t off = 0;
        ig.yz_off = -1;
        ig.yz_stride = 0;
        for (int i = 0; i < ND; ++i) {
            ig.dir[i].lds_off = off;
            if (D0 + i == 1) {
                ig.yz_off = off;
                ig.yz_stride = ig.dir[i].lds_len / YZ_COPIES;
            }
            off += ig.dir[i].lds_len;
        }
        ig.lds_dwords = off;
        ig.n_chunks = (int32_t)((ze - zs + Tr::T - 1) / Tr::T);
    }
    __syncthreads();
    for (int i = tid; i < ig.lds_dwords; i += NW * 64) lds[i] = 0u;
    __syncthreads();

    project_rows<VT, D0, ND, FAST>(vol + y * pitch_y, L, pitch_z, zs, ze, R, CT, lds, ig);
    __syncthreads();

    if (img) {
        StaticFor<0, ND>::run([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const int64_t lo = ig.dir[i].rb_lo, hi = ig.dir[i].rb_hi, o = ig.dir[i].o;
            constexpr int pp = dir_pp(D0 + i, VecOf<VT>::G);
            const SegView vn = seg_view(lds, ig, i, 0, D0 + i == 1, pp), vp = seg_view(lds, ig, i, 1, D0 + i == 1, pp);
            int32_t *row = img + img_off[i] + y * img_w[i];
            for (int64_t b = lo + tid; b <= hi; b += NW * 64)
                row[b] = (int32_t)(b < o ? seg_value(vn, (int32_t)(o - b)) : seg_value(vp, (int32_t)(b - o)));
        });
    }

    // row sides to the power-sum input: slot 2d + side, a = 0 .. len-1
    StaticFor<0, ND>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int d = D0 + i;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int s = 2 * d + side;
            const int32_t len = slot_len[s];
            if (len == 0) continue;
            const SegView v = seg_view(lds, ig, i, side, d == 1, dir_pp(d, VecOf<VT>::G));
            // 16-byte stores: len is a multiple of 64 and the rows are 256-byte aligned
            int4 *dst = reinterpret_cast<int4 *>(rows_out + slot_off[s]);
            for (int32_t a = 4 * tid; a < len; a += 4 * NW * 64) {
                int32_t e[4];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    e[c] = (int32_t)((a + c >= v.alo && a + c <= v.ahi) ? seg_value(v, a + c) : 0u);
                dst[a >> 2] = make_int4(e[0], e[1], e[2], e[3]);
            }
        }
    });
}

// ------------------------------------------------------------ kernels
template <typename VT, int D0, int ND, bool FAST>
__global__ void __launch_bounds__(slice_waves((int)sizeof(VT)) * 64)
slice_kernel(SliceArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ ItemGeom ig;
    const int64_t item = blockIdx.x;
    const int64_t y = item / a.zsplits;
    const int64_t zs = (item % a.zsplits) * a.zrows;
    const int64_t ze = zs + a.zrows < a.N ? zs + a.zrows : a.N;
    slice_item<VT, D0, ND, FAST>(reinterpret_cast<const VT *>(a.vol), a.L, a.N, a.pitch_y, a.pitch_z, y, zs,
                                 ze, a.R, a.CT, a.rows + item * a.rl.row_stride, a.rl.slot_off,
                                 a.rl.slot_len, a.images, a.img_off, a.img_w, lds, ig);
}

template <typename VT, int D0, int ND>
__global__ void __launch_bounds__(slice_waves((int)sizeof(VT)) * 64)
slice_batched_kernel(BatchSliceArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ ItemGeom ig;
    const BatchItem it = a.items[blockIdx.x];
    const RoiDesc &rd = a.rois[it.roi];
    if (rd.elem != (int)sizeof(VT)) return;
    slice_item<VT, D0, ND, false>(reinterpret_cast<const VT *>(a.packed + rd.offset), rd.L, rd.N, rd.L,
                                  rd.L * rd.M, it.y, it.zs, it.ze, rd.R, rd.CT,
                                  a.rows + rd.row_base + (int64_t)it.y * rd.row_stride, rd.slot_off,
                                  rd.slot_len, nullptr, nullptr, nullptr, lds, ig);
}

// ------------------------------------------------------------ launch helpers
template <typename VT, int D0, int ND, bool FAST>
hipError_t launch_one(const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    auto k = slice_kernel<VT, D0, ND, FAST>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(items), dim3(slice_waves((int)sizeof(VT)) * 64), lds, st, a);
    return hipGetLastError();
}

template <typename VT, int D0, bool FAST>
hipError_t launch_nd(int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    switch (nd) {
        case 1: return launch_one<VT, D0, 1, FAST>(a, items, lds, st);
        case 2: return launch_one<VT, D0, 2, FAST>(a, items, lds, st);
        case 3: return launch_one<VT, D0, 3, FAST>(a, items, lds, st);
        case 4: return launch_one<VT, D0, 4, FAST>(a, items, lds, st);
        case 5: return launch_one<VT, D0, 5, FAST>(a, items, lds, st);
        default:
            if constexpr (D0 == 0) {
                if (nd == 6) return launch_one<VT, D0, 6, FAST>(a, items, lds, st);
                if (nd == 7) return launch_one<VT, D0, 7, FAST>(a, items, lds, st);
            }
            return hipErrorInvalidValue;
    }
}

template <typename VT, int D0, int ND>
hipError_t launch_b_one(const BatchSliceArgs &a, int items, size_t lds, hipStream_t st) {
    auto k = slice_batched_kernel<VT, D0, ND>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(items), dim3(slice_waves((int)sizeof(VT)) * 64), lds, st, a);
    return hipGetLastError();
}

}  // namespace dpm
