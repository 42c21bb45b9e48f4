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

// Sum over each aligned group of gs lanes (gs = 1, 2, 4 or 8, uniform); every lane of the
// group gets the total.
__device__ __forceinline__ uint32_t group_sum(uint32_t s, int gs) {
    if (gs >= 2) s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0xB1, 0xF, 0xF, false);
    if (gs >= 4) s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x4E, 0xF, 0xF, false);
    if (gs >= 8) s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x141, 0xF, 0xF, false);
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

// safe_end (general loads only, may be null): every byte before it may be read, so a lane
// whose dwords all lie before it loads them without a check per dword.  NTL (whole-row
// loads): non-temporal, for a volume read once; plain where sibling workgroups of the same
// XCD read the same rows after this one (the direction groups of one launch), so that the
// lines stay in L2 for them.
template <typename VT, bool FAST, bool NTL = true>
__device__ __forceinline__ typename VecOf<VT>::type load_lane(const VT *row, int64_t x0, int64_t L, bool in,
                                                              const uint8_t *safe_end = nullptr) {
    using Vec = typename VecOf<VT>::type;
    using Raw = typename VecOf<VT>::raw;
    constexpr int G = VecOf<VT>::G;
    Vec v{};
    if constexpr (FAST) {
        Raw r;
        if constexpr (NTL)  // streamed once: does not evict the small shared tables
            r = __builtin_nontemporal_load(reinterpret_cast<const Raw *>(row + x0));
        else
            r = *reinterpret_cast<const Raw *>(row + x0);
        __builtin_memcpy(&v, &r, sizeof(Vec));
    } else if (in) {
        // Any alignment, ragged row end: the aligned dwords that hold at least one
        // byte of the lane's nv voxels (never a dword past the row's last byte, so never
        // a page the row does not touch), funnel-shifted into place; bytes past the row
        // end are cleared.
        constexpr int NB = (int)sizeof(Vec);  // bytes of a full lane
        constexpr int NDW = NB / 4 + 1;
        const int64_t nv = L - x0 < G ? L - x0 : G;  // >= 1 (x0 < L)
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(row + x0);
        const uintptr_t last = a0 + (uintptr_t)nv * sizeof(VT) - 1;
        const uint32_t *dw = reinterpret_cast<const uint32_t *>(a0 & ~(uintptr_t)3);
        const uint32_t sh = (uint32_t)(a0 & 3);
        uint32_t d[NDW];
        if (safe_end && reinterpret_cast<const uint8_t *>(dw + NDW) <= safe_end) {
#pragma unroll
            for (int k = 0; k < NDW; ++k) d[k] = dw[k];  // bytes past the row are cleared below
        } else {
#pragma unroll
            for (int k = 0; k < NDW; ++k)
                d[k] = (reinterpret_cast<uintptr_t>(dw + k) <= last) ? dw[k] : 0u;
        }
        const int nbv = (int)(nv * (int64_t)sizeof(VT));
        uint32_t w[NB / 4];
#pragma unroll
        for (int i = 0; i < NB / 4; ++i) {
            const uint32_t x = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh);
            const int keep = nbv - 4 * i;  // bytes of this dword inside the row
            w[i] = keep >= 4 ? x : keep <= 0 ? 0u : (x & ((1u << (8 * keep)) - 1u));
        }
        __builtin_memcpy(&v, w, sizeof(Vec));
    }
    return v;
}

template <int ND>
struct Tr0 {
    static constexpr bool has_xy = true;
    static constexpr bool has_yz = ND >= 2;
};

template <int D0, int ND>
struct GroupTraits {
    static constexpr int g = D0 == 0 ? 0 : D0 == 7 ? 1 : 2;
    static constexpr int T = group_rows(g);
    static constexpr bool has_xy = (D0 == 0);
    static constexpr bool has_yz = (D0 == 0 && ND >= 2);
};

// ------------------------------------------------------------ step 1: projection
// Units (T rows of a lane's voxels) whose loads are in flight per wave.  One: the load
// buffers then hold few registers (about 110 instead of 200 for the uint16 first group),
// so more waves share a CU -- eight-wave workgroups, or the power sums and recombination of
// another volume on a second stream -- which hides the load latency better than a second
// buffer in each wave.
#ifndef SLICE_UNITS_IN_FLIGHT
#define SLICE_UNITS_IN_FLIGHT 1
#endif

// MS: the item is nsl consecutive slices (slice s at slice + s pitch_y, its row
// accumulators at lds + s sw), whose units the sub-rows share: small slices then keep
// more of the wave busy.
template <typename VT, int D0, int ND, bool FAST, int NW, bool MS = false, int NBU = SLICE_UNITS_IN_FLIGHT,
          bool NTL = true>
__device__ __forceinline__ void project_rows(const VT *__restrict__ slice, int64_t L, int64_t pitch_z, int64_t zs,
                             int64_t ze, int R, int CT, uint32_t *lds, const ItemGeom &ig, int nsl = 1,
                             int64_t pitch_y = 0, int32_t sw = 0, const uint8_t *safe_end = nullptr) {
    using Tr = GroupTraits<D0, ND>;
    using Vec = typename VecOf<VT>::type;
    constexpr int G = VecOf<VT>::G;
    constexpr int T = Tr::T;
    const int lane = threadIdx.x & 63;
    // a one-wave item may run inside a larger workgroup (the fused batched kernel): its
    // wave is then the only one of the item
    const int wave = NW == 1 ? 0 : (int)(threadIdx.x >> 6);
    const int SR = 64 / R;
    const int sr = lane / R, r = lane % R;
    // (0,1) row sums over 8-lane groups; multi-slice items may have narrower sub-rows
    // (R = 1, 2 or 4), whose sums then take the whole sub-row
    int gs = 8;
    if constexpr (MS) gs = R < 8 ? R : 8;
    const int gsr = wave * SR + sr, NSR = NW * SR;
    const int64_t nch = ig.n_chunks;
    const int64_t U1 = (int64_t)CT * nch;  // units of one slice
    const int64_t U = MS ? U1 * nsl : U1;
    // (multi-slice items are small: 32-bit unit arithmetic)
    const int64_t u_begin = MS ? (int64_t)((uint32_t)(gsr * U) / (uint32_t)NSR) : (int64_t)gsr * U / NSR;
    const int64_t u_end = MS ? (int64_t)((uint32_t)((gsr + 1) * U) / (uint32_t)NSR) : (int64_t)(gsr + 1) * U / NSR;

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

    // unit u = (sl * CT + ct) * nch + ch: slice sl (MS only), column tile ct, T-row chunk
    // ch.  Positions advance by counters (no divisions in the loop); a unit's first row
    // pointer is kept per lane.
    struct Pos {
        int32_t ct, ch, sl;
        const VT *p;  // row zs + ch * T of this lane's voxels
    };
    const int64_t chunk_step = (int64_t)T * pitch_z;
    auto pos_of = [&](int64_t u) {
        Pos q;
        q.sl = 0;
        if constexpr (MS) {
            q.sl = (int32_t)((uint32_t)u / (uint32_t)U1);
            u -= (int64_t)q.sl * U1;
            q.ct = (int32_t)((uint32_t)u / (uint32_t)nch);
        } else {
            q.ct = (int32_t)(u / nch);
        }
        q.ch = (int32_t)(u - (int64_t)q.ct * nch);
        q.p = slice + (MS ? q.sl * pitch_y : 0) + (zs + (int64_t)q.ch * T) * pitch_z +
              ((int64_t)q.ct * 64 * G + (int64_t)r * G);
        return q;
    };
    auto next_pos = [&](Pos q) {
        ++q.ch;
        q.p += chunk_step;
        if (q.ch == nch) {
            q.ch = 0;
            ++q.ct;
            if constexpr (MS) {
                if (q.ct == CT) {
                    q.ct = 0;
                    ++q.sl;
                }
            }
            q.p = slice + (MS ? q.sl * pitch_y : 0) + zs * pitch_z + ((int64_t)q.ct * 64 * G + (int64_t)r * G);
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
                buf[t] = load_lane<VT, true, NTL>(q.p + t * pitch_z, 0, L, true);
            } else {
                const int64_t z = zc0 + t;
                const bool in = valid && z < ze;
                buf[t] = load_lane<VT, false>(slice + (MS ? q.sl * pitch_y : 0) + (z < ze ? z : ze - 1) * pitch_z,
                                              x0, L, in, MS ? safe_end : nullptr);
            }
        });
    };

    auto process_unit = [&](const Vec(&dat)[T], const Pos &q, bool last_in_tile) {
        uint32_t *const ul = lds + (MS ? q.sl * sw : 0);  // this unit's slice's accumulators
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
            if constexpr (Tr::has_yz) {
                if constexpr (MS) yzs[t] = group_sum(lane_sum<VT>(v), gs);
                else yzs[t] = group8_sum(lane_sum<VT>(v));
            }
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
                            uint32_t *base = ul + doff + (lb + lb / PP);
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
            bool writer = (lane & 7) == 0;
            if constexpr (MS) writer = (lane & (gs - 1)) == 0;
            if (writer) {
                uint32_t *base = ul + yz_off + ((lane >> 3) & (YZ_COPIES - 1)) * yz_stride +
                                 (uint32_t)(zc0 - zs);
                StaticFor<0, T>::run([&](auto tc) {
                    constexpr int t = decltype(tc)::value;
                    atomicAdd(base + t, yzs[t]);
                });
            }
        }
        // XY: flush when the next unit of this sub-row is in another column tile (or slice)
        if constexpr (Tr::has_xy) {
            if (last_in_tile) {
                if (FAST || valid) {
                    const uint32_t x0u = (uint32_t)x0;
                    uint32_t *base = ul + coff[0] + (x0u + x0u / (uint32_t)dir_pp(0, G));
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

    if (u_begin >= u_end) return;
    const int32_t n = (int32_t)(u_end - u_begin);
    if constexpr (NBU == 1) {
        // one unit's loads at a time (fewer registers; the other waves hide the latency)
        Vec one[T];
        Pos q = pos_of(u_begin);
        for (int32_t u = 0; u < n; ++u) {
            load_unit(one, q);
            const Pos nq = next_pos(q);
            process_unit(one, q, u + 1 >= n || nq.ct != q.ct || (MS && nq.sl != q.sl));
            q = nq;
        }
        return;
    }
    // NB units in flight: the loads of unit u + NB - 1 are issued before unit u is summed
    // (buffer u % NB; the position of unit u + 1 tells whether u ends its column tile)
    constexpr int NB = NBU;
    Vec buf[NB][T];
    Pos pos[NB];
    pos[0] = pos_of(u_begin);
    load_unit(buf[0], pos[0]);
    StaticFor<1, NB - 1>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        pos[i] = next_pos(pos[i - 1]);
        if (i < n) load_unit(buf[i], pos[i]);
    });
    for (int32_t k = 0; k < n; k += NB) {
        StaticFor<0, NB>::run([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            constexpr int lj = (j + NB - 1) % NB, pj = (j + NB - 2) % NB, nj = (j + 1) % NB;
            const int32_t u = k + j;
            if (u < n) {
                pos[lj] = next_pos(pos[pj]);
                if (u + NB - 1 < n) load_unit(buf[lj], pos[lj]);
                process_unit(buf[j], pos[j], u + 1 >= n || pos[nj].ct != pos[j].ct || (MS && pos[nj].sl != pos[j].sl));
            }
        });
    }
}

// ------------------------------------------------------------ step 1, chained windows
// Variant for whole 64-lane rows (R = 64) of the first direction group, P-row units.
// For direction (alpha, beta) a lane's voxels of one row fall in alpha (G-1) + 1 bins
// that move by beta per row; the lane keeps them in a ring of W = alpha G registers
// (bin mod W).  When the window has moved past a bin, the lane hands the bin's partial
// sum to the neighbouring lane whose window reaches it next (DPP wave shift): that bin
// lands in the neighbour's ring slot it is vacating at the same moment (W = alpha G), so
// the hand-over is one register move.  Each sum travels down the lanes collecting every
// contribution of the wave; only the lane at the end of the chain (lane 0 for beta > 0,
// lane 63 for beta < 0) holds finished bins, and it shifts them into a lane-spread
// register that is written to LDS once per unit (one ds_add of P lanes).
constexpr int CH_P = 32;     // rows per unit
constexpr int CH_LA = 16;    // row slots per lane (loads run LA - 1 rows ahead)
constexpr int CH_WAVES = 4;  // waves per workgroup (about 207 registers: 2 waves per SIMD)

__device__ constexpr int chain_ring(int d) { return dir_alpha(d) * 8; }

template <int D0, int I>
__device__ constexpr int chain_off() {
    int o = 0;
    for (int i = 0; i < I; ++i)
        if (D0 + i >= 2) o += chain_ring(D0 + i);
    return o;
}
template <int D0, int I>
__device__ constexpr int chain_eoff() {
    int o = 0;
    for (int i = 0; i < I; ++i)
        if (D0 + i >= 2) o += iabs_c(dir_beta(D0 + i));
    return o;
}

// Which bin (relative to the unit's frame) ring slot s holds after the last row of a
// unit, in steady state; CH_NONE if none.  Simulates two units of the schedule: adds
// of each row, then the hand-over of the bins the next row cannot reach (the slot
// receives the neighbour's bin, alpha G further along).  CH_BAD flags an add into a
// slot holding another bin (the chain reasoning would be wrong).
constexpr int CH_NONE = -1000000, CH_BAD = -2000000;
template <int D>
__device__ constexpr int chain_slot_bin(int s) {
    constexpr int A = dir_alpha(D), B = dir_beta(D), AB = B < 0 ? -B : B, W = chain_ring(D), P = CH_P;
    int bin[64] = {};
    bool has[64] = {};
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1)
            for (int k = 0; k < W; ++k)
                if (has[k]) bin[k] += B > 0 ? -B * P : AB * P;
        for (int t = 0; t < P; ++t) {
            const int vt = B > 0 ? B * t : AB * (P - 1 - t);
            for (int j = 0; j < 8; ++j) {
                const int v = A * j + vt, sl = v % W;
                if (has[sl] && bin[sl] != v) return CH_BAD;
                has[sl] = true;
                bin[sl] = v;
            }
            const int r0 = B > 0 ? vt : vt + A * 7 - AB + 1;
            for (int k = 0; k < AB; ++k) {
                const int v = r0 + k, sl = v % W;
                if (!has[sl] || bin[sl] != v) return CH_BAD;
                bin[sl] = v + (B > 0 ? A * 8 : -A * 8);
            }
        }
    }
    return has[s] ? bin[s] : CH_NONE;
}
template <int D>
__device__ constexpr bool chain_ok() {
    for (int s = 0; s < chain_ring(D); ++s)
        if (chain_slot_bin<D>(s) == CH_BAD) return false;
    return true;
}

template <typename VT, int ND, int NW>
__device__ void project_rows_chain(const VT *__restrict__ slice, int64_t L, int64_t pitch_z, int64_t zs,
                                   int64_t ze, int CT, uint32_t *lds, const ItemGeom &ig) {
    using Vec = typename VecOf<VT>::type;
    constexpr int G = VecOf<VT>::G;
    static_assert(G == 8, "chained windows assume 8 voxels per lane");
    constexpr int P = CH_P, LA = CH_LA;
    constexpr int NRING = chain_off<0, ND>(), NE = chain_eoff<0, ND>();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int32_t nper = (int32_t)((ze - zs) / P);  // caller guarantees (ze - zs) % P == 0
    const int32_t U = CT * nper;
    const int32_t u_begin = (int32_t)((int64_t)wave * U / NW), u_end = (int32_t)((int64_t)(wave + 1) * U / NW);
    if (u_begin >= u_end) return;
    const int32_t Z = nper * P;

    int32_t dlo[ND], doff[ND];
    StaticFor<0, ND>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        dlo[i] = __builtin_amdgcn_readfirstlane(ig.dir[i].o - ig.dir[i].lo);
        doff[i] = __builtin_amdgcn_readfirstlane(ig.dir[i].lds_off);
    });
    const int32_t yz_off = __builtin_amdgcn_readfirstlane(ig.yz_off);
    const int32_t yz_stride = __builtin_amdgcn_readfirstlane(ig.yz_stride);
    const int32_t sink = __builtin_amdgcn_readfirstlane(ig.lds_dwords) - LDS_SINK;

    uint32_t xy[G];
    uint32_t ring[NRING > 0 ? NRING : 1];
    uint32_t ebuf[NE > 0 ? NE : 1];
#pragma unroll
    for (int j = 0; j < G; ++j) xy[j] = 0u;
#pragma unroll
    for (int k = 0; k < NRING; ++k) ring[k] = 0u;
#pragma unroll
    for (int k = 0; k < NE; ++k) ebuf[k] = 0u;

    auto unit_base = [&](int32_t ct, int32_t per) -> const VT * {
        return slice + (zs + (int64_t)per * P) * pitch_z + ((int64_t)ct * 64 * G + (int64_t)lane * G);
    };
    auto pin = [&]() {
#pragma unroll
        for (int j = 0; j < G; ++j) asm volatile("" : "+v"(xy[j]));
#pragma unroll
        for (int k = 0; k < NRING; ++k) asm volatile("" : "+v"(ring[k]));
    };

    int32_t ct = u_begin / nper, per = u_begin - ct * nper;
    const VT *cb = unit_base(ct, per);
    Vec dbuf[LA];
    StaticFor<0, LA>::run([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        dbuf[t] = load_lane<VT, true>(cb + (int64_t)t * pitch_z, 0, L, true);
        __builtin_amdgcn_sched_barrier(0);
    });

    auto unit = [&](auto more_c) {
        constexpr bool more = decltype(more_c)::value;
        int32_t ct2 = ct, per2 = per + 1;
        if (per2 == nper) {
            per2 = 0;
            ++ct2;
        }
        const VT *nb = more ? unit_base(ct2, per2) : cb;
        const bool seg_end = !more || ct2 != ct;
        const int32_t x0 = ct * 64 * G + lane * G;
        const int32_t zrel0 = per * P;
        const int32_t yzb = (lane & 7) == 0 ? yz_off + ((lane >> 3) & (YZ_COPIES - 1)) * yz_stride + zrel0
                                            : sink + lane;
        // frame of each ring: U0 = alpha x0 + beta z_frame + o - lo, z_frame = first
        // (beta > 0) or last (beta < 0) row of the unit
        int32_t u0[ND];
        StaticFor<0, ND>::run([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int d = i;
            if constexpr (d >= 2) {
                constexpr int A = dir_alpha(d), B = dir_beta(d);
                const int32_t zf = (int32_t)zs + zrel0 + (B < 0 ? P - 1 : 0);
                u0[i] = A * x0 + B * zf + dlo[i];
            }
        });

        StaticFor<0, P>::run([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            const Vec v = dbuf[t % LA];
            if constexpr (Tr0<ND>::has_xy) {
                StaticFor<0, G>::run([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    xy[j] += voxel<VT>(v, j);
                });
            }
            if constexpr (Tr0<ND>::has_yz) atomicAdd(lds + yzb + t, group8_sum(lane_sum<VT>(v)));
            StaticFor<0, ND>::run([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int d = i;
                if constexpr (d >= 2) {
                    constexpr int A = dir_alpha(d), B = dir_beta(d), AB = B < 0 ? -B : B;
                    constexpr int W = chain_ring(d), RO = chain_off<0, i>(), EO = chain_eoff<0, i>();
                    constexpr int vt = B > 0 ? B * t : AB * (P - 1 - t);
                    StaticFor<0, G>::run([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        ring[RO + (A * j + vt) % W] += voxel<VT>(v, j);
                    });
                    // bins the next row cannot reach: hand them along the chain
                    constexpr int r0 = B > 0 ? vt : vt + A * (G - 1) - AB + 1;
                    StaticFor<0, AB>::run([&](auto kc) {
                        constexpr int k = decltype(kc)::value;
                        constexpr int sl = RO + (r0 + k) % W;
                        if constexpr (B > 0) {
                            // end lane 0 keeps its finished bin; lane l passes to l - 1
                            ebuf[EO + k] = (uint32_t)__builtin_amdgcn_update_dpp((int)ring[sl], (int)ebuf[EO + k],
                                                                                 0x138, 0xF, 0xF, false);
                            ring[sl] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)ring[sl], 0x130, 0xF, 0xF, true);
                        } else {
                            ebuf[EO + k] = (uint32_t)__builtin_amdgcn_update_dpp((int)ring[sl], (int)ebuf[EO + k],
                                                                                 0x130, 0xF, 0xF, false);
                            ring[sl] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)ring[sl], 0x138, 0xF, 0xF, true);
                        }
                    });
                }
            });
            if constexpr (t % 2 == 1) pin();
            if constexpr (t + LA < P) dbuf[t % LA] = load_lane<VT, true>(cb + (int64_t)(t + LA) * pitch_z, 0, L, true);
            else if constexpr (more) dbuf[t % LA] = load_lane<VT, true>(nb + (int64_t)(t + LA - P) * pitch_z, 0, L, true);
            __builtin_amdgcn_sched_barrier(0);
        });

        // finished bins of the end lane, one per row (two for |beta| = 2): lane j holds
        // row P-1-j's (beta > 0, lanes 0..P-1) or lane 63-j does (beta < 0)
        StaticFor<0, ND>::run([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int d = i;
            if constexpr (d >= 2) {
                constexpr int A = dir_alpha(d), B = dir_beta(d), AB = B < 0 ? -B : B;
                constexpr int EO = chain_eoff<0, i>();
                const int j = B > 0 ? lane : 63 - lane;
                if (j < P) {
                    // frame of the end lane, then the bin of row P-1-j
                    const int32_t ue = B > 0 ? u0[i] - A * G * lane : u0[i] + A * G * (63 - lane);
                    StaticFor<0, AB>::run([&](auto kc) {
                        constexpr int k = decltype(kc)::value;
                        const int32_t v = B > 0 ? B * (P - 1 - j) + k : AB * j + A * (G - 1) - AB + 1 + k;
                        const uint32_t u = (uint32_t)(ue + v);
                        atomicAdd(lds + doff[i] + (u + u / 8u), ebuf[EO + k]);
                    });
                }
            }
        });

        if (seg_end) {
            // every ring slot of every lane: bins v in [vlo, vlo + W) of its frame
            StaticFor<0, ND>::run([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int d = i;
                if constexpr (d >= 2) {
                    constexpr int A = dir_alpha(d), B = dir_beta(d), AB = B < 0 ? -B : B;
                    constexpr int W = chain_ring(d), RO = chain_off<0, i>();
                    static_assert(chain_ok<d>(), "chained windows: inconsistent ring schedule");
                    StaticFor<0, W>::run([&](auto kc) {
                        constexpr int sl = decltype(kc)::value;
                        constexpr int vb = chain_slot_bin<d>(sl);
                        if constexpr (vb != CH_NONE) {
                            const uint32_t u = (uint32_t)(u0[i] + vb);
                            // a slot of a bin outside the image holds zero: skip it
                            if (ring[RO + sl] != 0u) atomicAdd(lds + doff[i] + (u + u / 8u), ring[RO + sl]);
                        }
                    });
#pragma unroll
                    for (int k = 0; k < W; ++k) ring[RO + k] = 0u;
                }
            });
            if constexpr (Tr0<ND>::has_xy) {
                const uint32_t x0u = (uint32_t)x0;
                uint32_t *base = lds + doff[0] + (x0u + x0u / 8u);
                StaticFor<0, G>::run([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    atomicAdd(base + j, xy[j]);
                });
#pragma unroll
                for (int j = 0; j < G; ++j) xy[j] = 0u;
            }
        }
        ct = ct2;
        per = per2;
        cb = nb;
    };

    for (int32_t u = u_begin; u + 1 < u_end; ++u) unit(std::true_type{});
    unit(std::false_type{});
    (void)Z;
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
template <typename VT, int D0, int ND, bool FAST, bool CHAIN, int NW, bool NTL = true>
__device__ void slice_item(const VT *__restrict__ vol, int64_t L, int64_t N, int64_t pitch_y,
                           int64_t pitch_z, int64_t y, int64_t zs, int64_t ze, int R, int CT,
                           int32_t *__restrict__ rows_out, const int32_t *slot_off, const int32_t *slot_len,
                           int32_t *__restrict__ img, const int64_t *img_off, const int64_t *img_w,
                           uint32_t *lds, ItemGeom &ig, const ItemGeom *pre = nullptr) {
    using Tr = GroupTraits<D0, ND>;
    const int tid = threadIdx.x;

    if (pre) {
        // precomputed for the whole z range (batched items)
        const int32_t *src = reinterpret_cast<const int32_t *>(pre);
        int32_t *dst = reinterpret_cast<int32_t *>(&ig);
        for (int i = tid; i < (int)(sizeof(ItemGeom) / 4); i += NW * 64) dst[i] = src[i];
    } else if (tid < ND) {
        // geometry: one thread per direction, then the LDS offsets
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
    if (!pre && tid == 0) {
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
        ig.lds_dwords = off + LDS_SINK;
        ig.n_chunks = (int32_t)((ze - zs + Tr::T - 1) / Tr::T);
    }
    __syncthreads();
    for (int i = tid; i < ig.lds_dwords; i += NW * 64) lds[i] = 0u;
    __syncthreads();

    if constexpr (CHAIN) {
        static_assert(FAST && D0 == 0, "chained windows: first group, exact rows only");
        project_rows_chain<VT, ND, NW>(vol + y * pitch_y, L, pitch_z, zs, ze, CT, lds, ig);
    } else {
        project_rows<VT, D0, ND, FAST, NW, false, SLICE_UNITS_IN_FLIGHT, NTL>(vol + y * pitch_y, L, pitch_z, zs, ze, R,
                                                                            CT, lds, ig);
    }
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
// NWV: waves per workgroup (4, or 8 for the first group's whole-row kernel when the
// planner or the autotuner asks for it: few slices leave the CUs short of waves)
template <typename VT, int D0, int ND, bool FAST, bool CHAIN = false, int NWV = 4>
__global__ void __launch_bounds__((CHAIN ? CH_WAVES : NWV) * 64)
slice_kernel(SliceArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ ItemGeom ig;
    const int64_t item = blockIdx.x;
    const int64_t y = item / a.zsplits;
    const int64_t zs = (item % a.zsplits) * a.zrows;
    const int64_t ze = zs + a.zrows < a.N ? zs + a.zrows : a.N;
    slice_item<VT, D0, ND, FAST, CHAIN, CHAIN ? CH_WAVES : NWV>(reinterpret_cast<const VT *>(a.vol), a.L, a.N, a.pitch_y, a.pitch_z, y, zs,
                                 ze, a.R, a.CT, a.rows + item * a.rl.row_stride, a.rl.slot_off,
                                 a.rl.slot_len, a.images, a.img_off, a.img_w, lds, ig);
}

// Orders 7-16 in one launch: the direction groups of one work item run as sibling
// workgroups dispatched back to back onto the same XCD (the dispatcher hands workgroups
// to the 8 XCDs round-robin in index order), so the item's rows come from HBM about once
// and to the siblings from that XCD's L2 or the MALL.  Block b: XCD x = b % 8, local
// index l = b / 8; item = (l / NG) * 8 + x, group = l % NG.  Moments only (no images),
// whole-row loads only, and plain (not non-temporal) loads, so that the lines the first
// sibling brings in stay in L2 for the others.
constexpr int NXCD = 8;
// Waves per workgroup of the one-launch groups kernel: its LDS (the widest group's row
// accumulators, about 58 KB at 512^3) leaves room for two workgroups per CU, so eight
// waves each are what keeps four waves on every SIMD.
#ifndef GROUPS_WAVES
#define GROUPS_WAVES 8
#endif

template <typename VT, int ND1, int ND2>
__global__ void __launch_bounds__(GROUPS_WAVES * 64)
slice_groups_kernel(SliceArgs a, int items) {
    extern __shared__ uint32_t lds[];
    __shared__ ItemGeom ig;
    constexpr int NG = ND2 > 0 ? 3 : 2;
    constexpr int NW = GROUPS_WAVES;
    const int b = blockIdx.x, x = b % NXCD, l = b / NXCD;
    const int64_t item = (int64_t)(l / NG) * NXCD + x;
    const int g = l % NG;
    if (item >= items) return;  // uniform over the workgroup
    const int64_t y = item / a.zsplits;
    const int64_t zs = (item % a.zsplits) * a.zrows;
    const int64_t ze = zs + a.zrows < a.N ? zs + a.zrows : a.N;
    const VT *vol = reinterpret_cast<const VT *>(a.vol);
    int32_t *rows = a.rows + item * a.rl.row_stride;
    if (g == 0)
        slice_item<VT, 0, 7, true, false, NW, false>(vol, a.L, a.N, a.pitch_y, a.pitch_z, y, zs, ze, a.R, a.CT, rows,
                                              a.rl.slot_off, a.rl.slot_len, nullptr, nullptr, nullptr, lds, ig);
    else if (g == 1)
        slice_item<VT, 7, ND1, true, false, NW, false>(vol, a.L, a.N, a.pitch_y, a.pitch_z, y, zs, ze, a.R, a.CT, rows,
                                                a.rl.slot_off, a.rl.slot_len, nullptr, nullptr, nullptr, lds, ig);
    else if constexpr (ND2 > 0)
        slice_item<VT, 12, ND2, true, false, NW, false>(vol, a.L, a.N, a.pitch_y, a.pitch_z, y, zs, ze, a.R, a.CT, rows,
                                                 a.rl.slot_off, a.rl.slot_len, nullptr, nullptr, nullptr, lds, ig);
}

template <typename VT, int ND1, int ND2>
hipError_t launch_groups_one(const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    auto k = slice_groups_kernel<VT, ND1, ND2>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    constexpr int NG = ND2 > 0 ? 3 : 2;
    const int64_t blocks = (int64_t)((items + NXCD - 1) / NXCD) * NXCD * NG;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(GROUPS_WAVES * 64), lds, st, a, items);
    return hipGetLastError();
}

// nd = K + 1 in 8 .. 17
template <typename VT>
hipError_t launch_groups_nd(int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    switch (nd) {
        case 8: return launch_groups_one<VT, 1, 0>(a, items, lds, st);
        case 9: return launch_groups_one<VT, 2, 0>(a, items, lds, st);
        case 10: return launch_groups_one<VT, 3, 0>(a, items, lds, st);
        case 11: return launch_groups_one<VT, 4, 0>(a, items, lds, st);
        case 12: return launch_groups_one<VT, 5, 0>(a, items, lds, st);
        case 13: return launch_groups_one<VT, 5, 1>(a, items, lds, st);
        case 14: return launch_groups_one<VT, 5, 2>(a, items, lds, st);
        case 15: return launch_groups_one<VT, 5, 3>(a, items, lds, st);
        case 16: return launch_groups_one<VT, 5, 4>(a, items, lds, st);
        case 17: return launch_groups_one<VT, 5, 5>(a, items, lds, st);
        default: return hipErrorInvalidValue;
    }
}

// Batched items are small slices of small volumes: one wave per item, so that many
// items run side by side on a CU.
constexpr int BATCH_WAVES = 1;

template <typename VT, int D0, int ND>
__global__ void __launch_bounds__(BATCH_WAVES * 64)
slice_batched_kernel(BatchSliceArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ ItemGeom ig;
    const BatchItem it = a.items[blockIdx.x];
    const RoiDesc &rd = a.rois[it.roi];
    if (rd.elem != (int)sizeof(VT)) return;
    slice_item<VT, D0, ND, false, false, BATCH_WAVES>(reinterpret_cast<const VT *>(a.packed + rd.offset), rd.L, rd.N, rd.L,
                                  rd.L * rd.M, it.y, 0, rd.N, rd.R, rd.CT,
                                  a.rows + rd.row_base + (int64_t)it.y * rd.row_stride, rd.slot_off,
                                  rd.slot_len, nullptr, nullptr, nullptr, lds, ig, a.geom + it.roi);
}

// ------------------------------------------------------------ launch helpers
template <typename VT, int D0, int ND, bool FAST, bool CHAIN = false, int NWV = 4>
hipError_t launch_one(const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    auto k = slice_kernel<VT, D0, ND, FAST, CHAIN, NWV>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    const int nw = CHAIN ? CH_WAVES : NWV;
    hipLaunchKernelGGL(k, dim3(items), dim3(nw * 64), lds, st, a);
    return hipGetLastError();
}

template <typename VT, int D0, bool FAST, bool CHAIN = false, int NWV = 4>
hipError_t launch_nd(int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st) {
    switch (nd) {
        case 1: return launch_one<VT, D0, 1, FAST, CHAIN, NWV>(a, items, lds, st);
        case 2: return launch_one<VT, D0, 2, FAST, CHAIN, NWV>(a, items, lds, st);
        case 3: return launch_one<VT, D0, 3, FAST, CHAIN, NWV>(a, items, lds, st);
        case 4: return launch_one<VT, D0, 4, FAST, CHAIN, NWV>(a, items, lds, st);
        case 5: return launch_one<VT, D0, 5, FAST, CHAIN, NWV>(a, items, lds, st);
        default:
            if constexpr (D0 == 0) {
                if (nd == 6) return launch_one<VT, D0, 6, FAST, CHAIN, NWV>(a, items, lds, st);
                if (nd == 7) return launch_one<VT, D0, 7, FAST, CHAIN, NWV>(a, items, lds, st);
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
    hipLaunchKernelGGL(k, dim3(items), dim3(BATCH_WAVES * 64), lds, st, a);
    return hipGetLastError();
}

}  // namespace dpm
