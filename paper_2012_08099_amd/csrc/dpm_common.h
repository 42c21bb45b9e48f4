// Shared host/device definitions of the projection family, launch geometry and the
// per-workgroup LDS layout of the projection kernel.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define DPM_HD __host__ __device__ __forceinline__
#else
#define DPM_HD inline
#endif

namespace dpm {

constexpr int KMAX = 16;
constexpr int NDIR_MAX = KMAX + 1;

// The projection family.  Image d sums V over alpha_d x + beta_d z = const (eq. 4).
// (1,0) and (0,1) are the axis projections of eqs. (5) and (6), (1,1) and (1,-1)
// the +-pi/4 projections of eqs. (8) and (9); the others are the further aligned
// projections (arctan 1/2, arctan 2, ...) listed after eq. (9).  Order k needs the
// first k+1 of them: every direction lies in the xz-plane, so one image row per y is
// complete inside the workgroup that owns that y.
__host__ __device__ constexpr int dir_alpha(int d) {
    return d == 0 ? 1 : d == 1 ? 0 : d == 2 ? 1 : d == 3 ? 1 : d == 4 ? 2 : d == 5 ? 2
         : d == 6 ? 1 : d == 7 ? 1 : d == 8 ? 3 : d == 9 ? 3 : d == 10 ? 1 : d == 11 ? 1
         : d == 12 ? 3 : d == 13 ? 3 : d == 14 ? 2 : d == 15 ? 2 : 1;
}
__host__ __device__ constexpr int dir_beta(int d) {
    return d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 1 : d == 3 ? -1 : d == 4 ? 1 : d == 5 ? -1
         : d == 6 ? 2 : d == 7 ? -2 : d == 8 ? 1 : d == 9 ? -1 : d == 10 ? 3 : d == 11 ? -3
         : d == 12 ? 2 : d == 13 ? -2 : d == 14 ? 3 : d == 15 ? -3 : 4;
}
__host__ __device__ constexpr int iabs_c(int v) { return v < 0 ? -v : v; }
__host__ __device__ constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

// Voxels per lane along x: one 16-byte load (uint16) or 8-byte load (uint8).
__host__ __device__ constexpr int lane_voxels(int elem) { return 8; }

// LDS padding period of a row accumulator: one pad dword per PP bins.  Lanes of a
// sub-row flush windows at a stride of alpha*G bins; the padded stride is odd
// (conflict-free) except for alpha = 2 with G = 8, which stays two-way so that its
// window blocks stay 8 rows long.
__host__ __device__ constexpr int dir_pp(int d, int G) { return (G == 4 && dir_alpha(d) == 2) ? 8 : G; }
// Rows per window block: a multiple T of PP / gcd(beta, PP), so that beta*T = 0 mod PP,
// every block base is PP-aligned relative to the row origin and flush offsets are
// compile-time -- here the whole unit of group_rows() = 8 rows (PP = 8), so a window is
// flushed once per unit.
__host__ __device__ constexpr int dir_td(int d, int G) {
    return dir_beta(d) == 0 ? 1 : 8;
}
// Window slots of one lane per block: alpha (G-1) + |beta| (T_d - 1) + 1.
__host__ __device__ constexpr int dir_slots(int d, int G) {
    return dir_alpha(d) * (G - 1) + iabs_c(dir_beta(d)) * (dir_td(d, G) - 1) + 1;
}
// Slot shift that keeps slots non-negative for beta < 0.
__host__ __device__ constexpr int dir_shift(int d, int G) {
    return dir_beta(d) < 0 ? iabs_c(dir_beta(d)) * (dir_td(d, G) - 1) : 0;
}

// Direction groups: each is one launch of the projection kernel (register budget).
constexpr int NGROUP = 3;
__host__ __device__ constexpr int group_begin(int g) { return g == 0 ? 0 : g == 1 ? 7 : 12; }
__host__ __device__ constexpr int group_end(int g) { return g == 0 ? 7 : g == 1 ? 12 : 17; }
// Rows per chunk (unit of work and of double buffering): a multiple of every T_d.
__host__ __device__ constexpr int group_rows(int g) { return 8; }
static_assert(group_rows(0) == 8 && dir_pp(0, 8) == 8, "window blocks are one unit of 8 rows");
// Copies of the (0,1) row accumulator: 8-lane groups g and g+4 of a wave share copy g % 4.
constexpr int YZ_COPIES = 4;
// Dwords after the row accumulators that absorb the (0,1) adds of the lanes that hold
// no group sum (lane + row offset < 96), so that add needs no branch.
constexpr int LDS_SINK = 96;
constexpr int ZALIGN = 16;  // z-split boundaries are multiples of every group's chunk

__host__ __device__ constexpr int n_moments(int K) { return (K + 1) * (K + 2) * (K + 3) / 6; }
// graded position of (p, q, r)
__host__ __device__ constexpr int moment_index(int p, int q, int r) {
    return (p + q + r) * (p + q + r + 1) * (p + q + r + 2) / 6 + (q + r) * (q + r + 1) / 2 + r;
}
// Pairs (d, k) with d <= k <= K, ordered by d then k; image d only feeds degrees >= d.
__host__ __device__ constexpr int pair_index(int K, int d, int k) {
    return d * (K + 1) - d * (d - 1) / 2 + (k - d);
}
__host__ __device__ constexpr int n_pairs(int K) { return (K + 1) * (K + 2) / 2; }

// Geometry of one work item (one y-slice, rows [zs, ze)) for one direction group.
// Everything the projection kernel needs to place LDS rows and to enumerate the
// power-sum jobs.  Computed identically on host (sizes) and device (per item).
constexpr int MAXSEG = 2 * 7;  // per group: <= 7 directions, each split at its origin

struct DirGeom {
    int32_t lo;      // bin of LDS index 0
    int32_t o;       // image column of the true origin (|beta| (N-1) if beta < 0)
    int32_t rb_lo;   // smallest bin that can hold voxels of this item
    int32_t rb_hi;   // largest such bin
    int32_t lds_off; // dword offset of the row accumulator
    int32_t lds_len; // dwords (padded)
};

// Power-sum segments: each direction's row split at its origin into a negative side
// (slot 2i, coordinate a = o - bin) and a non-negative side (slot 2i+1, a = bin - o).
// An empty side has alo > ahi.
struct ItemGeom {
    DirGeom dir[7];
    int32_t seg_alo[MAXSEG];
    int32_t seg_ahi[MAXSEG];
    int32_t yz_off;     // dword offset of the (0,1) accumulator copies
    int32_t yz_stride;  // dwords between copies (odd)
    int32_t n_chunks;   // chunks of group_rows() rows in [zs, ze)
    int32_t lds_dwords; // projection part of LDS (row accumulators + sink)
};

DPM_HD int64_t padded(int64_t u, int pp) { return u + u / pp; }

// Geometry of direction i of group g for rows [zs, ze) and G voxels per lane (no LDS
// offset yet).
DPM_HD void dir_geometry(int g, int i, int G, int64_t L, int64_t N, int64_t zs, int64_t ze, DirGeom &dg,
                         int32_t &alo_neg, int32_t &ahi_neg, int32_t &alo_pos, int32_t &ahi_pos) {
    const int T = group_rows(g);
    const int64_t Xp = (L + G - 1) / G * G;    // padded x extent
    const int64_t nch = (ze - zs + T - 1) / T;
    const int64_t zlast = zs + nch * T - 1;    // last row any window may cover
    const int d = group_begin(g) + i;
    const int64_t a = dir_alpha(d), b = dir_beta(d);
    const int64_t o = b < 0 ? -b * (N - 1) : 0;
    int64_t bmin, bmax, rlo, rhi;
    if (d == 1) {  // (0,1): bin = z
        bmin = zs;
        bmax = zlast;
        rlo = zs;
        rhi = ze - 1;
    } else if (b >= 0) {
        bmin = b * zs + o;
        bmax = a * (Xp - 1) + b * zlast + o;
        rlo = b * zs + o;
        rhi = a * (L - 1) + b * (ze - 1) + o;
    } else {
        bmin = b * zlast + o;
        bmax = a * (Xp - 1) + b * zs + o;
        rlo = b * (ze - 1) + o;
        rhi = a * (L - 1) + b * zs + o;
    }
    dg.o = (int32_t)o;
    dg.lo = (int32_t)bmin;
    dg.rb_lo = (int32_t)rlo;
    dg.rb_hi = (int32_t)rhi;
    dg.lds_len = d == 1 ? (int32_t)(YZ_COPIES * ((nch * T) | 1)) : (int32_t)(padded(bmax - bmin, dir_pp(d, G)) + 1);
    // sides: negative [rlo, min(rhi, o-1)], non-negative [max(rlo, o), rhi]
    const int64_t n1 = rhi < o - 1 ? rhi : o - 1;
    const int64_t p0 = rlo > o ? rlo : o;
    alo_neg = (int32_t)(o - n1);
    ahi_neg = (int32_t)(o - rlo);
    if (n1 < rlo) {
        alo_neg = 1;
        ahi_neg = 0;
    }
    alo_pos = (int32_t)(p0 - o);
    ahi_pos = (int32_t)(rhi - o);
    if (rhi < p0) {
        alo_pos = 1;
        ahi_pos = 0;
    }
}

// Whole-item geometry (host, and device for batched items).
DPM_HD void item_geometry(int g, int nd, int G, int64_t L, int64_t N, int64_t zs, int64_t ze, ItemGeom &ig) {
    const int T = group_rows(g);
    const int64_t nch = (ze - zs + T - 1) / T;
    int32_t off = 0;
    ig.n_chunks = (int32_t)nch;
    ig.yz_off = -1;
    ig.yz_stride = 0;
    for (int i = 0; i < 7; ++i) {
        if (i >= nd) {
            ig.seg_alo[2 * i] = ig.seg_alo[2 * i + 1] = 1;
            ig.seg_ahi[2 * i] = ig.seg_ahi[2 * i + 1] = 0;
            continue;
        }
        DirGeom &dg = ig.dir[i];
        dir_geometry(g, i, G, L, N, zs, ze, dg, ig.seg_alo[2 * i], ig.seg_ahi[2 * i], ig.seg_alo[2 * i + 1],
                     ig.seg_ahi[2 * i + 1]);
        dg.lds_off = off;
        if (group_begin(g) + i == 1) {
            ig.yz_off = off;
            ig.yz_stride = dg.lds_len / YZ_COPIES;
        }
        off += dg.lds_len;
    }
    ig.lds_dwords = off + LDS_SINK;
}

// Fused batched kernel (one workgroup per (ROI, block of BK_YB y-slices)): LDS holds
//   store:   for every non-empty slot s, BK_YB rows of bk_plen(s) row values (2 or 4
//            bytes each) at a stride of bk_rstride() values (16 bytes more than a row,
//            so the 16 rows of a matrix-core tile fall in different banks), slot after
//            slot, 16-byte aligned in total;
//   scratch: BK_WAVES regions of bk_scratch_dwords() dwords, one per wave: the
//            projection's row accumulators of the spw slices the wave projects
//            together (bk_slice_dwords() each), later the wave's 4 x 256 limb-pair table.
constexpr int BK_WAVES = 4;
constexpr int BK_YB = 16;
constexpr int BK_SCR_MIN = 1024;
// values per slice of slot s: the side's extent 0 .. ahi rounded up to 16 (0 if empty)
DPM_HD int32_t bk_plen(const ItemGeom &ig, int s) {
    return ig.seg_ahi[s] >= ig.seg_alo[s] ? (ig.seg_ahi[s] + 16) / 16 * 16 : 0;
}
DPM_HD int32_t bk_rstride(int32_t plen, int rowbytes) { return plen ? plen + 16 / rowbytes : 0; }
DPM_HD int32_t bk_store_bytes(const ItemGeom &ig, int nd, int rowbytes) {
    int32_t tot = 0;
    for (int s = 0; s < 2 * nd; ++s) tot += BK_YB * bk_rstride(bk_plen(ig, s), rowbytes);
    return (tot * rowbytes + 15) / 16 * 16;
}
DPM_HD int32_t bk_slice_dwords(const ItemGeom &ig) { return (ig.lds_dwords + 3) / 4 * 4; }
DPM_HD int32_t bk_scratch_dwords(const ItemGeom &ig, int spw) {
    const int32_t w = spw * bk_slice_dwords(ig);
    return w > BK_SCR_MIN ? w : BK_SCR_MIN;
}
DPM_HD int64_t bk_lds_bytes(const ItemGeom &ig, int nd, int rowbytes, int spw) {
    return (int64_t)bk_store_bytes(ig, nd, rowbytes) + (int64_t)BK_WAVES * bk_scratch_dwords(ig, spw) * 4;
}

// Row storage of the power-sum input: segment slot s of every item holds `len` int32
// values for a = 0 .. len-1 (zero outside the item's [alo, ahi]); len is a multiple of
// 64 and equal for all items of a launch.
DPM_HD int32_t round64(int64_t v) { return (int32_t)((v + 63) / 64 * 64); }

}  // namespace dpm
