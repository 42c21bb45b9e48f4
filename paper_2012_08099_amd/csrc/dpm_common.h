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
constexpr int G = 8;

// LDS padding period of a sheared row accumulator: one pad dword per PP bins makes
// the flush of lane windows (lane stride alpha*G bins) conflict-free.
__host__ __device__ constexpr int dir_pp(int d) {
    return (dir_alpha(d) == 2 && iabs_c(dir_beta(d)) != 3) ? 16 : 8;
}
// Rows per window block: the smallest T with beta*T = 0 mod PP, so every block base
// is PP-aligned relative to the row origin and flush offsets are compile-time.
__host__ __device__ constexpr int dir_td(int d) {
    return dir_beta(d) == 0 ? 1 : dir_pp(d) / gcd_c(iabs_c(dir_beta(d)), dir_pp(d));
}
// Window slots of one lane per block: alpha (G-1) + |beta| (T_d - 1) + 1.
__host__ __device__ constexpr int dir_slots(int d) {
    return dir_alpha(d) * (G - 1) + iabs_c(dir_beta(d)) * (dir_td(d) - 1) + 1;
}
// Slot shift that keeps slots non-negative for beta < 0.
__host__ __device__ constexpr int dir_shift(int d) {
    return dir_beta(d) < 0 ? iabs_c(dir_beta(d)) * (dir_td(d) - 1) : 0;
}

// Direction groups: each is one launch of the projection kernel (register budget).
constexpr int NGROUP = 3;
__host__ __device__ constexpr int group_begin(int g) { return g == 0 ? 0 : g == 1 ? 7 : 12; }
__host__ __device__ constexpr int group_end(int g) { return g == 0 ? 7 : g == 1 ? 12 : 17; }
// Rows per chunk of a group = lcm of its T_d (16 for group 0, 8 otherwise).
__host__ __device__ constexpr int group_rows(int g) { return g == 0 ? 16 : 8; }
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
    int64_t lo;      // bin of LDS index 0
    int64_t o;       // image column of the true origin (|beta| (N-1) if beta < 0)
    int64_t rb_lo;   // smallest bin that can hold voxels of this item
    int64_t rb_hi;   // largest such bin
    int32_t lds_off; // dword offset of the row accumulator
    int32_t lds_len; // dwords (padded)
};

struct ItemGeom {
    DirGeom dir[7];
    int32_t yz_off;     // dword offset of the (0,1) accumulator copies
    int32_t yz_stride;  // dwords between copies (odd)
    int32_t n_chunks;   // chunks of group_rows() rows in [zs, ze)
    int32_t lds_dwords; // projection part of LDS
};

DPM_HD int64_t padded(int64_t u, int pp) { return u + u / pp; }

// xlanes = lanes that hold voxels per row = ceil(L / G)
DPM_HD void item_geometry(int g, int nd, int64_t L, int64_t N, int64_t zs, int64_t ze,
                          ItemGeom &ig) {
    const int T = group_rows(g);
    const int64_t xl = (L + G - 1) / G;
    const int64_t Xp = xl * G;                 // padded x extent
    const int64_t nch = (ze - zs + T - 1) / T;
    const int64_t zlast = zs + nch * T - 1;    // last row any window may cover
    int32_t off = 0;
    ig.n_chunks = (int32_t)nch;
    ig.yz_off = -1;
    ig.yz_stride = 0;
    for (int i = 0; i < nd; ++i) {
        const int d = group_begin(g) + i;
        const int64_t a = dir_alpha(d), b = dir_beta(d);
        DirGeom &dg = ig.dir[i];
        dg.o = b < 0 ? -b * (N - 1) : 0;
        if (d == 1) {  // (0,1): bin = z; 8 copies, one per 8-lane group of a wave
            dg.lo = zs;
            dg.rb_lo = zs;
            dg.rb_hi = ze - 1;
            int32_t stride = (int32_t)(nch * T) | 1;
            ig.yz_off = off;
            ig.yz_stride = stride;
            dg.lds_off = off;
            dg.lds_len = 8 * stride;
            off += dg.lds_len;
            continue;
        }
        int64_t bmin, bmax;
        if (b >= 0) {
            bmin = b * zs + dg.o;
            bmax = a * (Xp - 1) + b * zlast + dg.o;
            dg.rb_lo = b * zs + dg.o;
            dg.rb_hi = a * (L - 1) + b * (ze - 1) + dg.o;
        } else {
            bmin = b * zlast + dg.o;
            bmax = a * (Xp - 1) + b * zs + dg.o;
            dg.rb_lo = b * (ze - 1) + dg.o;
            dg.rb_hi = a * (L - 1) + b * zs + dg.o;
        }
        dg.lo = bmin;
        const int pp = dir_pp(d);
        dg.lds_off = off;
        dg.lds_len = (int32_t)(padded(bmax - bmin, pp) + 1);
        off += dg.lds_len;
    }
    ig.lds_dwords = off;
}

// Power-sum jobs: each direction's real bin range split at its origin into a
// negative side (coordinate a = o - b) and a non-negative side (a = b - o), each cut
// into pieces of at most `jobbins` bins.
DPM_HD bool seg_range(const DirGeom &dg, int side, int64_t &b0, int64_t &b1) {
    if (side == 0) {
        b0 = dg.rb_lo;
        b1 = dg.rb_hi < dg.o - 1 ? dg.rb_hi : dg.o - 1;
    } else {
        b0 = dg.rb_lo > dg.o ? dg.rb_lo : dg.o;
        b1 = dg.rb_hi;
    }
    return b1 >= b0;
}

DPM_HD int count_jobs(const ItemGeom &ig, int nd, int jobbins) {
    int n = 0;
    for (int i = 0; i < nd; ++i)
        for (int side = 0; side < 2; ++side) {
            int64_t b0, b1;
            if (seg_range(ig.dir[i], side, b0, b1)) n += (int)((b1 - b0 + jobbins) / jobbins);
        }
    return n;
}

}  // namespace dpm
