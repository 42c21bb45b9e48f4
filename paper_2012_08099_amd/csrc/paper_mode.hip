// Paper-literal mode (Sections 3.1, 3.2 and 5, orders <= 4) and the 1D-integral route for
// the 2D moments of any set of projection images.  Interfaces: paper.h.
//
// 1. paper_project_kernel: one pass over the volume.  A workgroup owns a tile of PP_BY
//    rows of y x PP_BZ planes of z x PP_XT voxels of x; wave w walks PP_ZW planes of the
//    tile for every y of it, lane l owns 8 consecutive x.  Per voxel: XY, ZX and the two
//    diagonal images accumulate in registers (ZX over the y loop, the others over the
//    wave's planes), the row sum for YZ too; XY and X+-Z rows meet in LDS (one add per
//    register slot per y), ZX and YZ go to their partial planes directly.  ZX needs all y
//    and XY / X+-Z all z, so no tile holds a whole image: the tiles' partial images are
//    written out and
// 2. paper_reduce_kernel sums them in a fixed order into the five images.
// 3. drt_tile_kernel: the 1D integrals of Section 5 (Vert, Horiz, Diag, AntiDiag, X2Y) of
//    one tile of an image by additions only, then their 1D moments.
// 4. paper_finish_kernel / drt_to_part_kernel: 1D moments -> 2D moments (exact inverse of
//    the small system), then eqs. 10-16 (paper mode) or the tile partials of the family
//    recombination.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dpm_common.h"
#include "mw.h"
#include "paper.h"

namespace dpm {

namespace {

__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) v += __shfl_xor(v, s, 64);
    return v;
}

__device__ __forceinline__ __int128 wave_sum_i128(__int128 v) {
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
        const unsigned long long olo = __shfl_xor(lo, s, 64), ohi = __shfl_xor(hi, s, 64);
        v += (__int128)(((unsigned __int128)ohi << 64) | olo);
    }
    return v;
}

// 8 voxels of row (y, z) from x = xl on, packed as they are in memory (4 dwords for
// uint16, 2 for uint8), zeros where outside the volume.  FAST: L is a multiple of 8 and
// rows are aligned to one lane's load (16 bytes uint16, 8 bytes uint8).
template <typename T, bool FAST>
__device__ __forceinline__ void load8(const PaperProjArgs &a, int64_t y, int64_t z, int64_t xl, uint32_t (&w)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = 0u;
    if (z >= a.N || xl >= a.L) return;
    const T *row = reinterpret_cast<const T *>(a.vol) + (z * a.M + y) * a.L;
    if (FAST) {
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        if (sizeof(T) == 2) {
            const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(row + xl));
            w[0] = q.x;
            w[1] = q.y;
            w[2] = q.z;
            w[3] = q.w;
        } else {
            const u32x2 q = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(row + xl));
            w[0] = q.x;
            w[1] = q.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (xl + k < a.L) {
                const uint32_t e = row[xl + k];
                if (sizeof(T) == 2) w[k / 2] |= e << (16 * (k % 2));
                else w[k / 4] |= e << (8 * (k % 4));
            }
    }
}

template <typename T>
__device__ __forceinline__ int32_t voxel_of(const uint32_t (&w)[4], int k) {
    if (sizeof(T) == 2) return (int32_t)((w[k / 2] >> (16 * (k % 2))) & 0xffffu);
    return (int32_t)((w[k / 4] >> (8 * (k % 4))) & 0xffu);
}

// The 8 values r[0..7] of every lane summed over the wave: lane 8 z (z < 8) ends up
// holding the sum for z.  Halving exchanges: 4 + 2 + 1 shuffles pair up the values, 3
// more finish the sums (10 shuffles instead of 8 full reductions).
__device__ __forceinline__ int32_t wave_sum8(const int32_t (&r)[8], int lane) {
    int32_t a4[4], a2[2];
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t keep = b5 ? r[q + 4] : r[q], send = b5 ? r[q] : r[q + 4];
        a4[q] = keep + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int32_t keep = b4 ? a4[q + 2] : a4[q], send = b4 ? a4[q] : a4[q + 2];
        a2[q] = keep + __shfl_xor(send, 16, 64);
    }
    int32_t a1 = (b3 ? a2[1] : a2[0]) + __shfl_xor(b3 ? a2[0] : a2[1], 8, 64);
    a1 += __shfl_xor(a1, 4, 64);
    a1 += __shfl_xor(a1, 2, 64);
    a1 += __shfl_xor(a1, 1, 64);
    return a1;  // lane l: value index (l >> 3) & 7, when l % 8 == 0
}

template <typename T, bool FAST>
__global__ void __launch_bounds__(PP_WAVES * 64) paper_project_kernel(PaperProjArgs a) {
    __shared__ int32_t s_xy[PP_BY][PP_XT];
    __shared__ int32_t s_xpz[PP_BY][PP_DW];
    __shared__ int32_t s_xmz[PP_BY][PP_DW];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int xt = blockIdx.x % a.nxt;
    const int zb = (blockIdx.x / a.nxt) % a.nzb;
    const int yb = blockIdx.x / (a.nxt * a.nzb);
    const int64_t x0 = (int64_t)xt * PP_XT, y0 = (int64_t)yb * PP_BY, z0 = (int64_t)zb * PP_BZ;
    const int64_t zw0 = z0 + w * PP_ZW, xl = x0 + 8 * lane;
    const bool diag = a.nimg >= 4, anti = a.nimg >= 5;
    for (int i = tid; i < PP_BY * PP_XT; i += PP_WAVES * 64) (&s_xy[0][0])[i] = 0;
    for (int i = tid; i < PP_BY * PP_DW; i += PP_WAVES * 64) {
        (&s_xpz[0][0])[i] = 0;
        (&s_xmz[0][0])[i] = 0;
    }
    __syncthreads();

    int32_t zx[PP_ZW][8];
#pragma unroll
    for (int zz = 0; zz < PP_ZW; ++zz)
#pragma unroll
        for (int k = 0; k < 8; ++k) zx[zz][k] = 0;

    for (int yy = 0; yy < PP_BY; ++yy) {
        const int64_t y = y0 + yy;
        if (y >= a.M) break;  // the same for the whole workgroup
        uint32_t v[PP_ZW][4];
#pragma unroll
        for (int zz = 0; zz < PP_ZW; ++zz) load8<T, FAST>(a, y, zw0 + zz, xl, v[zz]);
        int32_t xy[8], wp[8 + PP_ZW - 1], wm[8 + PP_ZW - 1], rs[PP_ZW];
#pragma unroll
        for (int k = 0; k < 8; ++k) xy[k] = 0;
#pragma unroll
        for (int s = 0; s < 8 + PP_ZW - 1; ++s) wp[s] = wm[s] = 0;
#pragma unroll
        for (int zz = 0; zz < PP_ZW; ++zz) {
            int32_t s = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int32_t e = voxel_of<T>(v[zz], k);
                xy[k] += e;                  // I(x, y), eq. 5: summed over z
                zx[zz][k] += e;              // I(z, x), eq. 7: summed over y
                s += e;                      // I(y, z), eq. 6: summed over x
                wp[k + zz] += e;             // I(x + z, y), eq. 8
                wm[k - zz + PP_ZW - 1] += e; // I(x - z, y), eq. 9
            }
            rs[zz] = s;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (xy[k]) atomicAdd(&s_xy[yy][8 * lane + k], xy[k]);
        if (diag) {
            const int bp = 8 * lane + w * PP_ZW;
#pragma unroll
            for (int s = 0; s < 8 + PP_ZW - 1; ++s)
                if (wp[s]) atomicAdd(&s_xpz[yy][bp + s], wp[s]);
        }
        if (anti) {
            const int bm = 8 * lane - w * PP_ZW + PP_BZ - PP_ZW;
#pragma unroll
            for (int s = 0; s < 8 + PP_ZW - 1; ++s)
                if (wm[s]) atomicAdd(&s_xmz[yy][bm + s], wm[s]);
        }
        {
            static_assert(PP_ZW == 8, "wave_sum8 reduces 8 planes");
            const int32_t t = wave_sum8(rs, lane);
            const int64_t z = zw0 + (lane >> 3);
            if ((lane & 7) == 0 && z < a.N) a.yz[((int64_t)xt * a.N + z) * a.M + y] = t;
        }
    }
    // ZX partial of this y-block: [yb][z][x], 8 consecutive x per lane
#pragma unroll
    for (int zz = 0; zz < PP_ZW; ++zz) {
        const int64_t z = zw0 + zz;
        if (z >= a.N) break;
        int32_t *dst = a.zx + ((int64_t)yb * a.N + z) * a.L;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (xl + k < a.L) dst[xl + k] = zx[zz][k];
    }
    __syncthreads();
    // XY and X+-Z partial rows of this z-block
    const int64_t ylim = a.M - y0 < PP_BY ? a.M - y0 : PP_BY;
    for (int i = tid; i < ylim * PP_XT; i += PP_WAVES * 64) {
        const int yy = i / PP_XT, xx = i % PP_XT;
        if (x0 + xx < a.L) a.xy[((int64_t)zb * a.M + y0 + yy) * a.L + x0 + xx] = s_xy[yy][xx];
    }
    for (int i = tid; diag && i < ylim * PP_DW; i += PP_WAVES * 64) {
        const int yy = i / PP_DW, s = i % PP_DW;
        const int64_t r = (((int64_t)zb * a.nxt + xt) * a.M + y0 + yy) * PP_DW + s;
        a.xpz[r] = s_xpz[yy][s];
        if (anti) a.xmz[r] = s_xmz[yy][s];
    }
}

// One thread per image pixel; partials summed in ascending block order.
__global__ void __launch_bounds__(256) paper_reduce_kernel(PaperReduceArgs a) {
    const int e = blockIdx.y, tid = threadIdx.x;
    if (e >= a.nimg) return;
    const int64_t L = a.L, M = a.M, N = a.N, DW = PP_DW;
    if (e == 2) {
        // ZX[x][z] = sum over y-blocks of the [z][x] partials: reads along x, one
        // transposed store per element
        const int64_t el = (int64_t)blockIdx.x * 256 + tid;
        if (el >= N * L) return;
        const int64_t z = el / L, x = el % L;
        int32_t s = 0;
        for (int yb = 0; yb < a.nyb; ++yb) s += a.zx[((int64_t)yb * N + z) * L + x];
        a.img[2][x * N + z] = s;  // [j = x][i = z]
        return;
    }
    const int64_t W = e == 0 ? L : e == 1 ? M : L + N - 1;
    const int64_t H = e == 1 ? N : M;
    const int64_t pix = (int64_t)blockIdx.x * 256 + tid;
    if (pix >= W * H) return;
    const int64_t j = pix / W, i = pix % W;
    int32_t s = 0;
    if (e == 0) {
        for (int zb = 0; zb < a.nzb; ++zb) s += a.xy[((int64_t)zb * M + j) * L + i];
    } else if (e == 1) {
        for (int xt = 0; xt < a.nxt; ++xt) s += a.yz[((int64_t)xt * N + j) * M + i];
    } else {
        // bin of (zb, xt): column i = base + s_local, base = x0 + z0 (X+Z) or x0 - z0 + N - BZ (X-Z)
        for (int zb = 0; zb < a.nzb; ++zb) {
            const int64_t z0 = (int64_t)zb * PP_BZ;
            const int64_t c = e == 3 ? i - z0 : i + z0 - N + PP_BZ;  // = x0 + s_local
            int64_t xlo = c - (DW - 1);
            xlo = xlo <= 0 ? 0 : (xlo + PP_XT - 1) / PP_XT;
            int64_t xhi = c < 0 ? -1 : c / PP_XT;
            if (xhi > a.nxt - 1) xhi = a.nxt - 1;
            for (int64_t xt = xlo; xt <= xhi; ++xt) {
                const int64_t sl = c - xt * PP_XT;
                const int32_t *src = e == 3 ? a.xpz : a.xmz;
                s += src[(((int64_t)zb * a.nxt + xt) * M + j) * DW + sl];
            }
        }
    }
    a.img[e][pix] = s;
}

// Section 5's 1D integrals of one tile of one image, then their 1D moments.
__global__ void __launch_bounds__(256) drt_tile_kernel(DrtArgs a) {
    __shared__ long long s_diag[DRT_IB + DRT_RB - 1], s_anti[DRT_IB + DRT_RB - 1], s_x2y[DRT_IB + 2 * DRT_RB - 1];
    __shared__ long long s_hor[DRT_RB];
    __shared__ __int128 s_red[4][DRT_NDIR][DRT_KMAX + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int tile = blockIdx.x;
    int e = 0;
    while (e + 1 < a.nimg && tile >= a.im[e + 1].tile0) ++e;
    const DrtImage im = a.im[e];
    const int local = tile - im.tile0;
    const int64_t i0 = (int64_t)(local % im.tiles_i) * DRT_IB, j0 = (int64_t)(local / im.tiles_i) * DRT_RB;
    for (int b = tid; b < DRT_IB + 2 * DRT_RB - 1; b += 256) {
        if (b < DRT_IB + DRT_RB - 1) s_diag[b] = s_anti[b] = 0;
        s_x2y[b] = 0;
        if (b < DRT_RB) s_hor[b] = 0;
    }
    __syncthreads();
    const int64_t i = i0 + tid;
    // all rows of the tile in flight at once
    int32_t col[DRT_RB];
#pragma unroll
    for (int jj = 0; jj < DRT_RB; ++jj) {
        const int64_t j = j0 + jj;
        col[jj] = (i < im.W && j < im.H) ? im.img[j * im.W + i] : 0;
    }
    long long vert = 0;
#pragma unroll
    for (int jj = 0; jj < DRT_RB; ++jj) {
        if (j0 + jj >= im.H) break;  // the same for the whole workgroup
        const long long v = col[jj];
        vert += v;                                       // Vert[i]
        const long long hs = wave_sum_i64(v);
        if (lane == 0 && hs) atomicAdd((unsigned long long *)&s_hor[jj], (unsigned long long)hs);  // Horiz[j]
        if (v) {
            if (a.ndir > 2) atomicAdd((unsigned long long *)&s_diag[tid + jj], (unsigned long long)v);  // Diag[i + j]
            if (a.ndir > 3)
                atomicAdd((unsigned long long *)&s_anti[tid - jj + DRT_RB - 1], (unsigned long long)v);  // AntiDiag[i - j]
            if (a.ndir > 4) atomicAdd((unsigned long long *)&s_x2y[tid + 2 * jj], (unsigned long long)v);  // X2Y[i + 2j]
        }
    }
    __syncthreads();
    __int128 acc[DRT_NDIR][DRT_KMAX + 1];
#pragma unroll
    for (int g = 0; g < DRT_NDIR; ++g)
#pragma unroll
        for (int n = 0; n <= DRT_KMAX; ++n) acc[g][n] = 0;
    const int K = a.K;
    auto addm = [&](int g, int64_t t, long long P) {
        if (!P) return;
        int64_t tp = 1;  // t^n, |t| < 2^15 (checked by the planner)
#pragma unroll
        for (int n = 0; n <= DRT_KMAX; ++n) {
            if (n <= K) acc[g][n] += (__int128)tp * P;
            if (n < DRT_KMAX) tp *= t;
        }
    };
    const int64_t io = im.io;
    if (i < im.W) addm(0, i - io, vert);                                     // t = i
    if (tid < DRT_RB) addm(1, j0 + tid, s_hor[tid]);                         // t = j
    for (int b = tid; b < DRT_IB + DRT_RB - 1; b += 256) {
        if (a.ndir > 2) addm(2, b + i0 + j0 - io, s_diag[b]);                // t = i + j
        if (a.ndir > 3) addm(3, b + i0 - j0 - (DRT_RB - 1) - io, s_anti[b]);  // t = i - j
    }
    for (int b = tid; a.ndir > 4 && b < DRT_IB + 2 * DRT_RB - 1; b += 256)
        addm(4, b + i0 + 2 * j0 - io, s_x2y[b]);                             // t = i + 2j
#pragma unroll
    for (int g = 0; g < DRT_NDIR; ++g)
#pragma unroll
        for (int n = 0; n <= DRT_KMAX; ++n) {
            const __int128 s = wave_sum_i128(acc[g][n]);
            if (lane == 0) s_red[wv][g][n] = s;
        }
    __syncthreads();
    if (tid < DRT_NDIR * (DRT_KMAX + 1)) {
        const int g = tid / (DRT_KMAX + 1), n = tid % (DRT_KMAX + 1);
        a.part1d[((int64_t)tile * DRT_NDIR + g) * (DRT_KMAX + 1) + n] =
            s_red[0][g][n] + s_red[1][g][n] + s_red[2][g][n] + s_red[3][g][n];
    }
}

__global__ void __launch_bounds__(64) drt_sum_kernel(DrtSumArgs a) {
    const int e = blockIdx.x, gn = blockIdx.y, lane = threadIdx.x;
    constexpr int NV = DRT_NDIR * (DRT_KMAX + 1);
    __int128 s = 0;
    for (int t = a.tile0[e] + lane; t < a.tile0[e + 1]; t += 64) s += a.part1d[(int64_t)t * NV + gn];
    s = wave_sum_i128(s);
    if (lane == 0) a.m1d[(int64_t)e * NV + gn] = s;
}

__device__ void load_m1d(const __int128 *m1d, int nimg, __int128 (*m)[DRT_NDIR][DRT_KMAX + 1]) {
    constexpr int NV = DRT_NDIR * (DRT_KMAX + 1);
    for (int v = threadIdx.x; v < nimg * NV; v += blockDim.x)
        m[v / NV][(v % NV) / (DRT_KMAX + 1)][v % (DRT_KMAX + 1)] = m1d[v];
}

// 2D moment M_{p,q} of an image from its 1D moments (exact).
__device__ __int128 moment2d(const DrtSolve &sv, const __int128 (&m)[DRT_NDIR][DRT_KMAX + 1], int p, int q) {
    const int n = p + q;
    __int128 num = 0;
    for (int g = 0; g <= n; ++g) num += (__int128)sv.num[n][p][g] * m[g][n];
    num >>= sv.shift[n][p];  // arithmetic: exact, the sum is a multiple of den
    const unsigned __int128 inv = ((unsigned __int128)sv.inv_hi[n][p] << 64) | sv.inv_lo[n][p];
    return (__int128)((unsigned __int128)num * inv);
}

__device__ __forceinline__ void put_i128(void *exact, double *fp64, int idx, __int128 v) {
    if (exact) {
        uint64_t *o = reinterpret_cast<uint64_t *>(exact) + 2 * idx;
        o[0] = (uint64_t)v;
        o[1] = (uint64_t)((unsigned __int128)v >> 64);
    }
    if (fp64) {
        mw::Int<4> w;
        const unsigned __int128 u = (unsigned __int128)v;
#pragma unroll
        for (int l = 0; l < 4; ++l) w.w[l] = (uint32_t)(u >> (32 * l));
        fp64[idx] = mw::to_double(w);
    }
}

__global__ void __launch_bounds__(256) paper_finish_kernel(PaperFinishArgs a) {
    __shared__ __int128 m[PAPER_NIMG][DRT_NDIR][DRT_KMAX + 1];
    load_m1d(a.m1d, a.nimg, m);
    __syncthreads();
    const int idx = threadIdx.x;
    if (idx >= n_moments(a.K)) return;
    // (p, q, r) of graded index idx
    int n = 0;
    while (n_moments(n) <= idx) ++n;
    int rem = idx - (n_moments(n) - (n + 1) * (n + 2) / 2), p = n;
    while (rem >= n - p + 1) {
        rem -= n - p + 1;
        --p;
    }
    const int q = n - p - rem, r = n - p - q;
    enum { XY = 0, YZ = 1, ZX = 2, XPZ = 3, XMZ = 4 };
    __int128 v;
    if (r == 0) {
        v = moment2d(a.solve, m[XY], p, q);        // eq. 10: M_pq0 = M^{0:0}_pq
    } else if (p == 0) {
        v = moment2d(a.solve, m[YZ], q, r);        // eq. 11: M_0pq = M^{0:pi/2}_pq
    } else if (q == 0) {
        v = moment2d(a.solve, m[ZX], r, p);        // eq. 12: M_q0p = M^{pi/2:0}_pq
    } else if (p == 1 && q == 1 && r == 1) {       // eq. 13
        v = (moment2d(a.solve, m[XPZ], 2, 1) - moment2d(a.solve, m[XY], 2, 1) - moment2d(a.solve, m[YZ], 1, 2)) >> 1;
    } else if (p == 1 && q == 2 && r == 1) {       // eq. 14
        v = (moment2d(a.solve, m[XPZ], 2, 2) - moment2d(a.solve, m[XY], 2, 2) - moment2d(a.solve, m[YZ], 2, 2)) >> 1;
    } else {
        // eqs. 15, 16 with their left-hand sides exchanged; the X-Z moment M31 shifted to
        // the origin x-hat = N - 1 first (Section 5)
        const __int128 xh = a.xhat;
        const __int128 mm31 = moment2d(a.solve, m[XMZ], 3, 1) - 3 * moment2d(a.solve, m[XMZ], 2, 1) * xh +
                              3 * moment2d(a.solve, m[XMZ], 1, 1) * xh * xh -
                              moment2d(a.solve, m[XMZ], 0, 1) * xh * xh * xh;
        const __int128 mp31 = moment2d(a.solve, m[XPZ], 3, 1);
        const unsigned __int128 inv3 = ((unsigned __int128)0xAAAAAAAAAAAAAAAAull << 64) | 0xAAAAAAAAAAAAAAABull;
        __int128 t;
        if (p == 1)  // M_112
            t = mp31 + mm31 - 2 * moment2d(a.solve, m[XY], 3, 1);
        else         // M_211
            t = mp31 - mm31 - 2 * moment2d(a.solve, m[YZ], 1, 3);
        v = (__int128)((unsigned __int128)(t >> 1) * inv3);  // exact division by 6
    }
    put_i128(a.exact, a.fp64, idx, v);
}

__global__ void __launch_bounds__(256) drt_to_part_kernel(DrtToPartArgs a) {
    __shared__ __int128 m[NDIR_MAX][DRT_NDIR][DRT_KMAX + 1];
    load_m1d(a.m1d, a.nimg, m);
    __syncthreads();
    const int K = a.K, K1 = K + 1;
    for (int v = threadIdx.x; v < a.nimg * K1 * K1; v += blockDim.x) {
        const int d = v / (K1 * K1), k = (v / K1) % K1, q = v % K1;
        __int128 val = 0;
        if (k + q <= K) val = moment2d(a.solve, m[d], k, q);
        const unsigned __int128 u = (unsigned __int128)val;
        uint32_t *dst = a.part + (size_t)v * a.nlr;
        const uint32_t ext = val < 0 ? 0xffffffffu : 0u;
        for (int l = 0; l < a.nlr; ++l) dst[l] = l < 4 ? (uint32_t)(u >> (32 * l)) : ext;
    }
}

}  // namespace

hipError_t launch_paper_project(int elem, bool fast, const PaperProjArgs &a, hipStream_t st) {
    const dim3 grid((unsigned)((int64_t)a.nyb * a.nzb * a.nxt)), block(PP_WAVES * 64);
    if (elem == 2 && fast) hipLaunchKernelGGL((paper_project_kernel<uint16_t, true>), grid, block, 0, st, a);
    else if (elem == 2) hipLaunchKernelGGL((paper_project_kernel<uint16_t, false>), grid, block, 0, st, a);
    else if (fast) hipLaunchKernelGGL((paper_project_kernel<uint8_t, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((paper_project_kernel<uint8_t, false>), grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_paper_reduce(const PaperReduceArgs &a, hipStream_t st) {
    const int64_t W34 = a.L + a.N - 1;
    int64_t blocks = std::max<int64_t>(std::max<int64_t>(a.L * a.M, a.M * a.N), W34 * a.M);
    blocks = (blocks + 255) / 256;
    blocks = std::max<int64_t>(blocks, (a.N * a.L + 255) / 256);
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(paper_reduce_kernel, dim3((unsigned)blocks, a.nimg), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_drt_tiles(const DrtArgs &a, hipStream_t st) {
    if (a.ntiles <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(drt_tile_kernel, dim3(a.ntiles), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_drt_sum(const DrtSumArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(drt_sum_kernel, dim3(a.nimg, DRT_NDIR * (DRT_KMAX + 1)), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_paper_finish(const PaperFinishArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(paper_finish_kernel, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_drt_to_part(const DrtToPartArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(drt_to_part_kernel, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace dpm
