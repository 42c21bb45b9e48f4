// Internal launch interfaces of the paper-literal mode and of the 1D-integral route for
// the 2D moments (not part of the public C ABI).
//
// Paper mode (orders <= 4): the five images of Section 3.1 -- XY (eq. 5), YZ (eq. 6),
// ZX (eq. 7), X+Z (eq. 8) and X-Z (eq. 9) -- from one pass over the volume; their 2D
// moments from the 1D integrals of Section 5 (Vert, Horiz, Diag, AntiDiag, X2Y); the 3D
// moments by eqs. 10-16 with the offset correction of Section 5.
//
// Every image is stored row-major as img[j][i] (row j, column i) with I(i, j) as the
// paper indexes it: XY i = x, j = y; YZ i = y, j = z; ZX i = z, j = x; X+Z i = x + z,
// j = y; X-Z i = x - z + N - 1, j = y.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpm_common.h"

namespace dpm {

constexpr int PAPER_NIMG = 5;   // XY, YZ, ZX, X+Z, X-Z
constexpr int DRT_NDIR = 5;     // Vert, Horiz, Diag, AntiDiag, X2Y: t = a i + b j
constexpr int DRT_KMAX = 4;

// Projection tile of one workgroup: PP_BY rows of y, PP_BZ planes of z (PP_WAVES waves,
// PP_ZW planes each), PP_XT voxels of x (64 lanes x 8).
constexpr int PP_WAVES = 8;
constexpr int PP_ZW = 8;
constexpr int PP_BZ = PP_WAVES * PP_ZW;  // 64
constexpr int PP_BY = 16;
constexpr int PP_XT = 512;
constexpr int PP_DW = PP_XT + PP_BZ - 1;  // bins of an X+Z / X-Z partial row

// Partial images written by the projection and summed, in a fixed order, by the reduce
// kernel (int32; exact: every entry is a line sum of at most max(L, M, N) voxels):
//   xy  [nzb][M][L]            XY partial over the z-block zb
//   xpz [nzb][nxt][M][PP_DW]   X+Z partial: bin s of (zb, xt) is column x0 + z0 + s
//   xmz [nzb][nxt][M][PP_DW]   X-Z partial: bin s is column x0 - z0 + N - PP_BZ + s
//   zx  [nyb][N][L]            ZX partial over the y-block yb, stored [z][x]
//   yz  [nxt][N][M]            YZ partial over the x-tile xt, stored [z][y]
struct PaperProjArgs {
    const uint8_t *vol;
    int64_t L, M, N;
    int32_t nyb, nzb, nxt;
    int32_t *xy, *xpz, *xmz, *zx, *yz;
    int32_t nimg;               // 3 (orders <= 2), 4 (order 3) or 5
};

struct PaperReduceArgs {
    int64_t L, M, N;
    int32_t nyb, nzb, nxt, nimg;
    const int32_t *xy, *xpz, *xmz, *zx, *yz;
    int32_t *img[PAPER_NIMG];   // output images ([j][i])
};

hipError_t launch_paper_project(int elem, bool fast, const PaperProjArgs &a, hipStream_t st);
hipError_t launch_paper_reduce(const PaperReduceArgs &a, hipStream_t st);

// 1D-integral (DRT) route for the 2D moments of a set of images.  Each image is cut into
// tiles of DRT_IB columns x DRT_RB rows; a tile accumulates its part of the 1D integrals
// of Section 5 with additions only, then takes their 1D moments
//     m_g,n = sum_t (t - a_g io)^n P_g(t),   g < ndir, n <= K
// (t = a_g i + b_g j, io = the column of the image's moment origin) and writes them as
// int128 to part1d[tile][g][n].
constexpr int DRT_IB = 256;
constexpr int DRT_RB = 32;
constexpr int DRT_MAXIMG = 17;

struct DrtImage {
    const int32_t *img;
    int32_t W, H;               // columns (i), rows (j)
    int32_t io;                 // moment origin column
    int32_t tile0;              // first tile of this image
    int32_t tiles_i;            // tiles along i
};

struct DrtArgs {
    DrtImage im[DRT_MAXIMG];
    int32_t nimg, ntiles, ndir, K;
    __int128 *part1d;           // [tile][DRT_NDIR][DRT_KMAX + 1]
};

hipError_t launch_drt_tiles(const DrtArgs &a, hipStream_t st);

// m1d[e][g][n] = sum over the tiles of image e of part1d[tile][g][n], in tile order (one
// wave per (image, g, n)).
struct DrtSumArgs {
    const __int128 *part1d;
    int32_t tile0[DRT_MAXIMG + 1];
    int32_t nimg;
    __int128 *m1d;              // [DRT_MAXIMG][DRT_NDIR][DRT_KMAX + 1]
};
hipError_t launch_drt_sum(const DrtSumArgs &a, hipStream_t st);

// Exact inverse of the 1D-to-2D system of order n over the directions (a_g, b_g), g <= n:
//   m_g,n = sum_p C(n, p) a_g^p b_g^(n-p) M_{p, n-p}
//   M_{p, n-p} = sum_g num[n][p][g] m_g,n / den[n][p],  den = 2^shift * odd,
// the division done exactly as a shift and a multiplication by odd^-1 mod 2^128.
struct DrtSolve {
    int64_t num[DRT_KMAX + 1][DRT_KMAX + 1][DRT_NDIR];
    int32_t shift[DRT_KMAX + 1][DRT_KMAX + 1];
    uint64_t inv_lo[DRT_KMAX + 1][DRT_KMAX + 1], inv_hi[DRT_KMAX + 1][DRT_KMAX + 1];
};

// Paper finish: per image, the summed 1D moments solved into the 2D moments; X-Z shifted to its origin N - 1 (Section 5); eqs. 10-16 (15/16 with their
// left-hand sides exchanged) give the 3D moments.
struct PaperFinishArgs {
    const __int128 *m1d;        // DrtSumArgs::m1d
    int32_t nimg, ndir, K;
    int64_t xhat;               // N - 1
    DrtSolve solve;
    void *exact;                // dpm_i128[n_moments(K)] or null
    double *fp64;               // [n_moments(K)] or null
};
hipError_t launch_paper_finish(const PaperFinishArgs &a, hipStream_t st);

// Family route: the 2D moments M^d_{k,q} (k + q <= K) of images d = 0..K, about their
// origins, written into the tile partials the recombination kernel reads -- one tile per
// image, in slot 2d + 1 -- as nlr 32-bit limbs: part[d][k][q][nlr].
struct DrtToPartArgs {
    const __int128 *m1d;        // DrtSumArgs::m1d
    int32_t nimg, ndir, K, nlr;
    DrtSolve solve;
    uint32_t *part;
};
hipError_t launch_drt_to_part(const DrtToPartArgs &a, hipStream_t st);

// The directions of the 1D integrals of Section 5, t = a i + b j (i: column, j: row).
__host__ __device__ constexpr int drt_a(int g) { return g == 1 ? 0 : 1; }
__host__ __device__ constexpr int drt_b(int g) { return g == 0 ? 0 : g == 1 ? 1 : g == 2 ? 1 : g == 3 ? -1 : 2; }

}  // namespace dpm
