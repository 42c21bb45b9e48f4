// Internal launch interfaces of the HIP kernels (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpm_common.h"

namespace dpm {

// waves per projection workgroup
__host__ __device__ constexpr int slice_waves(int elem) { return 4; }
constexpr int NLR_MAX = 12;     // widest 2D-moment / recombination integer (32-bit limbs)

// Exact power sums on the matrix cores: the row values P(a) and the powers a^k are
// split into 7-bit limbs (int8 MFMA operands, int32 accumulation, all exact), and
// R_k = sum_a a^k P(a) is reassembled from the limb-pair sums.  `b` holds the powers'
// limbs already in the B-operand layout of v_mfma_i32_16x16x64_i8:
// b[(ks * nt + tile) * 64 + lane] = 16 bytes, byte i = limb column (16 tile + lane % 16)
// of a = 64 ks + 16 (lane / 16) + i.
struct PowTab {
    const uint4 *b;                 // null: use the VALU power sums
    int32_t amax;                   // a in [0, amax); multiple of 64
    int32_t nt;                     // 16-column tiles
    int32_t colstart[KMAX + 2];     // first limb column of a^k; colstart[K+1] = columns
};

// Image rows handed from the projection kernel to the power-sum kernel: item i, slot
// s = 2 d + side holds slot_len[s] int32 values (a = 0 .. len-1) at
// rows[i * row_stride + slot_off[s]].
constexpr int NSLOT = 2 * NDIR_MAX;
struct RowLayout {
    int32_t slot_off[NSLOT];
    int32_t slot_len[NSLOT];   // multiple of 64; 0 = empty slot
    int64_t row_stride;        // int32 values per item
    // power-sum tiles: 16 items x one slot x at most kchunk steps of 64 values of a;
    // slot s owns tiles [tile0[s], tile0[s+1]), nck[s] chunks per block of 16 items
    int32_t tile0[NSLOT + 1];
    int32_t nck[NSLOT];
    int32_t kchunk;
};

struct SliceArgs {
    const uint8_t *vol;
    int64_t L, M, N;
    int64_t pitch_y, pitch_z;  // elements
    int32_t zsplits, zrows;
    int32_t R, CT;             // lanes per sub-row, column tiles
    int32_t *rows;             // [item][row_stride]
    RowLayout rl;
    int32_t *images;           // optional
    int64_t img_off[7];        // element offset of each image of the group
    int64_t img_w[7];          // widths
    int32_t waves;             // first group, whole-row loads: 4 or 8 waves per workgroup
};

struct RoiDesc {
    int64_t offset;            // bytes into the packed buffer
    int64_t L, M, N;
    int32_t elem;              // bytes per voxel
    int32_t R, CT;
    int32_t item_pos;          // launch position of this ROI's first work item
    int32_t nitems;
    int32_t tile0;             // first power-sum tile of this ROI
    int32_t ntiles;            // power-sum tiles of this ROI
    int64_t row_base;          // int32 offset of item0's rows
    int32_t row_stride;        // int32 values per item
    int32_t slot_off[14];      // orders <= 6: slots 0..13
    int32_t slot_len[14];
    int32_t rowbytes;          // fused kernel: bytes of a row value in LDS (2 or 4)
    int32_t spw;               // fused kernel: slices a wave projects together (1, 2 or 4)
};

struct BatchItem {              // one y-slice of one ROI, whole z range (fused kernel: y = block of 16 slices)
    int32_t roi;
    int32_t y;
};

struct BatchSliceArgs {
    const uint8_t *packed;
    const RoiDesc *rois;
    BatchItem *items;          // written by the prep kernel, read by the projection
    int32_t K;
    int32_t *rows;
    int32_t *tile_roi;         // written by the prep kernel: ROI of every power-sum tile
    ItemGeom *geom;            // written by the prep kernel: geometry of every ROI
    const uint8_t *packed_end; // end of the ROIs' bytes in the packed buffer (readable before it)
};

// Power sums of the image rows, weighted in y per tile of 16 items:
// part[tile][k][q][NLR] = sum_{items i of the tile} y_i^q sum_a a^k row(i, slot, a), exact.
// Tiles are numbered slot-major over the non-empty slots (batched: from RoiDesc::tile0).
struct PowerArgs {
    const int32_t *rows;
    RowLayout rl;               // single volume
    const RoiDesc *rois;        // batched (null for a single volume)
    const int32_t *tile_roi;    // batched: ROI of every tile
    int32_t nrois;
    int32_t nitems;
    int32_t zsplits;            // single volume: y of item i is i / zsplits
    int32_t K;
    int32_t ntiles;             // work tiles (16 items x one slot)
    int32_t max_len;            // longest row slot (values)
    PowTab pow;                 // null b: VALU path
    uint32_t *part;
};
hipError_t launch_power(int nls, int nlr, const PowerArgs &a, hipStream_t st);
// Build the power table of `shape` (amax, nt, colstart; b ignored) into tab, which holds
// amax / 64 * nt * 64 uint4, on the device: the same bytes as the host build.
hipError_t launch_powtab_build(uint4 *tab, const PowTab &shape, int K, hipStream_t st);

// chain: the chained-window variant (uint16, first group, whole 64-lane rows, z ranges
// that are whole 32-row units)
hipError_t launch_slice(int elem, bool fast, bool chain, int g, int nd, const SliceArgs &a, int items, size_t lds,
                        hipStream_t st);
// One workgroup per ROI: its geometry, its work items (launch order item_pos + y) and
// the labels of its power-sum tiles.
hipError_t launch_batched_prep(int nd, const BatchSliceArgs &a, int nrois, hipStream_t st);
// Orders 7-16, whole-row loads, moments only: all direction groups in one launch
// (nd = K + 1 directions in total; lds = the largest group's LDS).
hipError_t launch_slice_groups(int elem, int nd, const SliceArgs &a, int items, size_t lds, hipStream_t st);
hipError_t launch_slice_batched(int elem, int g, int nd, const BatchSliceArgs &a, int items, size_t lds,
                                hipStream_t st);
// Fused batched kernel: one workgroup per (ROI, block of 16 y-slices) projects the block's
// slices into LDS and takes their matrix-core power sums from there, writing the same tile
// partials as launch_power (pw: K, power table, part).  Workgroups of ROIs whose voxel
// size or row-value size differs from (elem, rowbytes) return at once.
struct BlockArgs {
    BatchSliceArgs b;
    PowerArgs pw;
};
hipError_t launch_slice_block(int elem, int rowbytes, int nd, const BlockArgs &a, int items, size_t lds,
                              hipStream_t st);

// Tile sums and recombination into the 3D moments; grid = (moments, volumes).
struct FinishArgs {
    const uint32_t *part;      // tile partials (PowerArgs::part)
    const RoiDesc *rois;       // batched (null for a single volume)
    int32_t nvol, K;
    int32_t tile0[NSLOT + 1];  // single volume: tiles of slot s are [tile0[s], tile0[s+1])
    void *exact;               // dpm_i128 [vol][n_moments(min(K,4))] or null
    double *fp64;              // [vol][n_moments(K)] or null
    uint32_t *raw;             // exact moments, NLR 32-bit limbs each, [vol][n_moments(K)], or null
};
hipError_t launch_finish(int nlr, const FinishArgs &a, hipStream_t st);

// Moments from supplied projection images: image d (the layout of dpm_project_images)
// gathered into the row slots of item y = one image row, split at the origin.  Entries
// outside [0, bound] are replaced by 0 and reported in *bad.
struct ImgArgs {
    const int32_t *images;
    int64_t off[NDIR_MAX];     // int32 offset of image d
    int32_t width[NDIR_MAX];
    int32_t origin[NDIR_MAX];  // column of the true origin, |beta| (N-1) for beta < 0
    int32_t nd, M;
    int64_t bound;
    int32_t *rows;
    RowLayout rl;
    uint32_t *bad;
};
hipError_t launch_images_to_rows(const ImgArgs &a, hipStream_t st);

// Features of one volume from its exact moments (FinishArgs::raw, nlr limbs each), in w
// limbs; outputs are device arrays of n_moments(K) doubles (eta, mu_phys optional).
struct FeatArgs {
    const uint32_t *raw;
    int32_t K;
    double spacing[3];
    double *centroid;          // 3 or null
    double *mu, *eta, *mu_phys;
};
hipError_t launch_features(int nlr, int w, const FeatArgs &f, hipStream_t st);

// recombination tables (host side generation, device upload)
struct RecombTables {
    int64_t num[KMAX + 1][KMAX + 1][KMAX + 1];  // [k][p][d]
    int32_t shift[KMAX + 1][KMAX + 1];          // den = 2^shift * odd
    uint32_t inv[KMAX + 1][KMAX + 1][NLR_MAX];  // odd^-1 mod 2^(32*NLR_MAX)
    uint64_t den[KMAX + 1][KMAX + 1];
    int32_t numsum_bits[KMAX + 1];              // bits of max_p sum_d |num|
};
bool build_recomb_tables(RecombTables &t);
hipError_t upload_recomb_tables(const RecombTables &t);

}  // namespace dpm
