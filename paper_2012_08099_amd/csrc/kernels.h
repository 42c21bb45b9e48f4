// Internal launch interfaces of the HIP kernels (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpm_common.h"

namespace dpm {

constexpr int SLICE_WAVES = 4;  // waves per projection workgroup
constexpr int NLR_MAX = 12;     // widest 2D-moment / recombination integer (32-bit limbs)

struct SliceArgs {
    const uint8_t *vol;
    int64_t L, M, N;
    int64_t pitch_y, pitch_z;  // elements
    int32_t zsplits, zrows;
    int32_t K;
    int32_t R, CT;             // lanes per sub-row, column tiles
    int32_t jobbins;
    int32_t npairs;            // pairs (d, k) over all groups
    uint32_t *part;            // [item][npairs][NLS]
    int32_t *images;           // optional
    int64_t img_off[7];        // element offset of each image of the group
    int64_t img_w[7];          // widths
};

struct RoiDesc {
    int64_t offset;            // bytes into the packed buffer
    int64_t L, M, N;
    int32_t elem;              // bytes per voxel
    int32_t R, CT;
    int32_t item0;             // first work item of this ROI
    int32_t nitems;
};

struct BatchItem {
    int32_t roi;
    int32_t slot;              // row of the partial-sum table
    int32_t y, zs, ze;
};

struct BatchSliceArgs {
    const uint8_t *packed;
    const RoiDesc *rois;
    const BatchItem *items;
    int32_t K;
    int32_t jobbins;
    int32_t npairs;
    uint32_t *part;
};

hipError_t launch_slice(int elem, int nls, bool fast, int g, int nd, const SliceArgs &a, int items,
                        size_t lds, hipStream_t st);
hipError_t launch_slice_batched(int elem, int nls, int g, int nd, const BatchSliceArgs &a, int items,
                                size_t lds, hipStream_t st);

// y-weighted reduction: M2[pair][q] = sum_items y^q part[item][pair]
struct ReduceArgs {
    const uint32_t *part;
    int32_t nitems, zsplits;
    int32_t K, npairs;
    uint32_t *m2;              // [pair][K+1][NLR]
};
hipError_t launch_reduce(int nls, int nlr, const ReduceArgs &a, hipStream_t st);

// batched: one block per ROI
struct ReduceBatchedArgs {
    const uint32_t *part;
    const RoiDesc *rois;
    const BatchItem *items;
    int32_t nrois, K, npairs;
    uint32_t *m2;              // [roi][pair][K+1][NLR]
};
hipError_t launch_reduce_batched(int nls, int nlr, const ReduceBatchedArgs &a, hipStream_t st);

// recombination into 3D moments; grid = number of volumes
struct RecombArgs {
    const uint32_t *m2;        // [vol][pair][K+1][NLR]
    int32_t nvol, K, npairs;
    void *exact;               // dpm_i128 [vol][n_moments(min(K,4))] or null
    double *fp64;              // [vol][n_moments(K)] or null
    uint32_t *wide;            // optional exact values [vol][n_moments(K)][NLR]
};
hipError_t launch_recombine(int nlr, const RecombArgs &a, hipStream_t st);

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
