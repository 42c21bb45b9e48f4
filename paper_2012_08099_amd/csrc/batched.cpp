// Batched regions of interest: many independent volumes of uneven size in one
// launch sequence (projection kernel over every (ROI, y-slice) work item, one
// reduction block per ROI, one recombination block per ROI).  Work items are laid out
// longest-first (LPT order) so the large ROIs start early and the small ones fill the
// tail of the grid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/dpm.h"
#include "dpm_common.h"
#include "kernels.h"

namespace dpm {
int batched_ensure_tables();  // dpm_api.cpp
int batched_numsum_bits(int k);
void batched_set_error(int e);
}  // namespace dpm

namespace {
using namespace dpm;

int bitlen_u64(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

struct BPlan {
    int K = 0, nrois = 0, items = 0, npairs = 0;
    int nls = 4, nlr = 4;
    int jobbins = 512;
    size_t lds = 0;
    bool has_u8 = false, has_u16 = false;
    std::vector<RoiDesc> rd;
    std::vector<BatchItem> it;
    size_t off_rd = 0, off_it = 0, off_part = 0, off_m2 = 0, total = 0;
};

size_t al(size_t v) { return (v + 255) / 256 * 256; }

int bplan(const dpm_roi *rois, int n, int K, BPlan &p) {
    if (!rois || n <= 0 || K < 0 || K > 6) return K > 6 ? DPM_ENOTSUP : DPM_EINVAL;
    p.K = K;
    p.nrois = n;
    p.npairs = n_pairs(K);
    p.rd.resize(n);
    int brec = 0, bsl = 0;
    std::vector<std::pair<int64_t, int>> order;  // (cost, roi)
    for (int i = 0; i < n; ++i) {
        const dpm_roi &r = rois[i];
        const int elem = r.dtype == DPM_U8 ? 1 : r.dtype == DPM_U16 ? 2 : 0;
        if (!elem || r.dims[0] <= 0 || r.dims[1] <= 0 || r.dims[2] <= 0) return DPM_EINVAL;
        if (r.dims[0] > 4096 || r.dims[1] > 4096 || r.dims[2] > 4096) return DPM_ERANGE;
        (elem == 1 ? p.has_u8 : p.has_u16) = true;
        RoiDesc &d = p.rd[i];
        d.offset = (int64_t)r.offset_bytes;
        d.L = r.dims[0];
        d.M = r.dims[1];
        d.N = r.dims[2];
        d.elem = elem;
        const int64_t lanes = (d.L + G - 1) / G;
        if (lanes <= 64) {
            int rr = 8;
            while (rr < lanes) rr <<= 1;
            d.R = rr;
            d.CT = 1;
        } else {
            d.R = 64;
            d.CT = (int)((lanes + 63) / 64);
        }
        // widths (same bounds as the single-volume plan)
        const uint64_t vmax = elem == 1 ? 255u : 65535u;
        int64_t umax = 1;
        for (int dd = 0; dd <= K; ++dd)
            umax = std::max<int64_t>(umax, dir_alpha(dd) * (d.L - 1) + iabs_c(dir_beta(dd)) * (d.N - 1));
        const int bu = bitlen_u64((uint64_t)umax);
        const int by = bitlen_u64((uint64_t)std::max<int64_t>(d.M - 1, 1));
        const int bvol = bitlen_u64(vmax) + bitlen_u64((uint64_t)(d.L * d.M * d.N));
        bsl = std::max(bsl, bitlen_u64(vmax) + bitlen_u64((uint64_t)(d.L * d.N)) + K * bu + 1);
        for (int k = 0; k <= K; ++k)
            for (int q = 0; k + q <= K; ++q)
                brec = std::max(brec, bvol + k * bu + q * by + batched_numsum_bits(k) + 2);
        order.push_back({d.L * d.N, i});
        // LDS of one item of this ROI (all items of a ROI share the geometry shape)
        ItemGeom ig;
        item_geometry(0, K + 1 < 7 ? K + 1 : 7, d.L, d.N, 0, d.N, ig);
        const int nj = count_jobs(ig, K + 1 < 7 ? K + 1 : 7, p.jobbins);
        p.lds = std::max(p.lds, ((size_t)ig.lds_dwords + (size_t)nj * (KMAX + 1) * 4) * 4);
    }
    if (bsl > 128) return DPM_ERANGE;
    p.nls = 4;
    if (brec <= 128) p.nlr = 4;
    else if (brec <= 256) p.nlr = 8;
    else return DPM_ERANGE;
    if (p.lds > 160 * 1024) return DPM_ERANGE;
    // items longest slice first; item slot = position in this order
    std::stable_sort(order.begin(), order.end(), [](auto &a, auto &b) { return a.first > b.first; });
    int slot = 0;
    std::vector<std::vector<BatchItem>> per(n);
    for (auto &o : order) {
        const int i = o.second;
        for (int64_t y = 0; y < p.rd[i].M; ++y) {
            BatchItem b{};
            b.roi = i;
            b.slot = slot++;
            b.y = (int32_t)y;
            b.zs = 0;
            b.ze = (int32_t)p.rd[i].N;
            per[i].push_back(b);
        }
    }
    // grid order = slot order; per-ROI index lists for the reduction
    p.it.resize(slot);
    std::vector<BatchItem> byroi;
    byroi.reserve(slot);
    for (int i = 0; i < n; ++i) {
        p.rd[i].item0 = (int32_t)byroi.size();
        p.rd[i].nitems = (int32_t)per[i].size();
        for (auto &b : per[i]) {
            byroi.push_back(b);
            p.it[b.slot] = b;
        }
    }
    // the grid walks p.it (slot order); the reduction walks byroi via item0/nitems
    p.it.insert(p.it.end(), byroi.begin(), byroi.end());
    p.items = slot;
    p.off_rd = 0;
    p.off_it = al(sizeof(RoiDesc) * n);
    p.off_part = p.off_it + al(sizeof(BatchItem) * p.it.size());
    p.off_m2 = p.off_part + al((size_t)p.items * p.npairs * p.nls * 4);
    p.total = p.off_m2 + al((size_t)n * p.npairs * (K + 1) * p.nlr * 4);
    return DPM_OK;
}

}  // namespace

extern "C" {

size_t dpm_batched_workspace_bytes(const dpm_roi *rois, int n_rois, int max_order) {
    BPlan p;
    if (bplan(rois, n_rois, max_order, p)) return 0;
    return p.total;
}

int dpm_moments_batched(const void *packed, const dpm_roi *rois, int n_rois, int max_order,
                        const dpm_out *out_device, void *workspace, size_t ws_bytes, void *stream) {
    if (!packed || !out_device || !workspace) return DPM_EINVAL;
    int rc = batched_ensure_tables();
    if (rc) return rc;
    BPlan p;
    if ((rc = bplan(rois, n_rois, max_order, p))) return rc;
    if (ws_bytes < p.total) return DPM_ENOMEM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    RoiDesc *drd = reinterpret_cast<RoiDesc *>(ws + p.off_rd);
    BatchItem *dit = reinterpret_cast<BatchItem *>(ws + p.off_it);
    uint32_t *part = reinterpret_cast<uint32_t *>(ws + p.off_part);
    uint32_t *m2 = reinterpret_cast<uint32_t *>(ws + p.off_m2);
    hipError_t e = hipMemcpyAsync(drd, p.rd.data(), sizeof(RoiDesc) * p.rd.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dit, p.it.data(), sizeof(BatchItem) * p.it.size(), hipMemcpyHostToDevice, st);
    // pageable sources: make sure the copies have consumed them before returning
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        batched_set_error((int)e);
        return DPM_EDEVICE;
    }
    const int nd = max_order + 1;
    BatchSliceArgs a{static_cast<const uint8_t *>(packed), drd, dit, max_order, p.jobbins, p.npairs, part};
    if (p.has_u16) e = launch_slice_batched(2, p.nls, 0, nd, a, p.items, p.lds, st);
    if (e == hipSuccess && p.has_u8) e = launch_slice_batched(1, p.nls, 0, nd, a, p.items, p.lds, st);
    if (e == hipSuccess) {
        // the reduction's per-ROI item lists follow the slot-ordered grid list
        ReduceBatchedArgs r{part, drd, dit + p.items, n_rois, max_order, p.npairs, m2};
        e = launch_reduce_batched(p.nls, p.nlr, r, st);
    }
    if (e == hipSuccess) {
        RecombArgs c{m2, n_rois, max_order, p.npairs, out_device->exact, out_device->fp64, nullptr};
        e = launch_recombine(p.nlr, c, st);
    }
    if (e != hipSuccess) {
        batched_set_error((int)e);
        return DPM_EDEVICE;
    }
    return DPM_OK;
}

}  // extern "C"
