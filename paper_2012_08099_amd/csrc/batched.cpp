// Batched regions of interest: many independent volumes of uneven size in one
// launch sequence (projection kernel over every (ROI, y-slice) work item, power-sum
// tiles of every ROI in one grid, one recombination workgroup per (ROI, moment)).  A prep kernel
// writes each ROI's geometry, its work items and its tile labels on the device; items are laid out
// longest-first (LPT order) so the large ROIs start early and the small ones fill the
// tail of the grid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/dpm.h"
#include "dpm_common.h"
#include "kernels.h"

namespace dpm {
int batched_ensure_tables();  // dpm_api.cpp
int batched_numsum_bits(int k);
void batched_set_error(int e);
void batched_prof_mark(int idx, hipStream_t st);
bool batched_profiling();
int batched_run(const void *packed, const dpm_roi *rois, int n_rois, int max_order, const dpm_out *out_device,
                void *workspace, size_t ws_bytes, void *stream, bool allow_graphs);
int batched_powtab(int amax, int K, PowTab &out);
bool batched_pow_columns(int amax, int K, int32_t colstart[KMAX + 2]);
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
    int K = 0, nrois = 0, items = 0, npairs = 0, ntiles = 0;
    int nls = 4, nlr = 4;
    size_t lds = 0;
    bool mfma = false;
    // ROIs whose block of 16 slices fits the fused kernel go to it (rows kept in LDS), the
    // others to the separate projection and power-sum kernels.  Their work items and tiles
    // come first: items [0, items_sep), tiles [0, ntiles_sep); the fused ROIs' blocks and
    // tiles follow.  LDS of each fused launch class (uint8 / uint16 row values, uint8 /
    // uint32, uint16 / uint32).
    int n_fused = 0, items_sep = 0, ntiles_sep = 0;
    bool sep_u8 = false, sep_u16 = false;
    size_t lds_block[3] = {0, 0, 0};
    int amax = 64;
    int64_t packed_bytes = 0;  // end of the last byte of any ROI in the packed buffer
    std::vector<RoiDesc> rd;
    size_t off_rd = 0, off_it = 0, off_geom = 0, off_rows = 0, off_part = 0, off_tmap = 0, total = 0;
};

size_t al(size_t v) { return (v + 255) / 256 * 256; }

// The fused kernel takes a batch whose every ROI's block fits this much LDS (two
// workgroups per CU at the limit); DPM_BATCH_FUSED=0 keeps the separate kernels.
constexpr int64_t kBlockLdsMax = 80 * 1024;
// Slices are grouped per wave while a ROI's block stays within the larger of this and
// the batch's largest block at one slice per wave.
constexpr int64_t kBlockLdsGroup = 48 * 1024;
bool fused_allowed() {
    const char *e = std::getenv("DPM_BATCH_FUSED");
    return !(e && e[0] == '0');
}
int block_class(int elem, int rowbytes) { return elem == 2 ? 2 : rowbytes == 2 ? 0 : 1; }

// Per-order overrides of the batch geometry (dpm_batch_tune_set), and a generation that
// every change bumps: cached graphs of an older generation never match again.
std::mutex g_btune_mu;
dpm_batch_tuning g_btune[7] = {};
uint64_t g_btune_gen = 0;
dpm_batch_tuning batch_tuning(int K, uint64_t *gen) {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    if (gen) *gen = g_btune_gen;
    return (K >= 0 && K <= 6) ? g_btune[K] : dpm_batch_tuning{};
}

// Pinned staging for the descriptor upload, so the call stays asynchronous: a buffer
// is reused only once the event recorded after its copy has fired.
struct Staging {
    void *p = nullptr;
    size_t n = 0;
    int dev = -1;
    hipEvent_t ev = nullptr;
};
std::mutex g_stage_mu;
std::vector<Staging> g_stage;

Staging *stage_acquire(size_t n, int dev) {
    for (auto &s : g_stage)
        if (s.dev == dev && s.n >= n && hipEventQuery(s.ev) == hipSuccess) return &s;
    Staging s;
    s.n = std::max<size_t>(n, 1 << 20);
    s.dev = dev;
    if (hipHostMalloc(&s.p, s.n, hipHostMallocDefault) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(s.p);
        return nullptr;
    }
    g_stage.push_back(s);
    return &g_stage.back();
}

int bplan(const dpm_roi *rois, int n, int K, BPlan &p) {
    if (!rois || n <= 0 || K < 0 || K > 6) return K > 6 ? DPM_ENOTSUP : DPM_EINVAL;
    p.K = K;
    p.nrois = n;
    p.npairs = n_pairs(K);
    p.rd.resize(n);
    const int nd = K + 1;
    int brec = 0, bsl = 0;
    bool small_p = true;
    std::vector<ItemGeom> geoms(n);
    std::vector<int64_t> lds1(n);   // fused block at one slice per wave
    std::vector<int32_t> nslot(n);  // non-empty slots
    std::vector<std::pair<int64_t, int>> order;  // (cost, roi)
    for (int i = 0; i < n; ++i) {
        const dpm_roi &r = rois[i];
        const int elem = r.dtype == DPM_U8 ? 1 : r.dtype == DPM_U16 ? 2 : 0;
        if (!elem || r.dims[0] <= 0 || r.dims[1] <= 0 || r.dims[2] <= 0) return DPM_EINVAL;
        if (r.dims[0] > 4096 || r.dims[1] > 4096 || r.dims[2] > 4096) return DPM_ERANGE;
        RoiDesc &d = p.rd[i];
        d = RoiDesc{};
        d.offset = (int64_t)r.offset_bytes;
        d.L = r.dims[0];
        d.M = r.dims[1];
        d.N = r.dims[2];
        d.elem = elem;
        p.packed_bytes = std::max<int64_t>(p.packed_bytes, d.offset + d.L * d.M * d.N * elem);
        const int G = lane_voxels(elem);
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
        if ((double)vmax * (double)std::max(d.L, d.N) >= 268435456.0) small_p = false;
        // geometry of this ROI's items (full z range): LDS and row layout
        ItemGeom &ig = geoms[i];
        item_geometry(0, nd, G, d.L, d.N, 0, d.N, ig);
        p.lds = std::max(p.lds, (size_t)ig.lds_dwords * 4);
        // row values of the fused kernel: uint16 for uint8 voxels when no line sum can reach
        // 2^16, else uint32 (the only instantiation for uint16 voxels)
        d.rowbytes = elem == 1 && (double)vmax * (double)std::max(d.L, d.N) < 65536.0 ? 2 : 4;
        d.spw = 1;
        lds1[i] = bk_lds_bytes(ig, nd, d.rowbytes, 1);
        int32_t off = 0, nsl = 0;
        for (int sl = 0; sl < 14; ++sl) {
            int32_t len = 0;
            if (sl < 2 * nd && ig.seg_ahi[sl] >= ig.seg_alo[sl]) len = round64((int64_t)ig.seg_ahi[sl] + 1);
            d.slot_off[sl] = off;
            d.slot_len[sl] = len;
            off += len;
            if (len) ++nsl;
            p.amax = std::max(p.amax, (int)len);
        }
        d.row_stride = off;
        nslot[i] = nsl;
        order.push_back({d.L * d.N, i});
    }
    if (bsl > 128) return DPM_ERANGE;
    p.nls = 4;
    if (brec <= 128) p.nlr = 4;
    else if (brec <= 256) p.nlr = 8;
    else return DPM_ERANGE;
    if (p.lds > 160 * 1024) return DPM_ERANGE;
    int32_t cs[KMAX + 2];
    p.mfma = small_p && p.amax <= 8192 && batched_pow_columns(p.amax, K, cs);
    const dpm_batch_tuning bt = batch_tuning(K, nullptr);
    const bool fuse_ok = p.mfma && p.nlr == 4 && fused_allowed() && bt.fused >= 0;
    const int spw_max = bt.max_spw ? bt.max_spw : 4;  // 1, 2 or 4
    const int units = bt.units ? bt.units : 2;        // units per sub-row the grouping aims at
    std::vector<char> fz(n, 0);
    int64_t lds_blk_max = 0;
    for (int i = 0; i < n; ++i)
        if (fuse_ok && lds1[i] <= kBlockLdsMax) {
            fz[i] = 1;
            ++p.n_fused;
            lds_blk_max = std::max(lds_blk_max, lds1[i]);
        }
    // separate ROIs: one work item per slice, rows in the workspace, their tiles first
    int64_t row_base = 0;
    int32_t tile0 = 0;
    for (int i = 0; i < n; ++i) {
        if (fz[i]) continue;
        RoiDesc &d = p.rd[i];
        d.row_base = row_base;
        row_base += (int64_t)d.row_stride * d.M;
        d.nitems = (int32_t)d.M;
        p.items_sep += d.nitems;
        d.tile0 = tile0;
        d.ntiles = nslot[i] * (int)((d.M + 15) / 16);
        tile0 += d.ntiles;
        (d.elem == 1 ? p.sep_u8 : p.sep_u16) = true;
    }
    p.ntiles_sep = tile0;
    if (p.n_fused) {
        // fused ROIs: work items (ROI, block of 16 slices), no rows
        const int64_t cap = std::max<int64_t>(lds_blk_max, kBlockLdsGroup);
        for (int i = 0; i < n; ++i) {
            if (!fz[i]) continue;
            RoiDesc &d = p.rd[i];
            d.nitems = (int32_t)((d.M + BK_YB - 1) / BK_YB);
            d.tile0 = tile0;
            d.ntiles = nslot[i] * (int)((d.M + 15) / 16);
            tile0 += d.ntiles;
            // the fused kernel's sub-rows may be narrower than 8 lanes: rows of <= 32
            // voxels keep their lanes busy
            if (d.CT == 1) {
                const int64_t lanes = (d.L + lane_voxels(d.elem) - 1) / lane_voxels(d.elem);
                int rr = 1;
                while (rr < lanes) rr <<= 1;
                d.R = rr;
            }
            // slices a wave projects together: enough units for two (or the tuned number)
            // per sub-row, as far as the LDS of the batch's largest block allows
            const int64_t u1 = (int64_t)d.CT * geoms[i].n_chunks, subrows = 64 / d.R;
            while (d.spw < spw_max && d.spw * u1 < units * subrows &&
                   bk_lds_bytes(geoms[i], nd, d.rowbytes, 2 * d.spw) <= cap)
                d.spw *= 2;
            size_t &cl = p.lds_block[block_class(d.elem, d.rowbytes)];
            cl = std::max(cl, (size_t)bk_lds_bytes(geoms[i], nd, d.rowbytes, d.spw));
        }
    }
    p.ntiles = tile0;
    // work items of each kind, largest slices first (LPT order)
    std::stable_sort(order.begin(), order.end(), [](auto &a, auto &b) { return a.first > b.first; });
    int32_t pos_s = 0, pos_f = p.items_sep;
    for (auto &o : order) {
        RoiDesc &d = p.rd[o.second];
        int32_t &pos = fz[o.second] ? pos_f : pos_s;
        d.item_pos = pos;
        pos += d.nitems;
    }
    p.items = pos_f;
    p.off_rd = 0;
    p.off_it = al(sizeof(RoiDesc) * n);
    p.off_geom = p.off_it + al(sizeof(BatchItem) * (size_t)p.items);
    p.off_rows = p.off_geom + al(sizeof(ItemGeom) * (size_t)n);
    p.off_part = p.off_rows + al((size_t)row_base * 4);
    p.off_tmap = p.off_part + al((size_t)p.ntiles * (K + 1) * (K + 1) * p.nlr * 4);
    p.total = p.off_tmap + al((size_t)p.ntiles * 4);
    return DPM_OK;
}

// The launch sequence of one batched call: prep, projection, power sums, recombination.
// drd holds the plan's ROI descriptors on the device.
hipError_t enqueue(const BPlan &p, const PowTab &pt, const uint8_t *packed, RoiDesc *drd, uint8_t *ws,
                   const dpm_out *out, hipStream_t st, bool marks) {
    const int K = p.K, nd = K + 1;
    BatchItem *dit = reinterpret_cast<BatchItem *>(ws + p.off_it);
    int32_t *rows = reinterpret_cast<int32_t *>(ws + p.off_rows);
    uint32_t *part = reinterpret_cast<uint32_t *>(ws + p.off_part);
    int32_t *tmap = reinterpret_cast<int32_t *>(ws + p.off_tmap);
    if (marks) batched_prof_mark(0, st);
    BatchSliceArgs a{packed, drd, dit, K, rows, tmap, reinterpret_cast<ItemGeom *>(ws + p.off_geom),
                     packed + p.packed_bytes};
    hipError_t e = launch_batched_prep(nd, a, p.nrois, st);
    if (e == hipSuccess && p.n_fused) {
        BlockArgs ba{};
        ba.b = a;
        ba.b.items = dit + p.items_sep;  // the fused ROIs' blocks
        ba.pw.rois = drd;
        ba.pw.tile_roi = tmap;
        ba.pw.nrois = p.nrois;
        ba.pw.K = K;
        ba.pw.ntiles = p.ntiles;
        ba.pw.max_len = p.amax;
        ba.pw.pow = pt;
        ba.pw.part = part;
        // one launch per class present; workgroups of the other classes return at once
        const int elems[3] = {1, 1, 2}, rbytes[3] = {2, 4, 4};
        for (int c = 0; c < 3 && e == hipSuccess; ++c)
            if (p.lds_block[c])
                e = launch_slice_block(elems[c], rbytes[c], nd, ba, p.items - p.items_sep, p.lds_block[c], st);
    }
    if (e == hipSuccess && p.sep_u16) e = launch_slice_batched(2, 0, nd, a, p.items_sep, p.lds, st);
    if (e == hipSuccess && p.sep_u8) e = launch_slice_batched(1, 0, nd, a, p.items_sep, p.lds, st);
    if (e == hipSuccess && marks) batched_prof_mark(1, st);
    if (e == hipSuccess && p.ntiles_sep) {
        PowerArgs pa{};
        pa.rows = rows;
        pa.rois = drd;
        pa.tile_roi = tmap;
        pa.nrois = p.nrois;
        pa.nitems = p.items_sep;
        pa.zsplits = 1;
        pa.K = K;
        pa.ntiles = p.ntiles_sep;  // the separate ROIs' tiles
        pa.max_len = p.amax;
        pa.pow = pt;
        pa.part = part;
        e = launch_power(p.nls, p.nlr, pa, st);
    }
    if (e == hipSuccess && marks) batched_prof_mark(2, st);
    if (e == hipSuccess) {
        FinishArgs f{};
        f.part = part;
        f.rois = drd;
        f.nvol = p.nrois;
        f.K = K;
        f.exact = out->exact;
        f.fp64 = out->fp64;
        e = launch_finish(p.nlr, f, st);
    }
    if (e == hipSuccess && marks) batched_prof_mark(3, st);
    return e;
}

// ---- hipGraph per repeated call
// A call whose ROI descriptors, buffers, order and device repeat an earlier call's is
// captured once (on its second sighting) and replayed from then on: the replay skips the
// host planning and the descriptor upload.  The graph owns a device copy of the
// descriptors; everything else lives in the caller's buffers, which the key pins.
struct GraphKey {
    int dev = -1, n = 0, K = 0;
    uint64_t tune_gen = 0;  // generation of the batch tuning the plan was made with
    const void *packed = nullptr, *exact = nullptr, *fp64 = nullptr, *ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<uint8_t> rois;
    uint64_t hash = 0;
    bool operator==(const GraphKey &o) const {
        return hash == o.hash && dev == o.dev && n == o.n && K == o.K && tune_gen == o.tune_gen && packed == o.packed &&
               exact == o.exact &&
               fp64 == o.fp64 && ws == o.ws && ws_bytes == o.ws_bytes && rois == o.rois;
    }
};
struct GraphEntry {
    GraphKey key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *drd = nullptr;        // device copy of the ROI descriptors
    hipEvent_t done = nullptr;  // recorded after every launch
    uint64_t last_use = 0;
};
constexpr size_t kGraphs = 16;  // cached graphs (least recently used goes first)
constexpr size_t kSeen = 64;    // remembered first sightings
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
std::vector<uint64_t> g_seen;
uint64_t g_graph_tick = 0;

bool graphs_enabled() {
    const char *e = std::getenv("DPM_NO_GRAPH");
    return !(e && atoi(e)) && !batched_profiling();
}

uint64_t key_hash(const GraphKey &k) {
    uint64_t h = 1469598103934665603ull;  // FNV-1a
    auto mix = [&](const void *p, size_t n) {
        const uint8_t *b = static_cast<const uint8_t *>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    };
    mix(&k.dev, sizeof k.dev);
    mix(&k.n, sizeof k.n);
    mix(&k.K, sizeof k.K);
    mix(&k.tune_gen, sizeof k.tune_gen);
    mix(&k.packed, sizeof k.packed);
    mix(&k.exact, sizeof k.exact);
    mix(&k.fp64, sizeof k.fp64);
    mix(&k.ws, sizeof k.ws);
    mix(&k.ws_bytes, sizeof k.ws_bytes);
    mix(k.rois.data(), k.rois.size());
    return h;
}

// true if this hash was seen before (then forgotten); else remembered.  Caller holds
// g_graph_mu.
bool seen_before(uint64_t h) {
    auto it = std::find(g_seen.begin(), g_seen.end(), h);
    if (it != g_seen.end()) {
        g_seen.erase(it);
        return true;
    }
    if (g_seen.size() >= kSeen) g_seen.erase(g_seen.begin());
    g_seen.push_back(h);
    return false;
}

void destroy_entry(GraphEntry &g) {
    if (g.done) (void)hipEventSynchronize(g.done);
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    if (g.drd) (void)hipFree(g.drd);
    if (g.done) (void)hipEventDestroy(g.done);
    g = GraphEntry{};
}

// Captures the call on a private stream, caches it and launches it on st.  false: the
// graph could not be made (nothing was launched; the caller runs the call eagerly).
bool build_and_launch_graph(const GraphKey &key, const BPlan &p, const PowTab &pt, const uint8_t *packed,
                            uint8_t *ws, const dpm_out *out, hipStream_t st) {
    GraphEntry g;
    g.key = key;
    const size_t brd = sizeof(RoiDesc) * p.rd.size();
    if (hipMalloc(&g.drd, brd) != hipSuccess) return false;
    if (hipMemcpy(g.drd, p.rd.data(), brd, hipMemcpyHostToDevice) != hipSuccess ||
        hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) {
        destroy_entry(g);
        return false;
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        destroy_entry(g);
        return false;
    }
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t el = enqueue(p, pt, packed, static_cast<RoiDesc *>(g.drd), ws, out, cs, false);
        e = hipStreamEndCapture(cs, &g.graph);
        if (el != hipSuccess) e = el;
    }
    (void)hipStreamDestroy(cs);
    if (e == hipSuccess && g.graph) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess || !g.exec) {
        (void)hipGetLastError();
        destroy_entry(g);
        return false;
    }
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (g_graphs.size() >= kGraphs) {
        auto victim = std::min_element(g_graphs.begin(), g_graphs.end(),
                                       [](const GraphEntry &a, const GraphEntry &b) { return a.last_use < b.last_use; });
        destroy_entry(*victim);
        g_graphs.erase(victim);
    }
    g.last_use = ++g_graph_tick;
    e = hipGraphLaunch(g.exec, st);
    if (e == hipSuccess) e = hipEventRecord(g.done, st);
    if (e != hipSuccess) {
        // not cached; clear the error so that the caller's eager launch starts clean (a
        // real device fault shows again there)
        batched_set_error((int)e);
        (void)hipGetLastError();
        destroy_entry(g);
        return false;
    }
    g_graphs.push_back(g);
    return true;
}

}  // namespace

namespace dpm {
// Where a batched call leaves ROI i's power-sum tiles: byte offsets (in the workspace) of
// the tile partials and of the ROI's device descriptor, and the limbs.
int batched_partials(const dpm_roi *rois, int n_rois, int max_order, int i, size_t *part_off, size_t *rd_off,
                     int *nlr) {
    BPlan p;
    int rc = bplan(rois, n_rois, max_order, p);
    if (rc) return rc;
    if (i < 0 || i >= n_rois) return DPM_EINVAL;
    *part_off = p.off_part;
    *rd_off = p.off_rd + sizeof(RoiDesc) * (size_t)i;
    *nlr = p.nlr;
    return DPM_OK;
}

// Frees the pinned staging buffers (called by dpm_release).
int batched_release() {
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (auto &g : g_graphs) destroy_entry(g);
        g_graphs.clear();
        g_seen.clear();
    }
    std::lock_guard<std::mutex> lk(g_stage_mu);
    int rc = DPM_OK;
    for (auto &s : g_stage) {
        if (hipEventSynchronize(s.ev) != hipSuccess) rc = DPM_EDEVICE;
        (void)hipEventDestroy(s.ev);
        if (hipHostFree(s.p) != hipSuccess) rc = DPM_EDEVICE;
    }
    g_stage.clear();
    return rc;
}
}  // namespace dpm

extern "C" {

size_t dpm_batched_workspace_bytes(const dpm_roi *rois, int n_rois, int max_order) {
    BPlan p;
    if (bplan(rois, n_rois, max_order, p)) return 0;
    return p.total;
}

int dpm_moments_batched(const void *packed, const dpm_roi *rois, int n_rois, int max_order,
                        const dpm_out *out_device, void *workspace, size_t ws_bytes, void *stream) {
    return dpm::batched_run(packed, rois, n_rois, max_order, out_device, workspace, ws_bytes, stream, true);
}

int dpm_batch_tune_set(int max_order, const dpm_batch_tuning *t) {
    if (max_order < 0 || max_order > 6) return DPM_EINVAL;
    if (t && (t->fused < -1 || t->fused > 0 || t->units < 0 || t->units > 16 ||
              (t->max_spw != 0 && t->max_spw != 1 && t->max_spw != 2 && t->max_spw != 4)))
        return DPM_EINVAL;
    std::lock_guard<std::mutex> lk(g_btune_mu);
    g_btune[max_order] = t ? *t : dpm_batch_tuning{};
    ++g_btune_gen;
    return DPM_OK;
}

int dpm_batched_graph_count(void) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    return (int)g_graphs.size();
}

}  // extern "C"

namespace dpm {
// The batched call; `graphs`: whether a repeated call may be captured and replayed (the
// served loop passes false: its batches rarely repeat, and a capture's synchronous
// allocation would stall its worker).
int batched_run(const void *packed, const dpm_roi *rois, int n_rois, int max_order, const dpm_out *out_device,
                void *workspace, size_t ws_bytes, void *stream, bool allow_graphs) {
    if (!packed || !out_device || !workspace) return DPM_EINVAL;
    int rc = batched_ensure_tables();
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    const bool graphs = allow_graphs && graphs_enabled() && rois && n_rois > 0 && max_order >= 0 && max_order <= 6;
    GraphKey key;
    bool repeat = false;
    if (graphs) {
        if ((e = hipGetDevice(&key.dev)) != hipSuccess) {
            batched_set_error((int)e);
            return DPM_EDEVICE;
        }
        key.n = n_rois;
        key.K = max_order;
        (void)batch_tuning(max_order, &key.tune_gen);
        key.packed = packed;
        key.exact = out_device->exact;
        key.fp64 = out_device->fp64;
        key.ws = workspace;
        key.ws_bytes = ws_bytes;
        key.rois.assign(reinterpret_cast<const uint8_t *>(rois),
                        reinterpret_cast<const uint8_t *>(rois) + sizeof(dpm_roi) * (size_t)n_rois);
        key.hash = key_hash(key);
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
            if (it->key == key) {
                // a repeated call: replay its graph (no planning, no descriptor upload)
                it->last_use = ++g_graph_tick;
                e = hipGraphLaunch(it->exec, st);
                if (e == hipSuccess) e = hipEventRecord(it->done, st);
                if (e == hipSuccess) return DPM_OK;
                // drop the graph and run the call eagerly below
                batched_set_error((int)e);
                (void)hipGetLastError();
                destroy_entry(*it);
                g_graphs.erase(it);
                break;
            }
        if (e == hipSuccess) repeat = seen_before(key.hash);
    }
    BPlan p;
    if ((rc = bplan(rois, n_rois, max_order, p))) return rc;
    if (ws_bytes < p.total) return DPM_ENOMEM;
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    PowTab pt{};
    if (p.mfma && (rc = batched_powtab(p.amax, max_order, pt))) return rc;
    if (repeat && build_and_launch_graph(key, p, pt, static_cast<const uint8_t *>(packed), ws, out_device, st))
        return DPM_OK;
    RoiDesc *drd = reinterpret_cast<RoiDesc *>(ws + p.off_rd);
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        int dev = 0;
        e = hipGetDevice(&dev);
        const size_t brd = sizeof(RoiDesc) * p.rd.size();
        Staging *sg = e == hipSuccess ? stage_acquire(brd, dev) : nullptr;
        if (!sg) return e == hipSuccess ? DPM_ENOMEM : (batched_set_error((int)e), DPM_EDEVICE);
        std::memcpy(sg->p, p.rd.data(), brd);
        e = hipMemcpyAsync(drd, sg->p, brd, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventRecord(sg->ev, st);
    }
    if (e == hipSuccess) e = enqueue(p, pt, static_cast<const uint8_t *>(packed), drd, ws, out_device, st, true);
    if (e != hipSuccess) {
        batched_set_error((int)e);
        return DPM_EDEVICE;
    }
    return DPM_OK;
}
}  // namespace dpm
