// C ABI of libdpm: argument checking, planning (bounds, integer widths, launch
// geometry, LDS layout), workspace management and the launch sequence
//   projection + row power sums  ->  y reduction  ->  recombination.
// See include/dpm.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/dpm.h"
#include "dpm_common.h"
#include "kernels.h"
#include "mw.h"

namespace {

using namespace dpm;

thread_local int g_last_hip_error = 0;

int hip_fail(hipError_t e) {
    g_last_hip_error = (int)e;
    return DPM_EDEVICE;
}

int bitlen_u64(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// ------------------------------------------------------------------ tables
std::recursive_mutex g_mu;  // recursive: planning helpers also take it
RecombTables g_tables;
bool g_tables_ok = false;
bool g_tables_built = false;
bool g_dev_uploaded[64] = {};

bool host_tables() {
    if (!g_tables_built) {
        g_tables_ok = build_recomb_tables(g_tables);
        g_tables_built = true;
    }
    return g_tables_ok;
}

int ensure_device_tables() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!host_tables()) return DPM_ERANGE;
    if (dev >= 0 && dev < 64 && g_dev_uploaded[dev]) return DPM_OK;
    e = upload_recomb_tables(g_tables);
    if (e != hipSuccess) return hip_fail(e);
    if (dev >= 0 && dev < 64) g_dev_uploaded[dev] = true;
    return DPM_OK;
}

// ------------------------------------------------------------------ MFMA power tables
// Limbs (7 bits) of a^k for a in [0, amax), k <= K, laid out as the B operand of
// v_mfma_i32_16x16x64_i8 (see PowTab).  Built once per (device, amax, K).
struct PowKey {
    int dev, amax, K;
    bool operator<(const PowKey &o) const {
        return dev != o.dev ? dev < o.dev : amax != o.amax ? amax < o.amax : K < o.K;
    }
};
std::map<PowKey, PowTab> g_pow;

// columns of a^k: 1 for k = 0, else ceil(bits((amax-1)^k) / 7)
int bitlen_mw(const mw::Int<8> &v) {
    for (int l = 7; l >= 0; --l)
        if (v.w[l]) return 32 * l + 32 - __builtin_clz(v.w[l]);
    return 0;
}

bool pow_columns(int amax, int K, int32_t colstart[KMAX + 2]) {
    mw::Int<8> p;
    mw::set_u64(p, 1);
    int c = 0;
    for (int k = 0; k <= K; ++k) {
        colstart[k] = c;
        if (k == 0) {
            c += 1;
        } else {
            mw::mul_u32(p, (uint32_t)(amax - 1));
            const int b = bitlen_mw(p);
            c += b == 0 ? 1 : (b + 6) / 7;
        }
    }
    colstart[K + 1] = c;
    return amax <= 65536;
}

int get_powtab(int amax, int K, PowTab &out) {
    // one table per 512 values of a: a table serves every shorter row, so a stream of
    // mixed shapes builds few tables (each build allocates and copies synchronously)
    amax = (amax + 511) / 512 * 512;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    auto it = g_pow.find(PowKey{dev, amax, K});
    if (it != g_pow.end()) {
        out = it->second;
        return DPM_OK;
    }
    PowTab t{};
    if (!pow_columns(amax, K, t.colstart)) return DPM_ENOTSUP;
    const int ncol = t.colstart[K + 1];
    t.amax = amax;
    t.nt = (ncol + 15) / 16;
    const int nks = amax / 64;
    std::vector<uint8_t> h((size_t)nks * t.nt * 64 * 16, 0);
    std::vector<int> colk(ncol), colu(ncol);
    for (int k = 0; k <= K; ++k)
        for (int c = t.colstart[k]; c < t.colstart[k + 1]; ++c) {
            colk[c] = k;
            colu[c] = c - t.colstart[k];
        }
    for (int a = 0; a < amax; ++a) {
        const int ks = a / 64, kq = (a % 64) / 16, i = a % 16;
        mw::Int<8> pw[KMAX + 1];
        mw::set_u64(pw[0], 1);
        for (int k = 1; k <= K; ++k) {
            pw[k] = pw[k - 1];
            mw::mul_u32(pw[k], (uint32_t)a);
        }
        for (int col = 0; col < ncol; ++col) {
            const int bit = 7 * colu[col];
            const mw::Int<8> &v = pw[colk[col]];
            const uint32_t lo = v.w[bit >> 5] >> (bit & 31);
            const uint32_t hi = ((bit >> 5) + 1 < 8 && (bit & 31)) ? v.w[(bit >> 5) + 1] << (32 - (bit & 31)) : 0u;
            const int tile = col / 16, lane = kq * 16 + (col % 16);
            h[(((size_t)ks * t.nt + tile) * 64 + lane) * 16 + i] = (uint8_t)((lo | hi) & 0x7f);
        }
    }
    void *d = nullptr;
    e = hipMalloc(&d, h.size());
    if (e != hipSuccess) {
        g_last_hip_error = (int)e;
        return DPM_ENOMEM;
    }
    e = hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    t.b = static_cast<const uint4 *>(d);
    g_pow[PowKey{dev, amax, K}] = t;
    out = t;
    return DPM_OK;
}

// ------------------------------------------------------------------ stage timing
constexpr int NPROF = 4;  // start, after projection, after power sums, end
struct StageEvents {
    hipEvent_t e[NPROF];
};
bool g_prof_on = false;
std::vector<StageEvents> g_prof;

// Record event `idx` of the current call (creates the call's events at idx 0).
void prof_mark(int idx, hipStream_t st) {
    if (!g_prof_on) return;
    if (idx == 0) {
        StageEvents ev{};
        for (int i = 0; i < NPROF; ++i) (void)hipEventCreate(&ev.e[i]);
        g_prof.push_back(ev);
    }
    if (!g_prof.empty()) (void)hipEventRecord(g_prof.back().e[idx], st);
}

// ------------------------------------------------------------------ planning
struct Plan {
    int K = 0, nd = 0, elem = 0;
    int64_t L = 0, M = 0, N = 0;
    int zsplits = 1, zrows = 0, items = 0;
    int R = 8, CT = 1;
    bool fast = false;
    bool chain = false;  // chained-window projection (first group)
    int nls = 4, nlr = 4;
    int ngroups = 0;
    int gnd[NGROUP] = {};
    size_t lds[NGROUP] = {};
    int jobbins = 512;
    int npairs = 0;
    int bits_slice = 0, bits_moment = 0;
    bool mfma = false;   // power sums on the matrix cores
    int pow_passes = 0;  // column-tile passes of the matrix-core power kernel
    dpm_tuning tune{};   // override of this shape (dpm_tune_set), zero if none
    bool one_launch = false;  // orders 7-16: all direction groups in one projection launch
    int waves = 4;            // waves per projection workgroup (first group, whole rows)
    int amax = 0;        // coordinate magnitudes covered by the power table
    RowLayout rl{};
    int nslots_used = 0;
    uint64_t slot_mask = 0;
    size_t rows_bytes = 0;
    int ntiles = 0;       // power-sum tiles: non-empty slots x ceil(items / 16)
    size_t part_bytes = 0, ws_bytes = 0;
};

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int elem_of(dpm_dtype t) { return t == DPM_U8 ? 1 : t == DPM_U16 ? 2 : 0; }

// Lane layout along x for a row of L voxels: sub-rows of R lanes (power of two in
// [8, 64]) or 64-lane column tiles.
void lane_layout(int64_t L, int G, int &R, int &CT) {
    const int64_t lanes = (L + G - 1) / G;
    if (lanes <= 64) {
        int r = 8;
        while (r < lanes) r <<= 1;
        R = r;
        CT = 1;
    } else {
        R = 64;
        CT = (int)((lanes + 63) / 64);
    }
}

// Bounds that decide the integer widths (all in bits).
int plan_widths(Plan &p) {
    const uint64_t vmax = p.elem == 1 ? 255u : 65535u;
    int64_t umax = 1;
    for (int d = 0; d < p.nd; ++d) {
        const int64_t u = (int64_t)dir_alpha(d) * (p.L - 1) + (int64_t)iabs_c(dir_beta(d)) * (p.N - 1);
        umax = std::max(umax, u);
    }
    if (umax >= (int64_t)1 << 30) return DPM_ERANGE;
    // a projection pixel sums at most max(L, N) voxels and must fit 32 bits
    const int64_t line = std::max(p.L, p.N);
    if ((double)vmax * (double)line >= 4294967296.0) return DPM_ERANGE;
    const int bu = bitlen_u64((uint64_t)umax);
    const int by = bitlen_u64((uint64_t)std::max<int64_t>(p.M - 1, 1));
    const int bslice = bitlen_u64(vmax) + bitlen_u64((uint64_t)(p.L * p.zrows)) + p.K * bu + 1;
    const int bvol = bitlen_u64(vmax) + bitlen_u64((uint64_t)(p.L * p.M * p.N));
    int brec = 0;
    for (int k = 0; k <= p.K; ++k)
        for (int q = 0; k + q <= p.K; ++q)
            brec = std::max(brec, bvol + k * bu + q * by + g_tables.numsum_bits[k] + 2);
    p.bits_slice = bslice;
    p.bits_moment = brec;
    if (bslice <= 128) p.nls = 4;
    else if (bslice <= 256) p.nls = 8;
    else return DPM_ERANGE;
    if (brec <= 128) p.nlr = 4;
    else if (brec <= 256) p.nlr = 8;
    else if (brec <= 384) p.nlr = 12;
    else return DPM_ERANGE;
    if (p.nlr < p.nls) p.nlr = p.nls;
    // orders <= 4 are returned as int128
    const int64_t cmax = std::max(std::max(p.L, p.M), p.N) - 1;
    const int b4 = bvol + std::min(p.K, 4) * bitlen_u64((uint64_t)std::max<int64_t>(cmax, 1)) + 1;
    if (b4 > 127) return DPM_ERANGE;
    return DPM_OK;
}

// ---- per-shape tuning overrides (dpm_tune_set)
struct TuneKey {
    int64_t L, M, N;
    int elem, K;
    bool operator<(const TuneKey &o) const {
        return std::tie(L, M, N, elem, K) < std::tie(o.L, o.M, o.N, o.elem, o.K);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, dpm_tuning> g_tune;

bool tune_lookup(const Plan &p, dpm_tuning &t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(TuneKey{p.L, p.M, p.N, p.elem, p.K});
    if (it == g_tune.end()) return false;
    t = it->second;
    return true;
}

int make_plan(const int64_t dims[3], dpm_dtype dtype, int K, bool full_rows, Plan &p,
              const void *vol_for_alignment) {
    if (!dims) return DPM_EINVAL;
    if (K < 0 || K > KMAX) return DPM_EINVAL;
    p.elem = elem_of(dtype);
    if (!p.elem) return DPM_EINVAL;
    p.L = dims[0];
    p.M = dims[1];
    p.N = dims[2];
    if (p.L <= 0 || p.M <= 0 || p.N <= 0) return DPM_EINVAL;
    if (p.L > (1 << 24) || p.M > (1 << 24) || p.N > (1 << 24)) return DPM_ERANGE;
    p.K = K;
    p.nd = K + 1;
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        if (!host_tables()) return DPM_ERANGE;
    }
    // z-splits: enough work items to fill the GPU, each at least 64 rows
    int zs = 1;
    if (!full_rows) {
        const int64_t want = 512;
        if (p.M < want) zs = (int)std::min<int64_t>((want + p.M - 1) / p.M, std::max<int64_t>(1, p.N / 64));
        if (tune_lookup(p, p.tune) && p.tune.z_splits > 0) zs = p.tune.z_splits;
        if (const char *e = std::getenv("DPM_ZSPLITS")) zs = std::max(1, atoi(e));
    }
    int64_t zrows = (p.N + zs - 1) / zs;
    zrows = (zrows + ZALIGN - 1) / ZALIGN * ZALIGN;
    p.zrows = (int)zrows;
    p.zsplits = (int)((p.N + zrows - 1) / zrows);
    if ((int64_t)p.M * p.zsplits > INT32_MAX / 2) return DPM_ERANGE;
    p.items = (int)(p.M * p.zsplits);
    int rc = plan_widths(p);
    if (rc) return rc;
    const int G = lane_voxels(p.elem);
    lane_layout(p.L, G, p.R, p.CT);
    const int64_t lanes = (p.L + G - 1) / G;
    const bool lanes_exact = (lanes == (int64_t)p.R * p.CT);
    const uintptr_t addr = (uintptr_t)vol_for_alignment;
    const size_t vec_bytes = p.elem == 2 ? 16 : 8;  // one lane's load
    p.fast = lanes_exact && (p.L % G == 0) && (p.N % ZALIGN == 0) && (addr % vec_bytes == 0);
    if (const char *e = std::getenv("DPM_FORCE_GENERIC")) {
        if (atoi(e)) p.fast = false;
    }

    // chained-window projection: opt-in (it is exact, but measured slower than the
    // windowed kernel on the 512^3 workload)
    p.chain = false;
    if (const char *e = std::getenv("DPM_CHAIN")) {
        if (atoi(e)) p.chain = p.fast && p.elem == 2 && p.R == 64 && p.zrows % 32 == 0 && p.N % 32 == 0;
    }
    p.npairs = n_pairs(K);
    // groups, LDS per group and the row layout (the first item is the largest; the
    // last one may differ)
    const int64_t firsts[2] = {0, (int64_t)(p.zsplits - 1) * p.zrows};
    p.ngroups = 0;
    int64_t lens[NSLOT] = {};
    for (int g = 0; g < NGROUP; ++g) {
        const int b = group_begin(g), e = std::min(group_end(g), p.nd);
        if (e <= b) break;
        p.gnd[g] = e - b;
        ++p.ngroups;
        size_t best = 0;
        for (int s = 0; s < 2; ++s) {
            const int64_t zs0 = firsts[s], ze0 = std::min<int64_t>(zs0 + p.zrows, p.N);
            ItemGeom ig;
            item_geometry(g, p.gnd[g], G, p.L, p.N, zs0, ze0, ig);
            best = std::max(best, (size_t)ig.lds_dwords * 4);
            for (int i = 0; i < p.gnd[g]; ++i)
                for (int side = 0; side < 2; ++side)
                    if (ig.seg_ahi[2 * i + side] >= ig.seg_alo[2 * i + side])
                        lens[2 * (b + i) + side] = std::max<int64_t>(lens[2 * (b + i) + side], ig.seg_ahi[2 * i + side] + 1);
        }
        p.lds[g] = best;
        if (best > 160 * 1024) return DPM_ERANGE;
    }
    p.one_launch = p.fast && p.ngroups > 1;
    p.waves = (p.fast && p.tune.waves != 4) ? 8 : 4;
    if (const char *e = std::getenv("DPM_SLICE_WAVES")) {
        if (atoi(e) == 8 && p.fast) p.waves = 8;
        if (atoi(e) == 4) p.waves = 4;
    }
    if (const char *e = std::getenv("DPM_GROUP_LAUNCHES")) {
        if (atoi(e)) p.one_launch = false;
    }
    int64_t off = 0, amax = 64;
    for (int sl = 0; sl < NSLOT; ++sl) {
        const int32_t len = lens[sl] ? round64(lens[sl]) : 0;
        p.rl.slot_off[sl] = (int32_t)off;
        p.rl.slot_len[sl] = len;
        if (len) {
            ++p.nslots_used;
            p.slot_mask |= (uint64_t)1 << sl;
        }
        off += len;
        amax = std::max<int64_t>(amax, len);
    }
    p.rl.row_stride = off;
    p.rows_bytes = align_up((size_t)p.items * off * 4);
    {
        // matrix-core power sums: row values below 2^28 (4 limbs of 7 bits)
        const uint64_t vmax = p.elem == 1 ? 255u : 65535u;
        const bool small_p = (double)vmax * (double)std::max<int64_t>(p.L, p.zrows) < 268435456.0;
        int32_t cs[KMAX + 2];
        p.mfma = small_p && amax <= 8192 && pow_columns((int)amax, p.K, cs);
        p.pow_passes = p.mfma ? (cs[p.K + 1] + 63) / 64 : 0;  // 4 column tiles of 16 per pass
        if (const char *e = std::getenv("DPM_NO_MFMA")) {
            if (atoi(e)) p.mfma = false;
        }
        p.amax = (int)amax;
    }
    {
        // power-sum tiles; on the matrix cores with all power columns in one pass, each
        // covers at most kchunk steps of 64 values of a, so long rows spread over more
        // workgroups (with several passes the per-tile reassembly dominates: no chunks)
        int kc = (p.mfma && p.pow_passes == 1) ? 8 : (1 << 30);
        if (p.mfma && p.tune.power_chunk != 0) kc = p.tune.power_chunk > 0 ? p.tune.power_chunk : (1 << 30);
        if (const char *e = std::getenv("DPM_PW_KCHUNK")) {
            if (atoi(e) > 0 && p.mfma) kc = atoi(e);
        }
        const int32_t ipt = (int32_t)((p.items + 15) / 16);
        p.rl.kchunk = kc;
        p.rl.tile0[0] = 0;
        for (int sl = 0; sl < NSLOT; ++sl) {
            const int32_t nks = p.rl.slot_len[sl] / 64;
            p.rl.nck[sl] = nks ? (nks + kc - 1) / kc : 0;
            p.rl.tile0[sl + 1] = p.rl.tile0[sl] + ipt * p.rl.nck[sl];
        }
        p.ntiles = p.rl.tile0[NSLOT];
    }
    p.part_bytes = align_up((size_t)p.ntiles * (K + 1) * (K + 1) * p.nlr * 4);
    p.ws_bytes = p.rows_bytes + p.part_bytes;
    return DPM_OK;
}

// ------------------------------------------------------------------ workspaces
int ensure_buf(void *&ptr, size_t &have, size_t need) {
    if (have >= need && ptr) return DPM_OK;
    if (ptr) {
        hipError_t e = hipFree(ptr);
        if (e != hipSuccess) return hip_fail(e);
        ptr = nullptr;
        have = 0;
    }
    hipError_t e = hipMalloc(&ptr, need);
    if (e != hipSuccess) {
        ptr = nullptr;
        g_last_hip_error = (int)e;
        return DPM_ENOMEM;
    }
    have = need;
    return DPM_OK;
}

struct DevWs {
    void *ptr = nullptr;
    size_t bytes = 0;
    void *out = nullptr;  // device staging for dpm_moments results
    size_t out_bytes = 0;
    hipEvent_t done = nullptr;  // recorded after the last work that used this workspace
    bool used = false;
};
DevWs g_ws[64];

// The library-owned workspace of a device is shared by every call that does not bring
// its own.  Calls on different streams must not overlap on it: each user's stream first
// waits for the event recorded after the previous user's work (ws_begin), and records it
// again after its own (ws_end).  Both run under g_mu.
int ws_begin(int dev, hipStream_t st) {
    DevWs &w = g_ws[dev];
    if (!w.done) {
        hipError_t e = hipEventCreateWithFlags(&w.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            w.done = nullptr;
            return hip_fail(e);
        }
    }
    if (w.used) {
        hipError_t e = hipStreamWaitEvent(st, w.done, 0);
        if (e != hipSuccess) return hip_fail(e);
    }
    return DPM_OK;
}

int ws_end(int dev, hipStream_t st) {
    DevWs &w = g_ws[dev];
    hipError_t e = hipEventRecord(w.done, st);
    if (e != hipSuccess) return hip_fail(e);
    w.used = true;
    return DPM_OK;
}

// Grow a buffer of the shared workspace: the old one may still be read by work in
// flight on another stream, so wait for that work before freeing it.
int ensure_ws_buf(int dev, void *&ptr, size_t &have, size_t need) {
    if (have >= need && ptr) return DPM_OK;
    if (ptr && g_ws[dev].used) {
        hipError_t e = hipEventSynchronize(g_ws[dev].done);
        if (e != hipSuccess) return hip_fail(e);
    }
    return ensure_buf(ptr, have, need);
}


// given_pow: a power table the caller built (the allocation-free entry point), else the
// library's cached one; such calls record no stage events either.
int run_plan(const Plan &p, const void *vol, int32_t *images, const int64_t *img_off,
             const int64_t *img_w, void *exact, double *fp64, void *ws, hipStream_t st,
             uint32_t *raw = nullptr, const ImgArgs *from_images = nullptr,
             const PowTab *given_pow = nullptr) {
    uint8_t *base = static_cast<uint8_t *>(ws);
    int32_t *rows = reinterpret_cast<int32_t *>(base);
    uint32_t *part = reinterpret_cast<uint32_t *>(base + p.rows_bytes);
    PowTab pt{};
    const bool moments = (exact || fp64 || raw);
    if (given_pow) {
        pt = *given_pow;
    } else if (p.mfma && moments) {
        int prc = get_powtab(p.amax, p.K, pt);
        if (prc) return prc;
    }
    auto mark = [&](int idx) {
        if (!given_pow) prof_mark(idx, st);
    };
    if (moments) mark(0);
    if (from_images) {
        // step 1 replaced by supplied images: gather them into the row slots
        ImgArgs ia = *from_images;
        ia.rows = rows;
        ia.rl = p.rl;
        hipError_t e = launch_images_to_rows(ia, st);
        if (e != hipSuccess) return hip_fail(e);
    } else if (p.one_launch && !images) {
        // orders 7-16: every direction group in one launch, sibling workgroups per item
        SliceArgs a{};
        a.vol = static_cast<const uint8_t *>(vol);
        a.L = p.L;
        a.M = p.M;
        a.N = p.N;
        a.pitch_y = p.L;
        a.pitch_z = p.L * p.M;
        a.zsplits = p.zsplits;
        a.zrows = p.zrows;
        a.R = p.R;
        a.CT = p.CT;
        a.rows = rows;
        a.rl = p.rl;
        size_t lds = 0;
        for (int g = 0; g < p.ngroups; ++g) lds = std::max(lds, p.lds[g]);
        hipError_t e = launch_slice_groups(p.elem, p.nd, a, p.items, lds, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    for (int g = 0; g < p.ngroups && !from_images && !(p.one_launch && !images); ++g) {
        SliceArgs a{};
        a.vol = static_cast<const uint8_t *>(vol);
        a.L = p.L;
        a.M = p.M;
        a.N = p.N;
        a.pitch_y = p.L;
        a.pitch_z = p.L * p.M;
        a.zsplits = p.zsplits;
        a.zrows = p.zrows;
        a.R = p.R;
        a.CT = p.CT;
        a.rows = rows;
        a.rl = p.rl;
        a.images = images;
        a.waves = p.waves;
        for (int i = 0; i < 7; ++i) {
            a.img_off[i] = (images && i < p.gnd[g]) ? img_off[group_begin(g) + i] : 0;
            a.img_w[i] = (images && i < p.gnd[g]) ? img_w[group_begin(g) + i] : 0;
        }
        hipError_t e = launch_slice(p.elem, p.fast, p.chain && g == 0, g, p.gnd[g], a, p.items, p.lds[g], st);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (!moments) return DPM_OK;
    PowerArgs pa{};
    pa.rows = rows;
    pa.rl = p.rl;
    pa.rois = nullptr;
    pa.nitems = p.items;
    pa.zsplits = p.zsplits;
    pa.K = p.K;
    pa.ntiles = p.ntiles;
    for (int s = 0; s < NSLOT; ++s) pa.max_len = std::max(pa.max_len, p.rl.slot_len[s]);
    pa.pow = pt;
    pa.part = part;
    mark(1);
    hipError_t e = launch_power(p.nls, p.nlr, pa, st);
    if (e != hipSuccess) return hip_fail(e);
    mark(2);
    FinishArgs f{};
    f.part = part;
    f.rois = nullptr;
    f.nvol = 1;
    f.K = p.K;
    for (int s = 0; s <= NSLOT; ++s) f.tile0[s] = p.rl.tile0[s];
    f.exact = exact;
    f.fp64 = fp64;
    f.raw = raw;
    e = launch_finish(p.nlr, f, st);
    if (e != hipSuccess) return hip_fail(e);
    mark(3);
    return DPM_OK;
}

int current_device(int &dev) {
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= 64) return DPM_ENOTSUP;
    return DPM_OK;
}

}  // namespace

namespace dpm {
// The launch sequence of dpm_moments_async with every device buffer taken from one
// caller-supplied region `scratch` (the allocation-free entry point): the power table of
// the matrix-core power sums is built there by a kernel on `st` (first), followed by the
// workspace.  Nothing is allocated.  *need = the bytes this request uses; DPM_ENOMEM if
// they exceed scratch_bytes (nothing is enqueued then).
int moments_in_scratch(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                       const dpm_out *out_device, uint8_t *scratch, size_t scratch_bytes, hipStream_t st,
                       size_t *need) {
    if (need) *need = 0;
    if (!volume || !out_device || !scratch) return DPM_EINVAL;
    if (int trc = ensure_device_tables()) return trc;
    Plan p;
    int rc = make_plan(dims, dtype, max_order, false, p, volume);
    if (rc) return rc;
    PowTab t{};
    size_t tab_bytes = 0;
    if (p.mfma) {
        t.amax = (p.amax + 511) / 512 * 512;
        if (!pow_columns(t.amax, p.K, t.colstart)) return DPM_ENOTSUP;
        t.nt = (t.colstart[p.K + 1] + 15) / 16;
        tab_bytes = align_up((size_t)(t.amax / 64) * t.nt * 64 * 16);
    }
    const size_t total = tab_bytes + p.ws_bytes;
    if (need) *need = total;
    if (total > scratch_bytes) return DPM_ENOMEM;
    if (p.mfma) {
        uint4 *tab = reinterpret_cast<uint4 *>(scratch);
        hipError_t e = launch_powtab_build(tab, t, p.K, st);
        if (e != hipSuccess) return hip_fail(e);
        t.b = tab;
    }
    return run_plan(p, volume, nullptr, nullptr, nullptr, out_device->exact, out_device->fp64, scratch + tab_bytes,
                    st, nullptr, nullptr, &t);
}

// The K+1 projection images of the family (the layout of dpm_project_images) into
// `images`, with the projection's own rows/partials in `ws`; used by the 1D-integral
// route.  *ws_need = the bytes ws must hold (query with images == null).
int family_images(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order, int32_t *images,
                  void *ws, size_t ws_bytes, hipStream_t st, size_t *ws_need) {
    if (int trc = ensure_device_tables()) return trc;
    Plan p;
    int rc = make_plan(dims, dtype, max_order, true, p, volume);
    if (rc) return rc;
    if (ws_need) *ws_need = p.ws_bytes;
    if (!images) return DPM_OK;
    if (!volume || !ws || ws_bytes < p.ws_bytes) return DPM_EINVAL;
    int64_t off[NDIR_MAX], w[NDIR_MAX];
    int64_t acc = 0;
    for (int d = 0; d < p.nd; ++d) {
        w[d] = dpm_image_width(dims, d);
        off[d] = acc;
        acc += w[d] * p.M;
    }
    return run_plan(p, volume, images, off, w, nullptr, nullptr, ws, st);
}

// Where a dpm_moments_async call of this request leaves its power-sum tiles in the
// workspace: byte offset of the tile partials, the tile range of every slot and the limbs.
int single_partials(const int64_t dims[3], dpm_dtype dtype, int max_order, size_t *part_off,
                    int32_t tile0[NSLOT + 1], int *nlr) {
    Plan p;
    int rc = make_plan(dims, dtype, max_order, false, p, nullptr);
    if (rc) return rc;
    *part_off = p.rows_bytes;
    for (int s = 0; s <= NSLOT; ++s) tile0[s] = p.rl.tile0[s];
    *nlr = p.nlr;
    return DPM_OK;
}

int batched_release();  // batched.cpp
int batched_powtab(int amax, int K, PowTab &out) { return get_powtab(amax, K, out); }
bool batched_pow_columns(int amax, int K, int32_t colstart[KMAX + 2]) { return pow_columns(amax, K, colstart); }
void batched_prof_mark(int idx, hipStream_t st) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    prof_mark(idx, st);
}
bool batched_profiling() {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    return g_prof_on;
}
int batched_ensure_tables() { return ensure_device_tables(); }
int batched_numsum_bits(int k) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    host_tables();
    return g_tables.numsum_bits[k];
}
void batched_set_error(int e) { g_last_hip_error = e; }
}  // namespace dpm

// ====================================================================== C ABI
extern "C" {

int dpm_num_moments(int max_order) {
    if (max_order < 0 || max_order > KMAX) return -1;
    return n_moments(max_order);
}

int dpm_moment_index(int p, int q, int r) {
    if (p < 0 || q < 0 || r < 0 || p + q + r > KMAX) return -1;
    return moment_index(p, q, r);
}

const char *dpm_strerror(int status) {
    switch (status) {
        case DPM_OK: return "success";
        case DPM_EINVAL: return "invalid argument";
        case DPM_ERANGE: return "volume or order outside the exact integer range of the library";
        case DPM_ENOMEM: return "workspace too small or allocation failed";
        case DPM_EDEVICE: return "HIP runtime error";
        case DPM_ENOTSUP: return "not supported";
        default: return "unknown status";
    }
}

int dpm_last_device_error(void) { return g_last_hip_error; }

int dpm_direction(int d, int *alpha, int *beta) {
    if (d < 0 || d > KMAX || !alpha || !beta) return DPM_EINVAL;
    *alpha = dir_alpha(d);
    *beta = dir_beta(d);
    return DPM_OK;
}

int64_t dpm_image_width(const int64_t dims[3], int d) {
    if (!dims || d < 0 || d > KMAX || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0) return 0;
    return (int64_t)dir_alpha(d) * (dims[0] - 1) + (int64_t)iabs_c(dir_beta(d)) * (dims[2] - 1) + 1;
}

size_t dpm_workspace_bytes(const int64_t dims[3], dpm_dtype dtype, int max_order) {
    Plan p;
    if (make_plan(dims, dtype, max_order, false, p, nullptr)) return 0;
    return p.ws_bytes;
}

int dpm_plan(const int64_t dims[3], dpm_dtype dtype, int max_order, dpm_plan_info *info) {
    if (!info) return DPM_EINVAL;
    Plan p;
    int rc = make_plan(dims, dtype, max_order, false, p, nullptr);
    if (rc) return rc;
    info->n_dirs = p.nd;
    info->n_groups = p.ngroups;
    info->n_items = p.items;
    info->z_splits = p.zsplits;
    info->power_tiles = p.ntiles;
    info->power_chunk = p.rl.kchunk >= (1 << 30) ? 0 : p.rl.kchunk;
    info->proj_waves = (p.fast && !p.chain) ? p.waves : 4;
    info->limbs_slice = p.nls;
    info->limbs_moment = p.nlr;
    info->bits_slice = p.bits_slice;
    info->bits_moment = p.bits_moment;
    size_t l = 0;
    for (int g = 0; g < p.ngroups; ++g) l = std::max(l, p.lds[g]);
    info->lds_bytes = (int64_t)l;
    info->workspace = (int64_t)p.ws_bytes;
    return DPM_OK;
}

int dpm_moments_async(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                      const dpm_out *out_device, void *workspace, size_t ws_bytes, void *stream) {
    if (!volume || !out_device) return DPM_EINVAL;
    if (int trc = ensure_device_tables()) return trc;
    Plan p;
    int rc = make_plan(dims, dtype, max_order, false, p, volume);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (workspace) {
        if (ws_bytes < p.ws_bytes) return DPM_ENOMEM;
        return run_plan(p, volume, nullptr, nullptr, nullptr, out_device->exact, out_device->fp64,
                        workspace, st);
    }
    int dev;
    if ((rc = current_device(dev))) return rc;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if ((rc = ensure_ws_buf(dev, g_ws[dev].ptr, g_ws[dev].bytes, p.ws_bytes))) return rc;
    if ((rc = ws_begin(dev, st))) return rc;
    rc = run_plan(p, volume, nullptr, nullptr, nullptr, out_device->exact, out_device->fp64,
                  g_ws[dev].ptr, st);
    const int rc2 = ws_end(dev, st);
    return rc ? rc : rc2;
}

int dpm_moments(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                dpm_out *out) {
    if (!volume || !out) return DPM_EINVAL;
    if (int trc = ensure_device_tables()) return trc;
    Plan p;
    int rc = make_plan(dims, dtype, max_order, false, p, volume);
    if (rc) return rc;
    int dev;
    if ((rc = current_device(dev))) return rc;
    const int nm = n_moments(max_order), nm4 = n_moments(std::min(max_order, 4));
    const size_t ex_bytes = align_up((size_t)nm4 * 16), fp_bytes = align_up((size_t)nm * 8);
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if ((rc = ensure_ws_buf(dev, g_ws[dev].ptr, g_ws[dev].bytes, p.ws_bytes))) return rc;
    if ((rc = ensure_ws_buf(dev, g_ws[dev].out, g_ws[dev].out_bytes, ex_bytes + fp_bytes))) return rc;
    uint8_t *ob = static_cast<uint8_t *>(g_ws[dev].out);
    void *dex = ob;
    double *dfp = reinterpret_cast<double *>(ob + ex_bytes);
    if ((rc = ws_begin(dev, nullptr))) return rc;
    rc = run_plan(p, volume, nullptr, nullptr, nullptr, dex, dfp, g_ws[dev].ptr, nullptr);
    const int rc2 = ws_end(dev, nullptr);
    if (rc || rc2) return rc ? rc : rc2;
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return hip_fail(e);
    if (out->exact) {
        e = hipMemcpy(out->exact, dex, (size_t)nm4 * 16, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (out->fp64) {
        e = hipMemcpy(out->fp64, dfp, (size_t)nm * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e);
    }
    return DPM_OK;
}

int dpm_features(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                 const double spacing[3], dpm_features_out *out) {
    if (!volume || !out || !out->mu || max_order < 0 || max_order > KMAX) return DPM_EINVAL;
    if (spacing && !(spacing[0] > 0 && spacing[1] > 0 && spacing[2] > 0)) return DPM_EINVAL;
    if (int trc = ensure_device_tables()) return trc;
    // the centroid needs the first-order moments whatever the order asked for
    const int kr = std::max(max_order, 1);
    Plan p;
    int rc = make_plan(dims, dtype, kr, false, p, volume);
    if (rc) return rc;
    // width of the exact numerators: |M000^n mu| < 2^n M000^(n+1) D^n, D = largest coordinate
    const uint64_t vmax = p.elem == 1 ? 255u : 65535u;
    const int b000 = bitlen_u64(vmax) + bitlen_u64((uint64_t)p.L) + bitlen_u64((uint64_t)p.M) +
                     bitlen_u64((uint64_t)p.N);
    const int bd = bitlen_u64((uint64_t)std::max<int64_t>(std::max(p.L, p.M), p.N));
    const int bits = max_order + (max_order + 1) * b000 + max_order * bd + 2;
    const int w = (bits + 31) / 32;
    if (w > 32) return DPM_ERANGE;
    int dev;
    if ((rc = current_device(dev))) return rc;
    const int nm = n_moments(max_order);
    const size_t raw_bytes = align_up((size_t)n_moments(kr) * p.nlr * 4), d_bytes = align_up((size_t)(3 + 3 * nm) * 8);
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if ((rc = ensure_ws_buf(dev, g_ws[dev].ptr, g_ws[dev].bytes, p.ws_bytes))) return rc;
    if ((rc = ensure_ws_buf(dev, g_ws[dev].out, g_ws[dev].out_bytes, raw_bytes + d_bytes))) return rc;
    uint8_t *ob = static_cast<uint8_t *>(g_ws[dev].out);
    uint32_t *draw = reinterpret_cast<uint32_t *>(ob);
    double *dd = reinterpret_cast<double *>(ob + raw_bytes);
    if ((rc = ws_begin(dev, nullptr))) return rc;
    rc = run_plan(p, volume, nullptr, nullptr, nullptr, nullptr, nullptr, g_ws[dev].ptr, nullptr, draw);
    if (rc) {
        (void)ws_end(dev, nullptr);
        return rc;
    }
    FeatArgs f{};
    f.raw = draw;
    f.K = max_order;
    for (int i = 0; i < 3; ++i) f.spacing[i] = spacing ? spacing[i] : 1.0;
    f.centroid = dd;
    f.mu = dd + 3;
    f.eta = dd + 3 + nm;
    f.mu_phys = dd + 3 + 2 * nm;
    hipError_t e = launch_features(p.nlr, w, f, nullptr);
    rc = ws_end(dev, nullptr);
    if (e != hipSuccess) return hip_fail(e);
    if (rc) return rc;
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return hip_fail(e);
    std::vector<double> h((size_t)3 + 3 * nm);
    if ((e = hipMemcpy(h.data(), dd, h.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e);
    for (int i = 0; i < 3; ++i) out->centroid[i] = h[i];
    std::memcpy(out->mu, h.data() + 3, (size_t)nm * 8);
    if (out->eta) std::memcpy(out->eta, h.data() + 3 + nm, (size_t)nm * 8);
    if (out->mu_phys) std::memcpy(out->mu_phys, h.data() + 3 + 2 * nm, (size_t)nm * 8);
    return DPM_OK;
}

int dpm_project_images(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                       int32_t *images_device, void *stream) {
    if (!volume || !images_device) return DPM_EINVAL;
    if (int trc = ensure_device_tables()) return trc;
    Plan p;
    int rc = make_plan(dims, dtype, max_order, true, p, volume);
    if (rc) return rc;
    int64_t off[NDIR_MAX], w[NDIR_MAX];
    int64_t acc = 0;
    for (int d = 0; d < p.nd; ++d) {
        w[d] = dpm_image_width(dims, d);
        off[d] = acc;
        acc += w[d] * p.M;
    }
    int dev;
    if ((rc = current_device(dev))) return rc;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if ((rc = ensure_ws_buf(dev, g_ws[dev].ptr, g_ws[dev].bytes, p.ws_bytes))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = ws_begin(dev, st))) return rc;
    rc = run_plan(p, volume, images_device, off, w, nullptr, nullptr, g_ws[dev].ptr, st);
    const int rc2 = ws_end(dev, st);
    return rc ? rc : rc2;
}

int dpm_moments_from_images(const int32_t *images_device, const int64_t dims[3], dpm_dtype dtype,
                            int max_order, dpm_out *out) {
    if (!images_device || !out) return DPM_EINVAL;
    if (int trc = ensure_device_tables()) return trc;
    Plan p;
    int rc = make_plan(dims, dtype, max_order, true, p, nullptr);
    if (rc) return rc;
    ImgArgs ia{};
    ia.images = images_device;
    ia.nd = p.nd;
    ia.M = (int32_t)p.M;
    int64_t acc = 0;
    for (int d = 0; d < p.nd; ++d) {
        const int64_t w = dpm_image_width(dims, d);
        ia.off[d] = acc;
        ia.width[d] = (int32_t)w;
        ia.origin[d] = dir_beta(d) < 0 ? (int32_t)(-dir_beta(d) * (p.N - 1)) : 0;
        acc += w * p.M;
    }
    // every entry is a line sum: at most max(L, N) voxels of at most vmax
    ia.bound = (int64_t)(p.elem == 1 ? 255 : 65535) * std::max(p.L, p.N);
    int dev;
    if ((rc = current_device(dev))) return rc;
    const int nm = n_moments(max_order), nm4 = n_moments(std::min(max_order, 4));
    const size_t ex_bytes = align_up((size_t)nm4 * 16), fp_bytes = align_up((size_t)nm * 8);
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if ((rc = ensure_ws_buf(dev, g_ws[dev].ptr, g_ws[dev].bytes, p.ws_bytes))) return rc;
    if ((rc = ensure_ws_buf(dev, g_ws[dev].out, g_ws[dev].out_bytes, ex_bytes + fp_bytes + 256))) return rc;
    uint8_t *ob = static_cast<uint8_t *>(g_ws[dev].out);
    void *dex = ob;
    double *dfp = reinterpret_cast<double *>(ob + ex_bytes);
    ia.bad = reinterpret_cast<uint32_t *>(ob + ex_bytes + fp_bytes);
    if ((rc = ws_begin(dev, nullptr))) return rc;
    hipError_t e = hipMemsetAsync(ia.bad, 0, 4, nullptr);
    if (e != hipSuccess) {
        (void)ws_end(dev, nullptr);
        return hip_fail(e);
    }
    rc = run_plan(p, nullptr, nullptr, nullptr, nullptr, dex, dfp, g_ws[dev].ptr, nullptr, nullptr, &ia);
    const int rc2 = ws_end(dev, nullptr);
    if (rc || rc2) return rc ? rc : rc2;
    uint32_t bad = 0;
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpy(&bad, ia.bad, 4, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e);
    if (bad) return DPM_ERANGE;
    if (out->exact && (e = hipMemcpy(out->exact, dex, (size_t)nm4 * 16, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e);
    if (out->fp64 && (e = hipMemcpy(out->fp64, dfp, (size_t)nm * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e);
    return DPM_OK;
}

int dpm_tune_set(const int64_t dims[3], dpm_dtype dtype, int max_order, const dpm_tuning *t) {
    if (!dims || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0) return DPM_EINVAL;
    const int elem = elem_of(dtype);
    if (!elem || max_order < 0 || max_order > KMAX) return DPM_EINVAL;
    const TuneKey key{dims[0], dims[1], dims[2], elem, max_order};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!t) {
        g_tune.erase(key);
        return DPM_OK;
    }
    if (t->z_splits < 0 || t->z_splits > 4096 || t->power_chunk < -1 || t->power_chunk > 4096 ||
        (t->waves != 0 && t->waves != 4 && t->waves != 8))
        return DPM_EINVAL;
    g_tune[key] = *t;
    return DPM_OK;
}

int dpm_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return DPM_OK;
}

int dpm_release(void) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    int rc = dpm::batched_release();
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_pow) {
        (void)hipSetDevice(kv.first.dev);
        if (hipFree(const_cast<uint4 *>(kv.second.b)) != hipSuccess) rc = DPM_EDEVICE;
    }
    g_pow.clear();
    for (int d = 0; d < 64; ++d) {
        if (!g_ws[d].ptr && !g_ws[d].out && !g_ws[d].done) continue;
        (void)hipSetDevice(d);
        if (g_ws[d].ptr && hipFree(g_ws[d].ptr) != hipSuccess) rc = DPM_EDEVICE;
        if (g_ws[d].out && hipFree(g_ws[d].out) != hipSuccess) rc = DPM_EDEVICE;
        if (g_ws[d].done && hipEventDestroy(g_ws[d].done) != hipSuccess) rc = DPM_EDEVICE;
        g_ws[d] = DevWs{};
    }
    (void)hipSetDevice(cur);
    return rc;
}

int dpm_profile_enable(int on) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    g_prof_on = on != 0;
    return DPM_OK;
}

int dpm_profile_collect(dpm_profile *out) {
    if (!out) return DPM_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    *out = dpm_profile{};
    int rc = DPM_OK;
    for (auto &ev : g_prof) {
        float t[NPROF - 1] = {}, tot = 0;
        hipError_t e = hipEventSynchronize(ev.e[NPROF - 1]);
        for (int i = 0; i + 1 < NPROF && e == hipSuccess; ++i) e = hipEventElapsedTime(&t[i], ev.e[i], ev.e[i + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&tot, ev.e[0], ev.e[NPROF - 1]);
        if (e != hipSuccess) {
            rc = hip_fail(e);
        } else {
            out->calls += 1;
            out->ms_project += t[0];
            out->ms_power += t[1];
            out->ms_combine += t[2];
            out->ms_total += tot;
        }
        for (int i = 0; i < NPROF; ++i) (void)hipEventDestroy(ev.e[i]);
    }
    g_prof.clear();
    return rc;
}

int dpm_recomb_weight(int k, int p, int d, int64_t *num, uint64_t *den) {
    if (k < 0 || k > KMAX || p < 0 || p > k || d < 0 || d > k || !num || !den) return DPM_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!host_tables()) return DPM_ERANGE;
    *num = g_tables.num[k][p][d];
    *den = g_tables.den[k][p];
    return DPM_OK;
}

}  // extern "C"
