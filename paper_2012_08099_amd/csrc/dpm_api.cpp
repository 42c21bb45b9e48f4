// C ABI of libdpm: argument checking, planning (bounds, integer widths, launch
// geometry, LDS layout), workspace management and the launch sequence
//   projection + row power sums  ->  y reduction  ->  recombination.
// See include/dpm.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/dpm.h"
#include "dpm_common.h"
#include "kernels.h"

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

// ------------------------------------------------------------------ planning
struct Plan {
    int K = 0, nd = 0, elem = 0;
    int64_t L = 0, M = 0, N = 0;
    int zsplits = 1, zrows = 0, items = 0;
    int R = 8, CT = 1;
    bool fast = false;
    int nls = 4, nlr = 4;
    int ngroups = 0;
    int gnd[NGROUP] = {};
    size_t lds[NGROUP] = {};
    int jobbins = 512;
    int npairs = 0;
    int bits_slice = 0, bits_moment = 0;
    size_t part_bytes = 0, m2_bytes = 0, ws_bytes = 0;
};

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int elem_of(dpm_dtype t) { return t == DPM_U8 ? 1 : t == DPM_U16 ? 2 : 0; }

// Lane layout along x for a row of L voxels: sub-rows of R lanes (power of two in
// [8, 64]) or 64-lane column tiles.
void lane_layout(int64_t L, int &R, int &CT) {
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
    if (p.nd > 7) {  // the later direction groups are built with 256-bit partials only
        p.nls = 8;
        if (p.nlr < 8) p.nlr = 8;
    }
    lane_layout(p.L, p.R, p.CT);
    const int64_t lanes = (p.L + G - 1) / G;
    const bool lanes_exact = (lanes == (int64_t)p.R * p.CT);
    const uintptr_t addr = (uintptr_t)vol_for_alignment;
    const size_t vec_bytes = p.elem == 2 ? 16 : 8;
    p.fast = lanes_exact && (p.L % G == 0) && (p.N % ZALIGN == 0) && (addr % vec_bytes == 0);
    if (const char *e = std::getenv("DPM_FORCE_GENERIC")) {
        if (atoi(e)) p.fast = false;
    }
    p.npairs = n_pairs(K);
    // groups and LDS per group (the largest item is the first; the last may differ)
    p.ngroups = 0;
    for (int g = 0; g < NGROUP; ++g) {
        const int b = group_begin(g), e = std::min(group_end(g), p.nd);
        if (e <= b) break;
        p.gnd[g] = e - b;
        ++p.ngroups;
        size_t best = 0;
        const int64_t firsts[2] = {0, (int64_t)(p.zsplits - 1) * p.zrows};
        for (int s = 0; s < 2; ++s) {
            const int64_t zs0 = firsts[s], ze0 = std::min<int64_t>(zs0 + p.zrows, p.N);
            ItemGeom ig;
            item_geometry(g, p.gnd[g], p.L, p.N, zs0, ze0, ig);
            const int nj = count_jobs(ig, p.gnd[g], p.jobbins);
            const size_t nk = (size_t)(KMAX + 1 - b);
            const size_t bytes = ((size_t)ig.lds_dwords + (size_t)nj * nk * p.nls) * 4;
            best = std::max(best, bytes);
        }
        p.lds[g] = best;
        if (best > 160 * 1024) return DPM_ERANGE;
    }
    p.part_bytes = align_up((size_t)p.items * p.npairs * p.nls * 4);
    p.m2_bytes = align_up((size_t)p.npairs * (K + 1) * p.nlr * 4);
    p.ws_bytes = p.part_bytes + p.m2_bytes;
    return DPM_OK;
}

// ------------------------------------------------------------------ workspaces
struct DevWs {
    void *ptr = nullptr;
    size_t bytes = 0;
    void *out = nullptr;  // device staging for dpm_moments results
    size_t out_bytes = 0;
};
DevWs g_ws[64];

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

int run_plan(const Plan &p, const void *vol, int32_t *images, const int64_t *img_off,
             const int64_t *img_w, void *exact, double *fp64, void *ws, hipStream_t st) {
    uint8_t *base = static_cast<uint8_t *>(ws);
    uint32_t *part = reinterpret_cast<uint32_t *>(base);
    uint32_t *m2 = reinterpret_cast<uint32_t *>(base + p.part_bytes);
    for (int g = 0; g < p.ngroups; ++g) {
        SliceArgs a{};
        a.vol = static_cast<const uint8_t *>(vol);
        a.L = p.L;
        a.M = p.M;
        a.N = p.N;
        a.pitch_y = p.L;
        a.pitch_z = p.L * p.M;
        a.zsplits = p.zsplits;
        a.zrows = p.zrows;
        a.K = p.K;
        a.R = p.R;
        a.CT = p.CT;
        a.jobbins = p.jobbins;
        a.npairs = p.npairs;
        a.part = part;
        a.images = images;
        for (int i = 0; i < 7; ++i) {
            a.img_off[i] = (images && i < p.gnd[g]) ? img_off[group_begin(g) + i] : 0;
            a.img_w[i] = (images && i < p.gnd[g]) ? img_w[group_begin(g) + i] : 0;
        }
        hipError_t e = launch_slice(p.elem, p.nls, p.fast, g, p.gnd[g], a, p.items, p.lds[g], st);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (!exact && !fp64) return DPM_OK;
    ReduceArgs r{part, p.items, p.zsplits, p.K, p.npairs, m2};
    hipError_t e = launch_reduce(p.nls, p.nlr, r, st);
    if (e != hipSuccess) return hip_fail(e);
    RecombArgs c{m2, 1, p.K, p.npairs, exact, fp64, nullptr};
    e = launch_recombine(p.nlr, c, st);
    if (e != hipSuccess) return hip_fail(e);
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
    if ((rc = ensure_buf(g_ws[dev].ptr, g_ws[dev].bytes, p.ws_bytes))) return rc;
    return run_plan(p, volume, nullptr, nullptr, nullptr, out_device->exact, out_device->fp64,
                    g_ws[dev].ptr, st);
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
    if ((rc = ensure_buf(g_ws[dev].ptr, g_ws[dev].bytes, p.ws_bytes))) return rc;
    if ((rc = ensure_buf(g_ws[dev].out, g_ws[dev].out_bytes, ex_bytes + fp_bytes))) return rc;
    uint8_t *ob = static_cast<uint8_t *>(g_ws[dev].out);
    void *dex = ob;
    double *dfp = reinterpret_cast<double *>(ob + ex_bytes);
    rc = run_plan(p, volume, nullptr, nullptr, nullptr, dex, dfp, g_ws[dev].ptr, nullptr);
    if (rc) return rc;
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
    if ((rc = ensure_buf(g_ws[dev].ptr, g_ws[dev].bytes, p.ws_bytes))) return rc;
    return run_plan(p, volume, images_device, off, w, nullptr, nullptr, g_ws[dev].ptr,
                    static_cast<hipStream_t>(stream));
}

int dpm_release(void) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    int rc = DPM_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (int d = 0; d < 64; ++d) {
        if (!g_ws[d].ptr && !g_ws[d].out) continue;
        (void)hipSetDevice(d);
        if (g_ws[d].ptr && hipFree(g_ws[d].ptr) != hipSuccess) rc = DPM_EDEVICE;
        if (g_ws[d].out && hipFree(g_ws[d].out) != hipSuccess) rc = DPM_EDEVICE;
        g_ws[d] = DevWs{};
    }
    (void)hipSetDevice(cur);
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
