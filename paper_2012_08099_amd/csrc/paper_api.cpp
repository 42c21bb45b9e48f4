// C ABI of the paper-literal mode (dpm_paper_*, dpm_moments_paper) and of the 1D-integral
// route for the family images (dpm_moments_drt): planning, integer-range checks,
// workspace layout and launch sequences.  Kernels: paper_mode.hip; contract:
// include/dpm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/dpm.h"
#include "dpm_common.h"
#include "kernels.h"
#include "paper.h"

namespace dpm {
int family_images(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order, int32_t *images,
                  void *ws, size_t ws_bytes, hipStream_t st, size_t *ws_need);  // dpm_api.cpp
void batched_set_error(int e);                                                // dpm_api.cpp
}  // namespace dpm

namespace {

using namespace dpm;

constexpr size_t kAlign = 256;
size_t al(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int bitlen(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

int elem_of(dpm_dtype t) { return t == DPM_U8 ? 1 : t == DPM_U16 ? 2 : 0; }

// ---------------------------------------------------------------- 1D -> 2D inverse
// For order n the directions g <= n give m_g = f(a_g, b_g) of the binary form
// f(x, y) = sum_p C(n,p) M_p x^p y^(n-p).  Lagrange: f = sum_g m_g prod_{e != g}
// (b_e x - a_e y) / D_g, D_g = prod_{e != g} (b_e a_g - a_e b_g), so C(n,p) M_p is
// sum_g m_g c_g[p] / D_g with c_g the coefficients of that product.
__int128 gcd128(__int128 a, __int128 b) {
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b != 0) {
        const __int128 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

bool build_drt_solve(DrtSolve &s, int &numsum_bits) {
    std::memset(&s, 0, sizeof(s));
    numsum_bits = 0;
    for (int n = 0; n <= DRT_KMAX; ++n) {
        __int128 binom[DRT_KMAX + 1];
        binom[0] = 1;
        for (int p = 1; p <= n; ++p) binom[p] = binom[p - 1] * (n - p + 1) / p;
        __int128 wn[DRT_KMAX + 1][DRT_NDIR], wd[DRT_KMAX + 1][DRT_NDIR];
        for (int g = 0; g <= n; ++g) {
            __int128 c[DRT_KMAX + 2] = {1};
            int deg = 0;
            __int128 D = 1;
            for (int e = 0; e <= n; ++e) {
                if (e == g) continue;
                __int128 nc[DRT_KMAX + 2] = {};
                for (int p = 0; p <= deg + 1; ++p) {
                    if (p >= 1) nc[p] += (__int128)drt_b(e) * c[p - 1];
                    if (p <= deg) nc[p] -= (__int128)drt_a(e) * c[p];
                }
                ++deg;
                for (int p = 0; p <= deg; ++p) c[p] = nc[p];
                D *= (__int128)drt_b(e) * drt_a(g) - (__int128)drt_a(e) * drt_b(g);
            }
            if (D == 0) return false;
            for (int p = 0; p <= n; ++p) {
                __int128 num = c[p], den = D * binom[p];
                if (den < 0) {
                    num = -num;
                    den = -den;
                }
                const __int128 gg = num == 0 ? den : gcd128(num, den);
                wn[p][g] = num / gg;
                wd[p][g] = den / gg;
            }
        }
        for (int p = 0; p <= n; ++p) {
            __int128 L = 1;
            for (int g = 0; g <= n; ++g) L = L / gcd128(L, wd[p][g]) * wd[p][g];
            unsigned __int128 sum = 0;
            for (int g = 0; g <= n; ++g) {
                const __int128 v = wn[p][g] * (L / wd[p][g]);
                s.num[n][p][g] = (int64_t)v;
                sum += (unsigned __int128)(v < 0 ? -v : v);
            }
            numsum_bits = std::max(numsum_bits, bitlen((uint64_t)sum));
            uint64_t den = (uint64_t)L;
            int sh = 0;
            while (!(den & 1u)) {
                den >>= 1;
                ++sh;
            }
            s.shift[n][p] = sh;
            unsigned __int128 x = den;  // den * den = 1 mod 8; Newton doubles the correct bits
            for (int it = 0; it < 7; ++it) x *= (unsigned __int128)2 - (unsigned __int128)den * x;
            s.inv_lo[n][p] = (uint64_t)x;
            s.inv_hi[n][p] = (uint64_t)(x >> 64);
        }
    }
    return true;
}

std::mutex g_mu;
DrtSolve g_solve;
int g_solve_bits = -1;

int solve_tables(const DrtSolve **out, int *numsum_bits) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_solve_bits < 0 && !build_drt_solve(g_solve, g_solve_bits)) return DPM_ERANGE;
    *out = &g_solve;
    *numsum_bits = g_solve_bits;
    return DPM_OK;
}

// Range checks of the 1D-integral route for images of W x H and K: coordinates
// t = a i + b j stay below 2^15 in magnitude (the tile kernel raises them to the 4th power
// in int64), and the int128 1D moments and solve sums below 2^126.
bool drt_fits(int64_t W, int64_t H, int K, int mass_bits, int numsum_bits) {
    if (W <= 0 || H <= 0 || W + 2 * (H - 1) >= (1 << 15)) return false;
    return mass_bits + K * 15 + numsum_bits + 2 <= 126;
}

// ---------------------------------------------------------------- paper plan
struct PaperPlan {
    int64_t L = 0, M = 0, N = 0;
    int elem = 0, K = 0, nimg = 0, ndir = 0;
    int nyb = 0, nzb = 0, nxt = 0;
    bool fast = false;
    int64_t W[PAPER_NIMG] = {}, H[PAPER_NIMG] = {};
    size_t img_off[PAPER_NIMG] = {};  // int32 offsets in the image block
    size_t img_bytes = 0;
    size_t o_xy = 0, o_xpz = 0, o_xmz = 0, o_zx = 0, o_yz = 0, o_p1 = 0, o_m1 = 0, ws = 0;  // workspace, after images
    int32_t tile0[PAPER_NIMG + 1] = {};
    int32_t tiles_i[PAPER_NIMG] = {};
};

int paper_plan(const int64_t dims[3], dpm_dtype dtype, int K, const void *vol, PaperPlan &p) {
    if (!dims) return DPM_EINVAL;
    p.elem = elem_of(dtype);
    if (!p.elem || K < 0 || K > DRT_KMAX) return p.elem ? DPM_ENOTSUP : DPM_EINVAL;
    p.L = dims[0];
    p.M = dims[1];
    p.N = dims[2];
    if (p.L <= 0 || p.M <= 0 || p.N <= 0) return DPM_EINVAL;
    p.K = K;
    p.nimg = K <= 2 ? 3 : K + 1;
    p.ndir = K + 1;
    const uint64_t vmax = p.elem == 1 ? 255u : 65535u;
    // every image entry and partial is a line sum of at most max(L, M, N) voxels (int32)
    if ((double)vmax * (double)std::max(std::max(p.L, p.M), p.N) >= 2147483648.0) return DPM_ERANGE;
    const DrtSolve *sv;
    int nsb;
    if (int rc = solve_tables(&sv, &nsb)) return rc;
    const int mass_bits = bitlen(vmax) + bitlen((uint64_t)p.L) + bitlen((uint64_t)p.M) + bitlen((uint64_t)p.N);
    p.W[0] = p.L, p.H[0] = p.M;              // XY: i = x, j = y
    p.W[1] = p.M, p.H[1] = p.N;              // YZ: i = y, j = z
    p.W[2] = p.N, p.H[2] = p.L;              // ZX: i = z, j = x
    p.W[3] = p.W[4] = p.L + p.N - 1;         // X+Z, X-Z: i = x +- z (+ N - 1), j = y
    p.H[3] = p.H[4] = p.M;
    size_t off = 0;
    int32_t t = 0;
    for (int e = 0; e < p.nimg; ++e) {
        if (!drt_fits(p.W[e], p.H[e], K, mass_bits, nsb)) return DPM_ERANGE;
        p.img_off[e] = off;
        off += (size_t)(p.W[e] * p.H[e]);
        p.tile0[e] = t;
        p.tiles_i[e] = (int32_t)((p.W[e] + DRT_IB - 1) / DRT_IB);
        t += p.tiles_i[e] * (int32_t)((p.H[e] + DRT_RB - 1) / DRT_RB);
    }
    p.tile0[p.nimg] = t;
    p.img_bytes = al(off * 4);
    p.nyb = (int)((p.M + PP_BY - 1) / PP_BY);
    p.nzb = (int)((p.N + PP_BZ - 1) / PP_BZ);
    p.nxt = (int)((p.L + PP_XT - 1) / PP_XT);
    if ((int64_t)p.nyb * p.nzb * p.nxt > INT32_MAX) return DPM_ERANGE;
    const uintptr_t addr = (uintptr_t)vol;
    p.fast = (p.L % 8 == 0) && (addr % (size_t)(8 * p.elem) == 0);
    size_t o = 0;
    p.o_xy = o;
    o += al((size_t)p.nzb * p.M * p.L * 4);
    p.o_xpz = o;
    o += al((size_t)p.nzb * p.nxt * p.M * PP_DW * 4);
    p.o_xmz = o;
    o += al((size_t)p.nzb * p.nxt * p.M * PP_DW * 4);
    p.o_zx = o;
    o += al((size_t)p.nyb * p.N * p.L * 4);
    p.o_yz = o;
    o += al((size_t)p.nxt * p.N * p.M * 4);
    p.o_p1 = o;
    o += al((size_t)t * DRT_NDIR * (DRT_KMAX + 1) * 16);
    p.o_m1 = o;
    o += al((size_t)DRT_MAXIMG * DRT_NDIR * (DRT_KMAX + 1) * 16);
    p.ws = o;
    return DPM_OK;
}

hipError_t paper_project(const PaperPlan &p, const void *vol, uint8_t *ws, int32_t *images, hipStream_t st) {
    PaperProjArgs a{};
    a.vol = static_cast<const uint8_t *>(vol);
    a.L = p.L;
    a.M = p.M;
    a.N = p.N;
    a.nyb = p.nyb;
    a.nzb = p.nzb;
    a.nxt = p.nxt;
    a.nimg = p.nimg;
    a.xy = reinterpret_cast<int32_t *>(ws + p.o_xy);
    a.xpz = reinterpret_cast<int32_t *>(ws + p.o_xpz);
    a.xmz = reinterpret_cast<int32_t *>(ws + p.o_xmz);
    a.zx = reinterpret_cast<int32_t *>(ws + p.o_zx);
    a.yz = reinterpret_cast<int32_t *>(ws + p.o_yz);
    hipError_t e = launch_paper_project(p.elem, p.fast, a, st);
    if (e != hipSuccess) return e;
    PaperReduceArgs r{};
    r.L = p.L;
    r.M = p.M;
    r.N = p.N;
    r.nyb = p.nyb;
    r.nzb = p.nzb;
    r.nxt = p.nxt;
    r.nimg = p.nimg;
    r.xy = a.xy;
    r.xpz = a.xpz;
    r.xmz = a.xmz;
    r.zx = a.zx;
    r.yz = a.yz;
    for (int i = 0; i < PAPER_NIMG; ++i) r.img[i] = i < p.nimg ? images + p.img_off[i] : nullptr;
    return launch_paper_reduce(r, st);
}

int hip_fail(hipError_t e) {
    dpm::batched_set_error((int)e);  // dpm_last_device_error
    return DPM_EDEVICE;
}

}  // namespace

extern "C" {

size_t dpm_paper_workspace_bytes(const int64_t dims[3], dpm_dtype dtype, int max_order) {
    PaperPlan p;
    if (paper_plan(dims, dtype, max_order, nullptr, p)) return 0;
    return p.img_bytes + p.ws;
}

int dpm_paper_images(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                     int32_t *images_device, void *workspace, size_t ws_bytes, void *stream) {
    if (!volume || !images_device || !workspace) return DPM_EINVAL;
    PaperPlan p;
    int rc = paper_plan(dims, dtype, max_order, volume, p);
    if (rc) return rc;
    if (ws_bytes < p.img_bytes + p.ws) return DPM_ENOMEM;
    hipError_t e = paper_project(p, volume, static_cast<uint8_t *>(workspace) + p.img_bytes, images_device,
                                 static_cast<hipStream_t>(stream));
    return e == hipSuccess ? DPM_OK : hip_fail(e);
}

int dpm_moments_paper(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                      const dpm_out *out_device, void *workspace, size_t ws_bytes, void *stream) {
    if (!volume || !out_device || !workspace) return DPM_EINVAL;
    PaperPlan p;
    int rc = paper_plan(dims, dtype, max_order, volume, p);
    if (rc) return rc;
    if (ws_bytes < p.img_bytes + p.ws) return DPM_ENOMEM;
    const DrtSolve *sv;
    int nsb;
    if ((rc = solve_tables(&sv, &nsb))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *base = static_cast<uint8_t *>(workspace);
    int32_t *images = reinterpret_cast<int32_t *>(base);
    uint8_t *ws = base + p.img_bytes;
    hipError_t e = paper_project(p, volume, ws, images, st);
    if (e != hipSuccess) return hip_fail(e);
    DrtArgs d{};
    for (int i = 0; i < p.nimg; ++i) {
        d.im[i].img = images + p.img_off[i];
        d.im[i].W = (int32_t)p.W[i];
        d.im[i].H = (int32_t)p.H[i];
        d.im[i].io = 0;  // X-Z: moments about the stored column, shifted in the finish (Section 5)
        d.im[i].tile0 = p.tile0[i];
        d.im[i].tiles_i = p.tiles_i[i];
    }
    d.nimg = p.nimg;
    d.ntiles = p.tile0[p.nimg];
    d.ndir = p.ndir;
    d.K = p.K;
    d.part1d = reinterpret_cast<__int128 *>(ws + p.o_p1);
    if ((e = launch_drt_tiles(d, st)) != hipSuccess) return hip_fail(e);
    DrtSumArgs sa{};
    sa.part1d = d.part1d;
    for (int i = 0; i <= p.nimg; ++i) sa.tile0[i] = p.tile0[i];
    sa.nimg = p.nimg;
    sa.m1d = reinterpret_cast<__int128 *>(ws + p.o_m1);
    if ((e = launch_drt_sum(sa, st)) != hipSuccess) return hip_fail(e);
    PaperFinishArgs f{};
    f.m1d = sa.m1d;
    f.nimg = p.nimg;
    f.ndir = p.ndir;
    f.K = p.K;
    f.xhat = p.N - 1;
    f.solve = *sv;
    f.exact = out_device->exact;
    f.fp64 = out_device->fp64;
    if ((e = launch_paper_finish(f, st)) != hipSuccess) return hip_fail(e);
    return DPM_OK;
}

size_t dpm_drt_workspace_bytes(const int64_t dims[3], dpm_dtype dtype, int max_order) {
    if (!dims || max_order < 0 || max_order > DRT_KMAX || !elem_of(dtype)) return 0;
    size_t fam = 0;
    if (dpm::family_images(nullptr, dims, dtype, max_order, nullptr, nullptr, 0, nullptr, &fam)) return 0;
    dpm_plan_info info;
    if (dpm_plan(dims, dtype, max_order, &info)) return 0;
    const DrtSolve *sv;
    int nsb;
    if (solve_tables(&sv, &nsb)) return 0;
    const uint64_t vmax = dtype == DPM_U8 ? 255u : 65535u;
    const int mass_bits = bitlen(vmax) + bitlen((uint64_t)dims[0]) + bitlen((uint64_t)dims[1]) + bitlen((uint64_t)dims[2]);
    size_t imgs = 0;
    int64_t tiles = 0;
    for (int d = 0; d <= max_order; ++d) {
        const int64_t w = dpm_image_width(dims, d);
        if (!drt_fits(w, dims[1], max_order, mass_bits, nsb)) return 0;
        imgs += (size_t)(w * dims[1]);
        tiles += ((w + DRT_IB - 1) / DRT_IB) * ((dims[1] + DRT_RB - 1) / DRT_RB);
    }
    const int K1 = max_order + 1;
    return al(imgs * 4) + al(fam) + al((size_t)tiles * DRT_NDIR * (DRT_KMAX + 1) * 16) +
           al((size_t)DRT_MAXIMG * DRT_NDIR * (DRT_KMAX + 1) * 16) + al((size_t)K1 * K1 * K1 * info.limbs_moment * 4);
}

int dpm_moments_drt(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                    const dpm_out *out_device, void *workspace, size_t ws_bytes, void *stream) {
    if (!volume || !out_device || !workspace) return DPM_EINVAL;
    const size_t need = dpm_drt_workspace_bytes(dims, dtype, max_order);
    if (!need) {
        if (!dims || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0 || !elem_of(dtype) || max_order < 0) return DPM_EINVAL;
        return max_order > DRT_KMAX ? DPM_ENOTSUP : DPM_ERANGE;
    }
    if (ws_bytes < need) return DPM_ENOMEM;
    size_t fam = 0;
    int rc = dpm::family_images(volume, dims, dtype, max_order, nullptr, nullptr, 0, nullptr, &fam);
    if (rc) return rc;
    dpm_plan_info info;
    if ((rc = dpm_plan(dims, dtype, max_order, &info))) return rc;
    const DrtSolve *sv;
    int nsb;
    if ((rc = solve_tables(&sv, &nsb))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int K = max_order, nd = K + 1;
    DrtArgs d{};
    size_t imgs = 0;
    int32_t t = 0;
    int64_t off[NDIR_MAX];
    for (int i = 0; i < nd; ++i) {
        const int64_t w = dpm_image_width(dims, i);
        int alpha, beta;
        dpm_direction(i, &alpha, &beta);
        off[i] = (int64_t)imgs;
        d.im[i].W = (int32_t)w;
        d.im[i].H = (int32_t)dims[1];
        d.im[i].io = beta < 0 ? (int32_t)(-beta * (dims[2] - 1)) : 0;  // true origin of the row
        d.im[i].tile0 = t;
        d.im[i].tiles_i = (int32_t)((w + DRT_IB - 1) / DRT_IB);
        t += d.im[i].tiles_i * (int32_t)((dims[1] + DRT_RB - 1) / DRT_RB);
        imgs += (size_t)(w * dims[1]);
    }
    uint8_t *base = static_cast<uint8_t *>(workspace);
    int32_t *images = reinterpret_cast<int32_t *>(base);
    uint8_t *fws = base + al(imgs * 4);
    __int128 *p1 = reinterpret_cast<__int128 *>(fws + al(fam));
    __int128 *m1 = reinterpret_cast<__int128 *>(reinterpret_cast<uint8_t *>(p1) + al((size_t)t * DRT_NDIR * (DRT_KMAX + 1) * 16));
    uint32_t *part = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(m1) +
                                                  al((size_t)DRT_MAXIMG * DRT_NDIR * (DRT_KMAX + 1) * 16));
    // step 1: the family projection images (Section 3.1)
    if ((rc = dpm::family_images(volume, dims, dtype, K, images, fws, fam, st, nullptr))) return rc;
    // step 2 by the 1D integrals of Section 5
    for (int i = 0; i < nd; ++i) d.im[i].img = images + off[i];
    d.nimg = nd;
    d.ntiles = t;
    d.ndir = nd;
    d.K = K;
    d.part1d = p1;
    hipError_t e = launch_drt_tiles(d, st);
    if (e != hipSuccess) return hip_fail(e);
    DrtSumArgs sa{};
    sa.part1d = p1;
    for (int i = 0; i <= nd; ++i) sa.tile0[i] = i < nd ? d.im[i].tile0 : t;
    sa.nimg = nd;
    sa.m1d = m1;
    if ((e = launch_drt_sum(sa, st)) != hipSuccess) return hip_fail(e);
    DrtToPartArgs tp{};
    tp.m1d = m1;
    tp.nimg = nd;
    tp.ndir = nd;
    tp.K = K;
    tp.nlr = info.limbs_moment;
    tp.solve = *sv;
    tp.part = part;
    if ((e = launch_drt_to_part(tp, st)) != hipSuccess) return hip_fail(e);
    // steps 3-4 unchanged: one tile per image in slot 2d + 1 (its origin side), then the
    // recombination of Section 3.2
    FinishArgs f{};
    f.part = part;
    f.rois = nullptr;
    f.nvol = 1;
    f.K = K;
    for (int s = 0; s <= NSLOT; ++s) f.tile0[s] = std::min(s / 2, nd);
    f.exact = out_device->exact;
    f.fp64 = out_device->fp64;
    f.raw = nullptr;
    if ((e = launch_finish(info.limbs_moment, f, st)) != hipSuccess) return hip_fail(e);
    return DPM_OK;
}

}  // extern "C"
