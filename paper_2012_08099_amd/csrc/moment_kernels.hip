// Last stage of the method, in exact multiword integers, one workgroup per 3D moment:
//
//  * the 2D moments M^d_{k,q} = sum_y y^q r_{d,k}(y) of every image d (eq. 1) are the
//    sums of the power-sum tiles of the image's two slots, the negative side taken with
//    the sign (-1)^k (its coordinates are -a);
//  * recombination (Section 3.2): for each x-z degree k and y power q the images
//    d = 0..k satisfy
//        M^d_{k,q} = sum_p C(k,p) alpha_d^p beta_d^(k-p) M_{p,q,k-p},
//    a (k+1)x(k+1) system with exact rational inverse (Lagrange form, tables built on
//    the host).  For k <= 4 this is eqs. (10)-(16): e.g. k = 2 gives eq. (13) and k = 3
//    the corrected eqs. (15)/(16).
//  The workgroup forms numerator = sum_d num[k][p][d] M^d_{k,q} directly from the tiles, and
//  the moment is numerator / denominator by an exact division (shift + multiply by the
//  odd part's inverse).
#include "dpm_common.h"
#include "kernels.h"
#include "lane_sum.h"
#include "mw.h"

namespace dpm {

__constant__ int64_t c_num[KMAX + 1][KMAX + 1][KMAX + 1];
__constant__ int32_t c_shift[KMAX + 1][KMAX + 1];
__constant__ uint32_t c_inv[KMAX + 1][KMAX + 1][NLR_MAX];

// decode graded index m -> (p, q, r)
__device__ __forceinline__ void decode_moment(int m, int &p, int &q, int &r) {
    int n = 0;
    while ((n + 1) * (n + 2) * (n + 3) / 6 <= m) ++n;
    int rem = m - n * (n + 1) * (n + 2) / 6;
    // within degree n: p from n down to 0; for each p, q from n-p down to 0
    p = n;
    while (rem >= n - p + 1) {
        rem -= n - p + 1;
        --p;
    }
    q = n - p - rem;
    r = n - p - q;
}

constexpr int FIN_THREADS = 256;   // one volume: up to 2 * 16 * (K+1) tiles per moment
constexpr int FIN_THREADS_ROI = 64; // batched ROIs: a few tiles per moment, one wave
constexpr int FIN_BATCH = 4;  // entries whose loads are in flight together

// moment m of volume vol = num / den(k, p), by an exact division (den = 2^shift * odd:
// arithmetic shift, then multiplication by the odd part's inverse mod 2^(32 NLR)), to the
// outputs the caller asked for.
template <int NLR>
__device__ __forceinline__ void finish_store(const FinishArgs &a, int vol, int m, int k, int p, mw::Int<NLR> num) {
    const int K = a.K;
    mw::sar(num, c_shift[k][p]);
    mw::Int<NLR> inv;
#pragma unroll
    for (int l = 0; l < NLR; ++l) inv.w[l] = c_inv[k][p][l];
    const mw::Int<NLR> val = mw::mul_mod(num, inv);
    const int nm = n_moments(K), nm4 = n_moments(K < 4 ? K : 4);
    if (a.fp64) a.fp64[(size_t)vol * nm + m] = mw::to_double(val);
    if (a.raw)
#pragma unroll
        for (int l = 0; l < NLR; ++l) a.raw[((size_t)vol * nm + m) * NLR + l] = val.w[l];
    if (a.exact && m < nm4) {
        uint64_t *e = reinterpret_cast<uint64_t *>(a.exact) + 2 * ((size_t)vol * nm4 + m);
        e[0] = (uint64_t)val.w[0] | ((uint64_t)val.w[1] << 32);
        e[1] = (uint64_t)val.w[2] | ((uint64_t)val.w[3] << 32);
    }
}

template <int NLR, int NT>
__global__ void __launch_bounds__(NT) finish_kernel(FinishArgs a) {
    __shared__ uint32_t wsum[NT / 64][NLR];
    const int vol = blockIdx.x, m = blockIdx.y, tid = threadIdx.x;
    const int K = a.K;
    int p, q, r;
    decode_moment(m, p, q, r);
    const int k = p + r;
    // The tiles of slots 0 .. 2k+1 (images d <= k) are the range [tbase, tbase + nent),
    // slot by slot.  One volume: slot s owns [tile0[s], tile0[s+1]).  Batched ROI: each
    // non-empty slot owns ipt tiles, in slot order.
    uint32_t mask = 0;
    int ipt = 0, nent;
    size_t tbase = 0;
    if (a.rois) {
        const RoiDesc &rd = a.rois[vol];
        for (int s = 0; s < 14 && s < 2 * (k + 1); ++s)
            if (rd.slot_len[s]) mask |= 1u << s;
        ipt = (int)((rd.M + 15) / 16);
        tbase = (size_t)rd.tile0;
        nent = __popc(mask) * ipt;
    } else {
        nent = a.tile0[2 * k + 2];
    }
    mw::Int<NLR> num;
    mw::set_zero(num);
    for (int e0 = tid; e0 < nent; e0 += FIN_BATCH * NT) {
        mw::Int<NLR> v[FIN_BATCH];
        int64_t c[FIN_BATCH];
        // all loads of the batch first (coefficient and tile value are independent)
#pragma unroll
        for (int b = 0; b < FIN_BATCH; ++b) {
            const int e = e0 + b * NT;
            mw::set_zero(v[b]);
            c[b] = 0;
            if (e < nent) {
                int s = 0;
                if (a.rois) {
                    // the (e / ipt)-th set bit of mask
                    uint32_t mm = mask;
                    for (int rank = e / ipt; rank > 0; --rank) mm &= mm - 1u;
                    s = __ffs(mm) - 1;
                } else {
                    while (e >= a.tile0[s + 1]) ++s;
                }
                const int d = s >> 1, side = s & 1;
                c[b] = (side == 0 && (k & 1)) ? -c_num[k][p][d] : c_num[k][p][d];
                const size_t tile = tbase + (size_t)e;
                const uint32_t *src = a.part + ((tile * (K + 1) + k) * (K + 1) + q) * NLR;
#pragma unroll
                for (int l = 0; l < NLR; ++l) v[b].w[l] = src[l];
            }
        }
#pragma unroll
        for (int b = 0; b < FIN_BATCH; ++b) mw::add(num, mw::mul_i64(v[b], c[b]));
    }
    wave_sum_last(num);  // the wave's total in its lane 63
    if (NT > 64) {
        if ((tid & 63) == 63)
#pragma unroll
            for (int l = 0; l < NLR; ++l) wsum[tid >> 6][l] = num.w[l];
        __syncthreads();
    }
    if (tid != 63) return;
    for (int w = 1; w < NT / 64; ++w) {
        mw::Int<NLR> o;
#pragma unroll
        for (int l = 0; l < NLR; ++l) o.w[l] = wsum[w][l];
        mw::add(num, o);
    }
    finish_store(a, vol, m, k, p, num);
}

// Recombination of batched ROIs: one workgroup per ROI.  Thread t takes the (moment, slot)
// pairs t, t + FIN_ROI_THREADS, ...: the slot's tiles of the ROI (their loads in flight
// together) times the slot's coefficient, into LDS; then thread m adds moment m's slot
// products.  Every pair's loads are issued at once instead of one slot after another.
constexpr int FIN_ROI_THREADS = 256;
constexpr int FIN_ROI_SLOTS = 14;            // 2 (K + 1) for K <= 6
constexpr int FIN_ROI_PAIRS = 84 * FIN_ROI_SLOTS;  // n_moments(6) x slots

template <int NLR>
__global__ void __launch_bounds__(FIN_ROI_THREADS) finish_roi_kernel(FinishArgs a) {
    __shared__ uint32_t prod[FIN_ROI_PAIRS][NLR];
    const int vol = blockIdx.x, tid = threadIdx.x, K = a.K;
    const int nm = n_moments(K), ns = 2 * (K + 1);
    const RoiDesc &rd = a.rois[vol];
    const int ipt = (int)((rd.M + 15) / 16);
    for (int pr = tid; pr < nm * ns; pr += FIN_ROI_THREADS) {
        const int m = pr / ns, s = pr - m * ns;
        int p, q, r;
        decode_moment(m, p, q, r);
        const int k = p + r;
        mw::Int<NLR> v;
        mw::set_zero(v);
        if (s < 2 * (k + 1) && rd.slot_len[s]) {
            const int d = s >> 1, side = s & 1;
            const int64_t c = (side == 0 && (k & 1)) ? -c_num[k][p][d] : c_num[k][p][d];
            if (c != 0) {
                int rank = 0;  // non-empty slots before s: this slot's tiles follow theirs
                for (int e = 0; e < s; ++e) rank += rd.slot_len[e] != 0;
                const size_t t0 = (size_t)rd.tile0 + (size_t)rank * ipt;
                for (int b0 = 0; b0 < ipt; b0 += FIN_BATCH) {
                    mw::Int<NLR> w[FIN_BATCH];
#pragma unroll
                    for (int b = 0; b < FIN_BATCH; ++b) {
                        mw::set_zero(w[b]);
                        if (b0 + b < ipt) {
                            const uint32_t *src = a.part + (((t0 + b0 + b) * (K + 1) + k) * (K + 1) + q) * NLR;
#pragma unroll
                            for (int l = 0; l < NLR; ++l) w[b].w[l] = src[l];
                        }
                    }
#pragma unroll
                    for (int b = 0; b < FIN_BATCH; ++b) mw::add(v, w[b]);
                }
                v = mw::mul_i64(v, c);
            }
        }
#pragma unroll
        for (int l = 0; l < NLR; ++l) prod[pr][l] = v.w[l];
    }
    __syncthreads();
    for (int m = tid; m < nm; m += FIN_ROI_THREADS) {
        int p, q, r;
        decode_moment(m, p, q, r);
        mw::Int<NLR> num;
        mw::set_zero(num);
        for (int s = 0; s < ns; ++s) {
            mw::Int<NLR> o;
#pragma unroll
            for (int l = 0; l < NLR; ++l) o.w[l] = prod[m * ns + s][l];
            mw::add(num, o);
        }
        finish_store(a, vol, m, p + r, p, num);
    }
}

template <int NLR>
static void finish_go(const FinishArgs &a, dim3 grid, hipStream_t st) {
    if (a.rois && a.K <= 6) hipLaunchKernelGGL((finish_roi_kernel<NLR>), dim3(a.nvol), dim3(FIN_ROI_THREADS), 0, st, a);
    else if (a.rois) hipLaunchKernelGGL((finish_kernel<NLR, FIN_THREADS_ROI>), grid, dim3(FIN_THREADS_ROI), 0, st, a);
    else hipLaunchKernelGGL((finish_kernel<NLR, FIN_THREADS>), grid, dim3(FIN_THREADS), 0, st, a);
}

hipError_t launch_finish(int nlr, const FinishArgs &a, hipStream_t st) {
    const dim3 grid(a.nvol, n_moments(a.K));  // volumes along x: no 65535 limit on batches
    if (nlr == 4) finish_go<4>(a, grid, st);
    else if (nlr == 8) finish_go<8>(a, grid, st);
    else if (nlr == 12) finish_go<12>(a, grid, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------ host: tables
static __int128 i128_abs(__int128 v) { return v < 0 ? -v : v; }
static __int128 i128_gcd(__int128 a, __int128 b) {
    a = i128_abs(a);
    b = i128_abs(b);
    while (b != 0) {
        __int128 t = a % b;
        a = b;
        b = t;
    }
    return a;
}
static int bitlen_u128(unsigned __int128 v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// Lagrange form of the inverse of the homogeneous Vandermonde system above:
//   f(x, z) = sum_p C(k,p) M_p x^p z^(k-p) is known at the k+1 directions d, and
//   f = sum_d f(alpha_d, beta_d) prod_{e != d} (beta_e x - alpha_e z) / D_d,
//   D_d = prod_{e != d} (beta_e alpha_d - alpha_e beta_d).
bool build_recomb_tables(RecombTables &t) {
    for (int k = 0; k <= KMAX; ++k) {
        for (int p = 0; p <= KMAX; ++p) {
            for (int d = 0; d <= KMAX; ++d) t.num[k][p][d] = 0;
            t.shift[k][p] = 0;
            t.den[k][p] = 1;
            for (int l = 0; l < NLR_MAX; ++l) t.inv[k][p][l] = l == 0 ? 1u : 0u;
        }
        t.numsum_bits[k] = 0;
    }
    __int128 binom[KMAX + 1][KMAX + 1] = {};
    for (int n = 0; n <= KMAX; ++n) {
        binom[n][0] = 1;
        for (int j = 1; j <= n; ++j) binom[n][j] = binom[n - 1][j - 1] + (j <= n - 1 ? binom[n - 1][j] : 0);
    }
    for (int k = 0; k <= KMAX; ++k) {
        __int128 wn[KMAX + 1][KMAX + 1], wd[KMAX + 1][KMAX + 1];  // [p][d] reduced fraction
        for (int d = 0; d <= k; ++d) {
            __int128 c[KMAX + 2] = {};
            c[0] = 1;
            int deg = 0;
            __int128 Dd = 1;
            for (int e = 0; e <= k; ++e) {
                if (e == d) continue;
                const __int128 ae = dir_alpha(e), be = dir_beta(e);
                __int128 nc[KMAX + 2] = {};
                for (int pp = 0; pp <= deg + 1; ++pp) {
                    __int128 v = 0;
                    if (pp >= 1) v += be * c[pp - 1];
                    if (pp <= deg) v -= ae * c[pp];
                    nc[pp] = v;
                }
                ++deg;
                for (int pp = 0; pp <= deg; ++pp) c[pp] = nc[pp];
                Dd *= (be * dir_alpha(d) - ae * dir_beta(d));
            }
            if (Dd == 0) return false;
            for (int p = 0; p <= k; ++p) {
                __int128 n = c[p], den = Dd * binom[k][p];
                if (den < 0) {
                    n = -n;
                    den = -den;
                }
                const __int128 g = n == 0 ? den : i128_gcd(n, den);
                wn[p][d] = n / g;
                wd[p][d] = den / g;
            }
        }
        unsigned __int128 maxsum = 0;
        for (int p = 0; p <= k; ++p) {
            __int128 L = 1;
            for (int d = 0; d <= k; ++d) L = L / i128_gcd(L, wd[p][d]) * wd[p][d];
            if (L <= 0 || L > (__int128)UINT64_MAX) return false;
            unsigned __int128 s = 0;
            for (int d = 0; d <= k; ++d) {
                const __int128 v = wn[p][d] * (L / wd[p][d]);
                if (v > INT64_MAX || v < INT64_MIN) return false;
                t.num[k][p][d] = (int64_t)v;
                s += (unsigned __int128)i128_abs(v);
            }
            if (s > maxsum) maxsum = s;
            uint64_t den = (uint64_t)L;
            t.den[k][p] = den;
            int sh = 0;
            while (!(den & 1u)) {
                den >>= 1;
                ++sh;
            }
            t.shift[k][p] = sh;
            // inverse of the odd part modulo 2^(32 NLR_MAX) by Newton's iteration
            mw::Int<NLR_MAX> od, x, two;
            mw::set_u64(od, den);
            x = od;  // od * od = 1 mod 8
            mw::set_u64(two, 2);
            for (int it = 0; it < 8; ++it) {
                mw::Int<NLR_MAX> ox = mw::mul_mod(od, x);
                mw::Int<NLR_MAX> f = two;
                mw::sub(f, ox);
                x = mw::mul_mod(x, f);
            }
            for (int l = 0; l < NLR_MAX; ++l) t.inv[k][p][l] = x.w[l];
        }
        t.numsum_bits[k] = bitlen_u128(maxsum);
    }
    return true;
}

hipError_t upload_recomb_tables(const RecombTables &t) {
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_num), t.num, sizeof(t.num));
    if (e != hipSuccess) return e;
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_shift), t.shift, sizeof(t.shift));
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_inv), t.inv, sizeof(t.inv));
}

}  // namespace dpm
