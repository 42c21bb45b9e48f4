// Second and third stages of the method, in exact multiword integers:
//
//  * reduce:    M^d_{k,q} = sum_y y^q r_{d,k}(y)  -- the y part of the 2D moments of
//               eq. (1) for every image d, from the per-slice row power sums.
//  * recombine: the 3D moments of Section 3.2.  For each x-z degree k and y power q,
//               the images d = 0..k satisfy
//                   M^d_{k,q} = sum_p C(k,p) alpha_d^p beta_d^(k-p) M_{p,q,k-p},
//               a (k+1)x(k+1) system with exact rational inverse (Lagrange form,
//               tables built on the host).  For k <= 4 this is eqs. (10)-(16): e.g.
//               k = 2 gives eq. (13) and k = 3 the corrected eqs. (15)/(16).
//               Every moment comes out as an exact integer: numerator / denominator
//               with an exact division (shift + multiply by the odd inverse).
#include "dpm_common.h"
#include "kernels.h"
#include "mw.h"

namespace dpm {

__constant__ int64_t c_num[KMAX + 1][KMAX + 1][KMAX + 1];
__constant__ int32_t c_shift[KMAX + 1][KMAX + 1];
__constant__ uint32_t c_inv[KMAX + 1][KMAX + 1][NLR_MAX];

constexpr int RED_THREADS = 256;

// decode triple t (pairs in pair order, q = 0..K-k) -> (pair, k, q)
__device__ __forceinline__ void decode_triple(int K, int t, int &pair, int &d, int &k, int &q) {
    pair = 0;
    for (d = 0; d <= K; ++d)
        for (k = d; k <= K; ++k, ++pair) {
            const int nq = K - k + 1;
            if (t < nq) {
                q = t;
                return;
            }
            t -= nq;
        }
}

template <int NLR>
__device__ void block_reduce_store(mw::Int<NLR> acc, uint32_t *dst, uint32_t *red) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int l = 0; l < NLR; ++l) red[tid * NLR + l] = acc.w[l];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            mw::Int<NLR> a, b;
#pragma unroll
            for (int l = 0; l < NLR; ++l) {
                a.w[l] = red[tid * NLR + l];
                b.w[l] = red[(tid + s) * NLR + l];
            }
            mw::add(a, b);
#pragma unroll
            for (int l = 0; l < NLR; ++l) red[tid * NLR + l] = a.w[l];
        }
        __syncthreads();
    }
    if (tid < NLR) dst[tid] = red[tid];
    __syncthreads();
}

template <int NLS, int NLR>
__device__ mw::Int<NLR> load_part(const uint32_t *p) {
    mw::Int<NLS> v;
#pragma unroll
    for (int l = 0; l < NLS; ++l) v.w[l] = p[l];
    return mw::resize<NLR, NLS>(v);
}

// x-z power sum of image d at degree k for one item: non-negative side plus (-1)^k
// times the negative side (a = o - bin).
template <int NLS, int NLR>
__device__ mw::Int<NLR> row_sum(const uint32_t *item_part, int K, int d, int k, uint64_t mask) {
    mw::Int<NLR> v;
    mw::set_zero(v);
    if ((mask >> (2 * d + 1)) & 1u) v = load_part<NLS, NLR>(item_part + ((size_t)(2 * d + 1) * (K + 1) + k) * NLS);
    if ((mask >> (2 * d)) & 1u) {
        const mw::Int<NLR> n = load_part<NLS, NLR>(item_part + ((size_t)(2 * d) * (K + 1) + k) * NLS);
        if (k & 1) mw::sub(v, n);
        else mw::add(v, n);
    }
    return v;
}

// grid: one block per (pair, q) triple
template <int NLS, int NLR>
__global__ void __launch_bounds__(RED_THREADS) reduce_kernel(ReduceArgs a) {
    __shared__ uint32_t red[RED_THREADS * NLR];
    int pair, d, k, q;
    decode_triple(a.K, blockIdx.x, pair, d, k, q);
    mw::Int<NLR> acc;
    mw::set_zero(acc);
    const size_t istride = (size_t)2 * (a.K + 1) * (a.K + 1) * NLS;
    for (int i = threadIdx.x; i < a.nitems; i += blockDim.x) {
        const uint32_t y = (uint32_t)(i / a.zsplits);
        mw::Int<NLR> v = row_sum<NLS, NLR>(a.part + i * istride, a.K, d, k, a.slot_mask);
        for (int j = 0; j < q; ++j) mw::mul_u32(v, y);
        mw::add(acc, v);
    }
    block_reduce_store<NLR>(acc, a.m2 + ((size_t)pair * (a.K + 1) + q) * NLR, red);
}

// grid: one block per ROI; every (pair, q) triple in turn
template <int NLS, int NLR>
__global__ void __launch_bounds__(RED_THREADS) reduce_batched_kernel(ReduceBatchedArgs a) {
    __shared__ uint32_t red[RED_THREADS * NLR];
    const RoiDesc rd = a.rois[blockIdx.x];
    uint64_t mask = 0;
    for (int s = 0; s < 14; ++s)
        if (rd.slot_len[s]) mask |= (uint64_t)1 << s;
    const size_t istride = (size_t)2 * (a.K + 1) * (a.K + 1) * NLS;
    int t = 0;
    for (int dd = 0; dd <= a.K; ++dd)
        for (int kk = dd; kk <= a.K; ++kk)
            for (int qq = 0; qq <= a.K - kk; ++qq, ++t) {
                const int pair = pair_index(a.K, dd, kk);
                mw::Int<NLR> acc;
                mw::set_zero(acc);
                for (int i = threadIdx.x; i < rd.nitems; i += blockDim.x) {
                    mw::Int<NLR> v = row_sum<NLS, NLR>(a.part + (size_t)(rd.item0 + i) * istride, a.K, dd, kk, mask);
                    for (int j = 0; j < qq; ++j) mw::mul_u32(v, (uint32_t)i);
                    mw::add(acc, v);
                }
                block_reduce_store<NLR>(
                    acc, a.m2 + (((size_t)blockIdx.x * a.npairs + pair) * (a.K + 1) + qq) * NLR, red);
            }
    (void)t;
}

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

template <int NLR>
__global__ void __launch_bounds__(RED_THREADS) recombine_kernel(RecombArgs a) {
    const int vol = blockIdx.x;
    const int K = a.K;
    const int nm = n_moments(K);
    const int nm4 = n_moments(K < 4 ? K : 4);
    const uint32_t *m2 = a.m2 + (size_t)vol * a.npairs * (K + 1) * NLR;
    for (int m = threadIdx.x; m < nm; m += blockDim.x) {
        int p, q, r;
        decode_moment(m, p, q, r);
        const int k = p + r;
        mw::Int<NLR> num;
        mw::set_zero(num);
        for (int d = 0; d <= k; ++d) {
            const int64_t c = c_num[k][p][d];
            if (c == 0) continue;
            mw::Int<NLR> v;
            const uint32_t *src = m2 + ((size_t)pair_index(K, d, k) * (K + 1) + q) * NLR;
#pragma unroll
            for (int l = 0; l < NLR; ++l) v.w[l] = src[l];
            mw::Int<NLR> t = mw::mul_i64(v, c);
            mw::add(num, t);
        }
        // exact division by den = 2^shift * odd
        mw::sar(num, c_shift[k][p]);
        mw::Int<NLR> inv;
#pragma unroll
        for (int l = 0; l < NLR; ++l) inv.w[l] = c_inv[k][p][l];
        const mw::Int<NLR> val = mw::mul_mod(num, inv);
        if (a.fp64) a.fp64[(size_t)vol * nm + m] = mw::to_double(val);
        if (a.exact && m < nm4) {
            uint64_t *e = reinterpret_cast<uint64_t *>(a.exact) + 2 * ((size_t)vol * nm4 + m);
            e[0] = (uint64_t)val.w[0] | ((uint64_t)val.w[1] << 32);
            e[1] = (uint64_t)val.w[2] | ((uint64_t)val.w[3] << 32);
        }
        if (a.wide) {
            uint32_t *w = a.wide + ((size_t)vol * nm + m) * NLR;
#pragma unroll
            for (int l = 0; l < NLR; ++l) w[l] = val.w[l];
        }
    }
}

// ------------------------------------------------------------ launchers
static int n_triples(int K) {
    int t = 0;
    for (int d = 0; d <= K; ++d)
        for (int k = d; k <= K; ++k) t += K - k + 1;
    return t;
}

template <int NLS, int NLR>
static hipError_t red_go(const ReduceArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((reduce_kernel<NLS, NLR>), dim3(n_triples(a.K)), dim3(RED_THREADS), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reduce(int nls, int nlr, const ReduceArgs &a, hipStream_t st) {
    if (nls == 4 && nlr == 4) return red_go<4, 4>(a, st);
    if (nls == 4 && nlr == 8) return red_go<4, 8>(a, st);
    if (nls == 4 && nlr == 12) return red_go<4, 12>(a, st);
    if (nls == 8 && nlr == 8) return red_go<8, 8>(a, st);
    if (nls == 8 && nlr == 12) return red_go<8, 12>(a, st);
    return hipErrorInvalidValue;
}

template <int NLS, int NLR>
static hipError_t redb_go(const ReduceBatchedArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((reduce_batched_kernel<NLS, NLR>), dim3(a.nrois), dim3(RED_THREADS), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reduce_batched(int nls, int nlr, const ReduceBatchedArgs &a, hipStream_t st) {
    if (nls == 4 && nlr == 4) return redb_go<4, 4>(a, st);
    if (nls == 4 && nlr == 8) return redb_go<4, 8>(a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_recombine(int nlr, const RecombArgs &a, hipStream_t st) {
    if (nlr == 4) hipLaunchKernelGGL((recombine_kernel<4>), dim3(a.nvol), dim3(RED_THREADS), 0, st, a);
    else if (nlr == 8) hipLaunchKernelGGL((recombine_kernel<8>), dim3(a.nvol), dim3(RED_THREADS), 0, st, a);
    else if (nlr == 12) hipLaunchKernelGGL((recombine_kernel<12>), dim3(a.nvol), dim3(RED_THREADS), 0, st, a);
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
