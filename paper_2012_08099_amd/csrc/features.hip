// Object features of one volume (Section 4, after the 3D moments), from its exact raw
// moments M_pqr (eq. 2):
//   centroid          (x̄, ȳ, z̄) = (M100, M010, M001) / M000
//   central moments   mu_pqr = sum V (x - x̄)^p (y - ȳ)^q (z - z̄)^r
//   scale-normalised  eta_pqr = mu_pqr / mu_000^((p+q+r)/3 + 1)
//   physical spacing  mu'_pqr = alpha^(1+p) beta^(1+q) delta^(1+r) mu_pqr
// Expanding the three binomials, with n = p + q + r, M000^n mu_pqr is the integer
//   N_pqr = sum_{a<=p, b<=q, c<=r} C(p,a) C(q,b) C(r,c) (-M100)^(p-a) (-M010)^(q-b)
//           (-M001)^(r-c) M000^(a+b+c) M_abc,
// formed exactly in W 32-bit limbs (no cancellation); mu_pqr = N_pqr / M000^n is the only
// rounding, two roundings to double (relative error below 2^-51).
#include <cmath>

#include "dpm_common.h"
#include "kernels.h"
#include "mw.h"

namespace dpm {

__device__ __forceinline__ void feat_decode(int m, int &p, int &q, int &r) {
    int n = 0;
    while (n_moments(n) <= m) ++n;
    int rem = m - (n > 0 ? n_moments(n - 1) : 0);
    // within degree n: p from n down to 0; for each p, q from n-p down to 0
    p = n;
    while (rem >= n - p + 1) {
        rem -= n - p + 1;
        --p;
    }
    q = n - p - rem;
    r = n - p - q;
}

__device__ __forceinline__ uint32_t binom(int n, int k) {
    uint32_t c = 1;  // C(n,k) <= C(16,8) = 12870
    for (int i = 1; i <= k; ++i) c = c * (uint32_t)(n - k + i) / (uint32_t)i;
    return c;
}

__device__ __forceinline__ double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// One 64-lane workgroup per moment; the lanes split its (a, b, c) terms.
template <int NLR, int W>
__global__ void __launch_bounds__(64) features_kernel(FeatArgs f) {
    __shared__ mw::Int<W> pw[4][KMAX + 1];  // powers of M000, -M100, -M010, -M001
    const int m = blockIdx.x, lane = threadIdx.x;
    auto raw = [&](int idx) {
        mw::Int<NLR> v;
#pragma unroll
        for (int l = 0; l < NLR; ++l) v.w[l] = f.raw[(size_t)idx * NLR + l];
        return mw::resize<W, NLR>(v);
    };
    if (lane < 4) {
        // graded index 0 = M000, 1 = M100, 2 = M010, 3 = M001
        mw::Int<W> base = raw(lane);
        if (lane > 0) mw::neg(base);
        mw::Int<W> pk;
        mw::set_u64(pk, 1);
        for (int k = 0; k <= f.K; ++k) {
            pw[lane][k] = pk;
            pk = mw::mul_mod(pk, base);
        }
    }
    __syncthreads();
    int p, q, r;
    feat_decode(m, p, q, r);
    const int n = p + q + r;
    const int nt = (p + 1) * (q + 1) * (r + 1);
    mw::Int<W> acc;
    mw::set_zero(acc);
    for (int t = lane; t < nt; t += 64) {
        const int c = t % (r + 1), b = (t / (r + 1)) % (q + 1), a = t / ((r + 1) * (q + 1));
        mw::Int<W> v = raw(moment_index(a, b, c));
        v = mw::mul_mod(v, pw[0][a + b + c]);
        v = mw::mul_mod(v, pw[1][p - a]);
        v = mw::mul_mod(v, pw[2][q - b]);
        v = mw::mul_mod(v, pw[3][r - c]);
        mw::mul_u32(v, binom(p, a));
        mw::mul_u32(v, binom(q, b));
        mw::mul_u32(v, binom(r, c));
        mw::add(acc, v);
    }
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) {
        mw::Int<W> o;
#pragma unroll
        for (int l = 0; l < W; ++l) o.w[l] = (uint32_t)__shfl_xor((int)acc.w[l], sh, 64);
        mw::add(acc, o);
    }
    if (lane != 0) return;
    const double m000 = mw::to_double(raw(0));
    const double mu = mw::to_double(acc) / mw::to_double(pw[0][n]);  // M000 = 0: NaN
    f.mu[m] = mu;
    if (f.eta) f.eta[m] = mu / pow(m000, n / 3.0 + 1.0);
    if (f.mu_phys) f.mu_phys[m] = ipow(f.spacing[0], 1 + p) * ipow(f.spacing[1], 1 + q) * ipow(f.spacing[2], 1 + r) * mu;
    if (m == 0 && f.centroid)
        for (int i = 0; i < 3; ++i) f.centroid[i] = mw::to_double(raw(1 + i)) / m000;
}

template <int NLR>
static hipError_t feat_w(int w, const FeatArgs &f, hipStream_t st) {
    const dim3 grid(n_moments(f.K));
    if (w <= 8) hipLaunchKernelGGL((features_kernel<NLR, 8>), grid, dim3(64), 0, st, f);
    else if (w <= 16) hipLaunchKernelGGL((features_kernel<NLR, 16>), grid, dim3(64), 0, st, f);
    else if (w <= 32) hipLaunchKernelGGL((features_kernel<NLR, 32>), grid, dim3(64), 0, st, f);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_features(int nlr, int w, const FeatArgs &f, hipStream_t st) {
    if (nlr == 4) return feat_w<4>(w, f, st);
    if (nlr == 8) return feat_w<8>(w, f, st);
    if (nlr == 12) return feat_w<12>(w, f, st);
    return hipErrorInvalidValue;
}

}  // namespace dpm
