// Fixed-width multiword integers for exact moment arithmetic (host and device).
//
// A value is N little-endian 32-bit limbs holding a two's complement integer modulo
// 2^(32N).  Sums and products of integers whose true value fits in N limbs (sign
// included) are therefore exact.  All loops have compile-time trip counts so that on
// the GPU the limbs stay in registers.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define MW_HD __host__ __device__ __forceinline__
#else
#define MW_HD inline
#endif

namespace mw {

template <int N>
struct Int {
    uint32_t w[N];
};

template <int N>
MW_HD void set_zero(Int<N> &a) {
#pragma unroll
    for (int i = 0; i < N; ++i) a.w[i] = 0u;
}

template <int N>
MW_HD void set_u64(Int<N> &a, uint64_t v) {
#pragma unroll
    for (int i = 0; i < N; ++i) a.w[i] = 0u;
    a.w[0] = (uint32_t)v;
    if (N > 1) a.w[1] = (uint32_t)(v >> 32);
}

template <int N>
MW_HD void set_i64(Int<N> &a, int64_t v) {
    uint32_t ext = v < 0 ? 0xffffffffu : 0u;
#pragma unroll
    for (int i = 0; i < N; ++i) a.w[i] = ext;
    a.w[0] = (uint32_t)(uint64_t)v;
    if (N > 1) a.w[1] = (uint32_t)((uint64_t)v >> 32);
}

template <int N>
MW_HD bool is_neg(const Int<N> &a) { return (a.w[N - 1] >> 31) != 0u; }

template <int N>
MW_HD bool is_zero(const Int<N> &a) {
    uint32_t o = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) o |= a.w[i];
    return o == 0u;
}

// a += b
template <int N>
MW_HD void add(Int<N> &a, const Int<N> &b) {
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        uint64_t t = (uint64_t)a.w[i] + b.w[i] + c;
        a.w[i] = (uint32_t)t;
        c = t >> 32;
    }
}

// a -= b
template <int N>
MW_HD void sub(Int<N> &a, const Int<N> &b) {
    uint64_t br = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        uint64_t t = (uint64_t)a.w[i] - b.w[i] - br;
        a.w[i] = (uint32_t)t;
        br = (t >> 63) & 1u;
    }
}

template <int N>
MW_HD void neg(Int<N> &a) {
    uint64_t c = 1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        uint64_t t = (uint64_t)(uint32_t)~a.w[i] + c;
        a.w[i] = (uint32_t)t;
        c = t >> 32;
    }
}

// a *= m (mod 2^(32N)); exact for non-negative a when the product fits, and for
// two's complement a as a product modulo 2^(32N).
template <int N>
MW_HD void mul_u32(Int<N> &a, uint32_t m) {
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        uint64_t t = (uint64_t)a.w[i] * m + c;
        a.w[i] = (uint32_t)t;
        c = t >> 32;
    }
}

// r = a * b mod 2^(32N)
template <int N>
MW_HD Int<N> mul_mod(const Int<N> &a, const Int<N> &b) {
    Int<N> r;
    set_zero(r);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        uint64_t c = 0;
#pragma unroll
        for (int j = 0; j + i < N; ++j) {
            uint64_t t = (uint64_t)a.w[i] * b.w[j] + r.w[i + j] + c;
            r.w[i + j] = (uint32_t)t;
            c = t >> 32;
        }
    }
    return r;
}

// a * m for a signed 64-bit m (mod 2^(32N))
template <int N>
MW_HD Int<N> mul_i64(const Int<N> &a, int64_t m) {
    uint64_t um = m < 0 ? (uint64_t)0 - (uint64_t)m : (uint64_t)m;
    uint32_t lo = (uint32_t)um, hi = (uint32_t)(um >> 32);
    Int<N> r;
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        uint64_t t = (uint64_t)a.w[i] * lo + c;
        r.w[i] = (uint32_t)t;
        c = t >> 32;
    }
    if (hi) {
        c = 0;
#pragma unroll
        for (int i = 0; i + 1 < N; ++i) {
            uint64_t t = (uint64_t)a.w[i] * hi + r.w[i + 1] + c;
            r.w[i + 1] = (uint32_t)t;
            c = t >> 32;
        }
    }
    if (m < 0) neg(r);
    return r;
}

// limb k of a, or `fill` when k is outside [0, N) (k may be a runtime value: the limbs
// are selected with compile-time indices so that they stay in registers)
template <int N>
MW_HD uint32_t limb_or(const Int<N> &a, int k, uint32_t fill) {
    uint32_t r = fill;
#pragma unroll
    for (int i = 0; i < N; ++i) r = (k == i) ? a.w[i] : r;
    return r;
}

// arithmetic shift right by s, 0 <= s < 32N
template <int N>
MW_HD void sar(Int<N> &a, int s) {
    const uint32_t ext = is_neg(a) ? 0xffffffffu : 0u;
    const int ws = s >> 5, bs = s & 31;
    Int<N> r;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const uint32_t lo = limb_or(a, i + ws, ext);
        const uint32_t hi = limb_or(a, i + ws + 1, ext);
        r.w[i] = bs ? ((lo >> bs) | (hi << (32 - bs))) : lo;
    }
    a = r;
}

// sign-extend / truncate between widths
template <int N, int M>
MW_HD Int<N> resize(const Int<M> &a) {
    Int<N> r;
    uint32_t ext = is_neg(a) ? 0xffffffffu : 0u;
#pragma unroll
    for (int i = 0; i < N; ++i) r.w[i] = i < M ? a.w[i] : ext;
    return r;
}

// true if the two's complement value fits in `bits` bits (sign included)
template <int N>
MW_HD bool fits_bits(const Int<N> &a, int bits) {
    uint32_t ext = is_neg(a) ? 0xffffffffu : 0u;
    for (int b = bits - 1; b < 32 * N; ++b) {
        uint32_t bit = (a.w[b >> 5] >> (b & 31)) & 1u;
        if (bit != (ext & 1u)) return false;
    }
    return true;
}

// Nearest double (round half to even) of the exact integer.
template <int N>
MW_HD double to_double(const Int<N> &a) {
    Int<N> m = a;
    bool negv = is_neg(m);
    if (negv) neg(m);
    int top = -1;
    uint32_t topw = 0;
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (m.w[i]) {
            top = i;
            topw = m.w[i];
        }
    if (top < 0) return 0.0;
    // 64-bit window holding the leading one, plus a sticky bit for what lies below
    int lz = __builtin_clz(topw);
    int msb = top * 32 + (31 - lz);  // index of the leading one
    uint64_t win;
    bool sticky = false;
    if (msb < 64) {
        win = (uint64_t)m.w[0] | (N > 1 ? ((uint64_t)m.w[1] << 32) : 0);
        double d = (double)(uint32_t)(win >> 32) * 4294967296.0 + (double)(uint32_t)win;
        return negv ? -d : d;
    }
    int lowbit = msb - 63;  // window = bits [lowbit, msb]
    Int<N> t = m;
    // sticky = any bit below lowbit
#pragma unroll
    for (int i = 0; i < N; ++i) {
        int b0 = i * 32;
        if (b0 + 32 <= lowbit) {
            if (t.w[i]) sticky = true;
        } else if (b0 < lowbit) {
            uint32_t mask = (1u << (lowbit - b0)) - 1u;
            if (t.w[i] & mask) sticky = true;
        }
    }
    sar(t, lowbit);
    win = (uint64_t)t.w[0] | ((uint64_t)t.w[1] << 32);
    if (sticky) win |= 1u;
    // two exactly representable halves, one rounding in the final add
    double hi = (double)(uint32_t)(win >> 32) * 4294967296.0;
    double lo = (double)(uint32_t)win;
    double d = hi + lo;
    // scale by 2^lowbit (exact)
    int e = lowbit;
    while (e > 0) {
        int s = e > 512 ? 512 : e;
        d *= __builtin_ldexp(1.0, s);
        e -= s;
    }
    return negv ? -d : d;
}

}  // namespace mw
