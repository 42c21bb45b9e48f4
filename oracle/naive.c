/*
 * Naive direct-sum CPU oracle for 3D geometric moments -- TEST INFRASTRUCTURE ONLY.
 *
 * Computes M_pqr = sum_{x,y,z} V(x,y,z) x^p y^q z^r  (Diggin & Diggin, "Fast 3D
 * Image Moments", arXiv 2012.08099, Section 1, eq. 2; bounds 0 <= x < L,
 * 0 <= y < M, 0 <= z < N; 0^0 = 1) in exact 128-bit integer arithmetic.
 *
 * Two entry points, both plain definitions of eq. (2):
 *   oracle_moments_direct  - per voxel, every monomial (the "naive" method the paper
 *                            times in Section 6), OpenMP over z;
 *   oracle_moments_hoisted - the same sum with loop-invariant powers hoisted:
 *                            sum_z z^r sum_y y^q sum_x x^p V.
 * Both refuse (return -2) when the largest possible moment could overflow a signed
 * 128-bit integer, so a result that is returned is exact.
 *
 * Volume layout: V[z][y][x], x contiguous; elem_bytes is 1 (uint8) or 2 (uint16).
 * Output: C(K+3,3) moments in graded order (p+q+r ascending; then p descending; then
 * q descending), each as two uint64 words (low, high) of a two's complement int128.
 * Only tests/ and the CPU-baseline leg of the benchmark load this library.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

static int n_moments(int K) { return (K + 1) * (K + 2) * (K + 3) / 6; }

static int bitlen_u128(u128 v) {
    int b = 0;
    while (v) { b++; v >>= 1; }
    return b;
}

static int bitlen_u64(uint64_t v) {
    int b = 0;
    while (v) { b++; v >>= 1; }
    return b;
}

static uint32_t voxel(const void *vol, int elem_bytes, size_t idx) {
    if (elem_bytes == 1) return ((const uint8_t *)vol)[idx];
    return ((const uint16_t *)vol)[idx];
}

/* Largest voxel value actually present. */
static uint32_t volume_max(const void *vol, int elem_bytes, size_t n) {
    uint32_t m = 0;
    for (size_t i = 0; i < n; i++) {
        uint32_t v = voxel(vol, elem_bytes, i);
        if (v > m) m = v;
    }
    return m;
}

/* Upper bound check: vmax * nvox * cmax^K must stay below 2^126. */
static int bound_ok(uint32_t vmax, int64_t L, int64_t M, int64_t N, int K) {
    int64_t cmax = L - 1;
    if (M - 1 > cmax) cmax = M - 1;
    if (N - 1 > cmax) cmax = N - 1;
    if (cmax < 1) cmax = 1;
    int bits = bitlen_u64(vmax) + bitlen_u64((uint64_t)(L * M * N)) + K * bitlen_u64((uint64_t)cmax);
    return bits <= 126;
}

/* graded position of (p,q,r) */
static int mindex(int p, int q, int r) {
    int n = p + q + r;
    return n * (n + 1) * (n + 2) / 6 + (n - p) * (n - p + 1) / 2 + (n - p - q);
}

static void store(uint64_t *out, int idx, i128 v) {
    u128 u = (u128)v;
    out[2 * idx] = (uint64_t)u;
    out[2 * idx + 1] = (uint64_t)(u >> 64);
}

int oracle_moments_direct(const void *vol, int elem_bytes, int64_t L, int64_t M, int64_t N,
                          int K, uint64_t *out) {
    if (!vol || !out || L <= 0 || M <= 0 || N <= 0 || K < 0 || (elem_bytes != 1 && elem_bytes != 2))
        return -1;
    size_t nvox = (size_t)L * (size_t)M * (size_t)N;
    if (!bound_ok(volume_max(vol, elem_bytes, nvox), L, M, N, K)) return -2;
    int nm = n_moments(K);
    /* monomial exponent tables in graded order */
    int *P = malloc(sizeof(int) * nm), *Q = malloc(sizeof(int) * nm), *R = malloc(sizeof(int) * nm);
    for (int n = 0, i = 0; n <= K; n++)
        for (int p = n; p >= 0; p--)
            for (int q = n - p; q >= 0; q--, i++) { P[i] = p; Q[i] = q; R[i] = n - p - q; }
    i128 *total = calloc((size_t)nm, sizeof(i128));
#pragma omp parallel
    {
        i128 *acc = calloc((size_t)nm, sizeof(i128));
        i128 px[17], py[17], pz[17];
#pragma omp for schedule(static)
        for (int64_t z = 0; z < N; z++) {
            pz[0] = 1;
            for (int k = 1; k <= K; k++) pz[k] = pz[k - 1] * z;
            for (int64_t y = 0; y < M; y++) {
                py[0] = 1;
                for (int k = 1; k <= K; k++) py[k] = py[k - 1] * y;
                for (int64_t x = 0; x < L; x++) {
                    uint32_t v = voxel(vol, elem_bytes, ((size_t)z * M + y) * L + x);
                    if (!v) continue;
                    px[0] = 1;
                    for (int k = 1; k <= K; k++) px[k] = px[k - 1] * x;
                    for (int i = 0; i < nm; i++) acc[i] += (i128)v * px[P[i]] * py[Q[i]] * pz[R[i]];
                }
            }
        }
#pragma omp critical
        for (int i = 0; i < nm; i++) total[i] += acc[i];
        free(acc);
    }
    for (int i = 0; i < nm; i++) store(out, i, total[i]);
    free(total); free(P); free(Q); free(R);
    return 0;
}

int oracle_moments_hoisted(const void *vol, int elem_bytes, int64_t L, int64_t M, int64_t N,
                           int K, uint64_t *out) {
    if (!vol || !out || L <= 0 || M <= 0 || N <= 0 || K < 0 || (elem_bytes != 1 && elem_bytes != 2))
        return -1;
    size_t nvox = (size_t)L * (size_t)M * (size_t)N;
    if (!bound_ok(volume_max(vol, elem_bytes, nvox), L, M, N, K)) return -2;
    int K1 = K + 1;
    /* B[z][p][q] = sum_y y^q sum_x x^p V */
    i128 *B = calloc((size_t)N * K1 * K1, sizeof(i128));
#pragma omp parallel
    {
        i128 *A = malloc(sizeof(i128) * K1);
        i128 *xp = malloc(sizeof(i128) * (size_t)L * K1);
        for (int64_t x = 0; x < L; x++) {
            xp[x * K1] = 1;
            for (int k = 1; k <= K; k++) xp[x * K1 + k] = xp[x * K1 + k - 1] * x;
        }
#pragma omp for schedule(static)
        for (int64_t z = 0; z < N; z++) {
            i128 *Bz = B + (size_t)z * K1 * K1;
            for (int64_t y = 0; y < M; y++) {
                for (int p = 0; p <= K; p++) A[p] = 0;
                for (int64_t x = 0; x < L; x++) {
                    uint32_t v = voxel(vol, elem_bytes, ((size_t)z * M + y) * L + x);
                    if (!v) continue;
                    for (int p = 0; p <= K; p++) A[p] += (i128)v * xp[x * K1 + p];
                }
                i128 yq = 1;
                for (int q = 0; q <= K; q++) {
                    for (int p = 0; p + q <= K; p++) Bz[p * K1 + q] += yq * A[p];
                    yq *= y;
                }
            }
        }
        free(A); free(xp);
    }
    int nm = n_moments(K);
    i128 *Mv = calloc((size_t)nm, sizeof(i128));
    for (int64_t z = 0; z < N; z++) {
        i128 zr = 1;
        for (int r = 0; r <= K; r++) {
            for (int p = 0; p + r <= K; p++)
                for (int q = 0; p + q + r <= K; q++)
                    Mv[mindex(p, q, r)] += zr * B[((size_t)z * K1 + p) * K1 + q];
            zr *= z;
        }
    }
    for (int i = 0; i < nm; i++) store(out, i, Mv[i]);
    free(Mv); free(B);
    return 0;
}

int oracle_num_threads(void) {
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}

/* keep the helper referenced so -Wall stays quiet */
int oracle_bitlen_probe(uint64_t lo, uint64_t hi) { return bitlen_u128(((u128)hi << 64) | lo); }
