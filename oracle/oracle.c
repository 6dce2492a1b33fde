/*
 * Plain, slow CPU reference arithmetic for the Hyena homomorphic convolution
 * (Roh & Choi, "Hyena: Optimizing Homomorphically Encrypted Convolution for
 * Private CNN Inference", ICCAD 2024).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the checker the GPU library is
 * compared against. Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it. It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * Every routine is the plain definition written out: schoolbook negacyclic
 * products with one exact reduction per term, O(N^2) evaluation of the
 * number-theoretic transform, and no blocking, fusion or reordering beyond
 * splitting independent outputs across OpenMP threads.
 *
 * Rings: R_q = Z_q[X]/(X^N + 1) (Background, "Homomorphic Operations in
 * BFV"), one residue ring per RNS limb q_i < 2^31. All residues are canonical,
 * in [0, q_i).
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (a * b) % q; }

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t q)
{
    uint64_t r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}

static uint32_t bitrev(uint32_t x, uint32_t logn)
{
    uint32_t r = 0;
    for (uint32_t i = 0; i < logn; i++) r |= ((x >> i) & 1u) << (logn - 1 - i);
    return r;
}

/*
 * r = a * b in Z_q[X]/(X^N+1), dense schoolbook: the coefficient of X^k is
 * sum_{i<=k} a_i b_{k-i} - sum_{i>k} a_i b_{N+k-i}  (X^N = -1).
 */
void orc_negacyclic_mul(const uint32_t *a, const uint32_t *b, uint32_t *r,
                        uint32_t N, uint32_t q)
{
    /* each sum has at most N < 2^15 products below 2^62: exact in 128 bits */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)N; k++) {
        unsigned __int128 pos = 0, neg = 0;
        for (uint32_t i = 0; i <= (uint32_t)k; i++)
            pos += (uint64_t)a[i] * b[k - i];
        for (uint32_t i = (uint32_t)k + 1; i < N; i++)
            neg += (uint64_t)a[i] * b[N + k - i];
        uint64_t p = (uint64_t)(pos % q), n = (uint64_t)(neg % q);
        r[k] = (uint32_t)((p + q - n) % q);
    }
}

/*
 * Sum over input ciphertexts of ciphertext-times-kernel-polynomial products,
 * each kernel polynomial given by its nonzero taps (exponent, small signed
 * integer weight):
 *
 *   out[u][p][i] = sum_{g} ct[tile(u)][g][p][i] * K_{o(u), g}  mod (X^N+1, q_i)
 *
 * for every requested output u = (tile, output channel), both ciphertext
 * parts p and every limb i. This is the padded convolution written as
 * PMult/CMult by scalar weights followed by HAdd (Background, "Prior Art on
 * Homomorphic Convolution"; "Enabling Output Channel Packing"): multiplying by the monomial
 * w * X^e is CMult by w after a rotation by e.
 *
 * ct       : uint32 [n_tiles][n_groups][2][L][N]
 * tap_ptr  : int64 [Co*n_groups + 1] CSR offsets into tap_exp / tap_w for
 *            the kernel polynomial of (o, g) at index o*n_groups + g
 * tap_exp  : uint32 exponents in [0, N)
 * tap_w    : int32 weights
 * sel_tile, sel_o : the n_sel requested outputs
 * out      : uint32 [n_sel][2][L][N]
 *
 * Accumulation is exact in int64: |sum| <= (#taps) * 2^31 * max|w|, which is
 * below 2^47 for every layer with at most 9*1024 taps and |w| <= 8 per
 * output; callers keep (#taps)*max|w| < 2^31.
 */
void orc_conv_products(const uint32_t *ct, uint32_t n_tiles, uint32_t n_groups,
                       uint32_t L, uint32_t N, const uint32_t *primes,
                       const int64_t *tap_ptr, const uint32_t *tap_exp,
                       const int32_t *tap_w, uint32_t n_sel,
                       const uint32_t *sel_tile, const uint32_t *sel_o,
                       uint32_t *out)
{
    (void)n_tiles;
    int64_t items = (int64_t)n_sel * 2 * L;
#pragma omp parallel
    {
        /* int64 accumulators, one per output coefficient, one buffer per thread */
        int64_t *a = (int64_t *)malloc(sizeof(int64_t) * N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t it = 0; it < items; it++) {
            uint32_t u = (uint32_t)(it / (2 * L));
            uint32_t p = (uint32_t)((it / L) % 2);
            uint32_t i = (uint32_t)(it % L);
            uint32_t tau = sel_tile[u], o = sel_o[u];
            int64_t q = primes[i];
            uint32_t *dst = out + (((size_t)u * 2 + p) * L + i) * N;
            for (uint32_t k = 0; k < N; k++) a[k] = 0;
            for (uint32_t g = 0; g < n_groups; g++) {
                const uint32_t *src = ct + ((((size_t)tau * n_groups + g) * 2 + p) * L + i) * N;
                int64_t t0 = tap_ptr[(size_t)o * n_groups + g];
                int64_t t1 = tap_ptr[(size_t)o * n_groups + g + 1];
                for (int64_t t = t0; t < t1; t++) {
                    uint32_t e = tap_exp[t];
                    int64_t w = tap_w[t];
                    /* X^e * X^j = X^(j+e); wraps past X^N with a sign flip */
                    for (uint32_t j = 0; j < N; j++) {
                        uint32_t d = j + e;
                        if (d < N) a[d] += w * (int64_t)src[j];
                        else       a[d - N] -= w * (int64_t)src[j];
                    }
                }
            }
            for (uint32_t k = 0; k < N; k++) {
                int64_t r = a[k] % q;
                if (r < 0) r += q;
                dst[k] = (uint32_t)r;
            }
        }
        free(a);
    }
}

/*
 * Forward negacyclic NTT by direct evaluation (O(N^2)):
 *   out[k] = sum_j a[j] * psi^((2*brv(k)+1)*j)  mod q
 * i.e. a(X) evaluated at the N odd powers of the primitive 2N-th root psi,
 * listed in bit-reversed order of k. Only the outputs listed in ks (n_k of
 * them; ks == NULL means all N in order) are produced.
 */
void orc_ntt_eval(const uint32_t *a, uint32_t *out, uint32_t N, uint32_t q,
                  uint32_t psi, const uint32_t *ks, uint32_t n_k)
{
    uint32_t logn = 0;
    while ((1u << logn) < N) logn++;
    uint32_t cnt = ks ? n_k : N;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < (int64_t)cnt; m++) {
        uint32_t k = ks ? ks[m] : (uint32_t)m;
        uint64_t w = powmod(psi, 2ull * bitrev(k, logn) + 1, q);
        uint64_t x = 1, s = 0;
        for (uint32_t j = 0; j < N; j++) {
            s = (s + mulmod(a[j], x, q)) % q;
            x = mulmod(x, w, q);
        }
        out[m] = (uint32_t)s;
    }
}

/*
 * Inverse of orc_ntt_eval (interpolation through the N roots of X^N+1):
 *   a[j] = N^-1 * sum_k A[k] * psi^(-(2*brv(k)+1)*j)  mod q
 */
void orc_intt_eval(const uint32_t *A, uint32_t *out, uint32_t N, uint32_t q,
                   uint32_t psi)
{
    uint32_t logn = 0;
    while ((1u << logn) < N) logn++;
    uint64_t psi_inv = powmod(psi, q - 2, q);
    uint64_t n_inv = powmod(N, q - 2, q);
    /* table of psi^-e for e in [0, 2N): psi has order 2N */
    uint64_t *pw = (uint64_t *)malloc(sizeof(uint64_t) * 2 * N);
    pw[0] = 1;
    for (uint32_t e = 1; e < 2 * N; e++) pw[e] = mulmod(pw[e - 1], psi_inv, q);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)N; j++) {
        uint64_t s = 0;
        for (uint32_t k = 0; k < N; k++) {
            uint64_t e = ((2ull * bitrev(k, logn) + 1) * (uint64_t)j) % (2ull * N);
            s = (s + mulmod(A[k], pw[e], q)) % q;
        }
        out[j] = (uint32_t)mulmod(s, n_inv, q);
    }
    free(pw);
}
