// BFV client-side definitions shared by the host operations (crypto.cpp) and
// their batched device versions (client.hip), so both draw the same randomness
// and use the same constants ("Homomorphic Operations in BFV" section).
#pragma once
#include <cstdint>
#include <vector>

#include "internal.h"

// Output number ctr of a SplitMix64 generator seeded with key: the counter-based
// generator behind the secret key and the encryption randomness.
__host__ __device__ inline uint64_t hy_sm64(uint64_t key, uint64_t ctr) {
    uint64_t z = key + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr int kErrBound = 32;   // error bound B = 10 sigma; the sampler has 2B thresholds

std::vector<uint32_t> bfv_delta_residues(const hyena_ctx *c);   // floor(q / t) mod q_i
void bfv_error_thresholds(uint64_t *t64);                        // the 2B sampler thresholds
// decryption's RNS rounding, per limb: A_i = floor(t y_i / q_i) and
// F_i = floor(2^64 (t y_i mod q_i) / q_i), y_i = (q / q_i)^-1 mod q_i
void bfv_hps_constants(const hyena_ctx *c, uint64_t *A, uint64_t *F);

// Decryption's v = c0 + c1 s for n ciphertexts ct [n][2][L][N] into
// v [n][L][N] in one kernel: per limb-polynomial the forward transform of c1,
// the product with mul [L][N] (NTT(s) 2^32 mod q_i), the inverse transform
// and the sum with c0. mul 16-byte aligned; v must not overlap ct (ntt.hip).
int launch_ntt_c1s_add(const hyena_ctx *c, const uint32_t *ct, size_t n, uint32_t *v, const uint32_t *mul,
                       hipStream_t s);

// Encryption's uniform polynomials drawn inside the transform: for message m
// and limb i, a = floor(q_i sm64(seed, 2 ((m L + i) N + j)) / 2^64); writes
// c1 = -a into ct [n][2][L][N] and a s mod q_i = INTT(NTT(a) . NTT(s)) into
// dst [n][L][N], with mul [L][N] holding NTT(s) 2^32 mod q_i, in one kernel
// (ntt.hip).
int launch_ntt_sample_as(const hyena_ctx *c, uint32_t *ct, size_t n, uint32_t *dst, const uint32_t *mul,
                         uint64_t seed, hipStream_t s);
