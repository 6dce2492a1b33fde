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
void bfv_hps_constants(const hyena_ctx *c, uint64_t *A, uint64_t *B);   // decryption, per limb

// Forward NTT of P polynomials with a gathered source and a pointwise product:
// dst[p][i] = NTT_i(src[p][i]) . mul[i] mod q_i, src[p][i] at
// src + p src_stride + i N, dst contiguous [P][L][N], mul [L][N] holding
// m 2^32 mod q_i (Montgomery form). src may equal dst with src_stride = L N;
// otherwise they must not overlap. dst and mul 16-byte aligned (ntt.hip).
int launch_ntt_fwd_mul(const hyena_ctx *c, const uint32_t *src, size_t src_stride, size_t P, uint32_t *dst,
                       const uint32_t *mul, hipStream_t s);

// Inverse NTT of P polynomials a [P][L][N] in place, adding as it stores
// limb i of polynomial p at add_src + p add_stride + i N (mod q_i; canonical
// inputs); add_src must not overlap a; a 16-byte aligned (ntt.hip).
int launch_ntt_inv_add(const hyena_ctx *c, uint32_t *a, size_t P, const uint32_t *add_src, size_t add_stride,
                       hipStream_t s);

// Encryption's uniform polynomials drawn inside the forward NTT: for message m
// and limb i, a = floor(q_i sm64(seed, 2 ((m L + i) N + j)) / 2^64); writes
// c1 = -a into ct [n][2][L][N] and NTT(a) . mul into dst [n][L][N] (ntt.hip).
int launch_ntt_fwd_sample(const hyena_ctx *c, uint32_t *ct, size_t n, uint32_t *dst, const uint32_t *mul,
                          uint64_t seed, hipStream_t s);
