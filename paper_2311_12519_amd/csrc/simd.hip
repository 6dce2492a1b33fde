// The SIMD (batch-encoded) pieces of the paper's own setting on gfx950: the
// parameter selection of the "Optimal Parameter Selection" section (h_{p,n}
// and the k minimising k h_{p,n} mod p), batch encoding with a prime
// plaintext modulus p = 1 mod 2n, the Galois automorphisms behind HRot, and
// PMult by a sparse plaintext such as the [k, -k] one (two monomials).
//
// Slot layout: slot s < n/2 holds the value at zeta^(3^s mod 2n), slot n/2 + s
// the value at zeta^(-3^s mod 2n), zeta the least primitive 2n-th root of
// unity mod p (the context's psi). X -> X^3 rotates both rows by one slot,
// X -> X^(2n-1) swaps them.
#include <cmath>

#include "internal.h"

namespace {

constexpr uint32_t STH = 256;                 // threads per block, one coefficient each
constexpr uint32_t MAX_TERMS = 16;            // monomials of a sparse plaintext

__device__ __forceinline__ uint32_t scsub(uint32_t x, uint32_t q) { return min(x, x - q); }

// a b 2^-32 mod q in [0, q) for a, b < q
__device__ __forceinline__ uint32_t smont(uint32_t a, uint32_t b, uint32_t q, uint32_t qn) {
    const uint64_t t = (uint64_t)a * b;
    const uint32_t m = (uint32_t)t * qn;
    return scsub((uint32_t)(((uint64_t)m * q + t) >> 32), q);
}

__device__ __forceinline__ uint32_t brev(uint32_t x, uint32_t logn) { return __brev(x) >> (32 - logn); }

// Lazy key-switch sums: products of residues below q summed in 64 bits and
// folded (hi 2^32 + lo -> hi r32 + lo, r32 = 2^32 mod q) before they could
// reach 2^64; ks_reduce folds once more (bringing the sum below q 2^32) and
// takes one Montgomery reduction: the sum times 2^-32 mod q, in [0, q).
__device__ __forceinline__ uint64_t ks_fold(uint64_t acc, uint32_t r32) {
    return (uint64_t)(uint32_t)(acc >> 32) * r32 + (uint32_t)acc;
}

__device__ __forceinline__ uint32_t ks_reduce(uint64_t acc, const LimbConst &lc) {
    const uint64_t y = ks_fold(acc, lc.r32);
    const uint32_t m = (uint32_t)y * lc.qinv_neg;
    return scsub((uint32_t)(((uint64_t)m * lc.q + y) >> 32), lc.q);
}

// sum_t d[t] k[t] 2^-32 mod q for TD terms below q < 2^31: even and odd terms
// in two independent chains, each folded after every second product (a
// fold leaves less than (r32 + 1) 2^32 <= 2^63, and two products add less
// than 2^63, so no sum reaches 2^64, with no branch between the terms)
template <uint32_t TD>
__device__ __forceinline__ uint32_t ks_dot(const uint32_t (&d)[TD + 1], const uint32_t (&k)[TD], const LimbConst &lc) {
    uint64_t a[2] = {0, 0};
#pragma unroll
    for (uint32_t t = 0; t < TD; t++) {
        a[t & 1] += (uint64_t)d[t] * k[t];
        if ((t & 3) == 3 && t + 1 < TD) {
            a[0] = ks_fold(a[0], lc.r32);
            a[1] = ks_fold(a[1], lc.r32);
        }
    }
    // each folded chain is below (r32 + 1) 2^32, so their sum fits 64 bits
    return ks_reduce(ks_fold(a[0], lc.r32) + ks_fold(a[1], lc.r32), lc);
}

// NTT index (evaluation at psi^(2 brv(k) + 1)) of slot s
__device__ __forceinline__ uint32_t slot_to_ntt(uint32_t s, uint32_t logN) {
    const uint32_t N = 1u << logN, mask = 2 * N - 1, h = N / 2;
    const uint32_t r = s < h ? s : s - h;
    uint32_t e = 1, b = 3;                     // 3^r mod 2N by squaring
    for (uint32_t x = r; x; x >>= 1) {
        if (x & 1) e = (e * b) & mask;
        b = (b * b) & mask;
    }
    if (s >= h) e = (2 * N - e) & mask;
    return brev((e - 1) >> 1, logN);
}

// Blocks walk chunks of 256 coefficients of a [P][N] (or [P][L][N]) array.
__global__ void __launch_bounds__(STH) slots_to_ntt_kernel(const uint32_t *slots, uint32_t *ntt, size_t P,
                                                           uint32_t logN, uint32_t p) {
    const size_t chunks = P << (logN - 8);
    for (size_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const size_t poly = c >> (logN - 8);
        const uint32_t s = ((uint32_t)(c & ((1u << (logN - 8)) - 1)) << 8) + threadIdx.x;
        const uint32_t v = slots[(poly << logN) + s];
        ntt[(poly << logN) + slot_to_ntt(s, logN)] = v < p ? v : v % p;
    }
}

__global__ void __launch_bounds__(STH) ntt_to_slots_kernel(const uint32_t *ntt, uint32_t *slots, size_t P,
                                                           uint32_t logN) {
    const size_t chunks = P << (logN - 8);
    for (size_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const size_t poly = c >> (logN - 8);
        const uint32_t s = ((uint32_t)(c & ((1u << (logN - 8)) - 1)) << 8) + threadIdx.x;
        slots[(poly << logN) + s] = ntt[(poly << logN) + slot_to_ntt(s, logN)];
    }
}

// Encoding's permutation with each polynomial staged in LDS (one block per
// polynomial, arrays 16-byte aligned): the global loads and stores are 16-byte
// pieces contiguous across lanes and the scatter happens in LDS (0.051 ->
// 0.036 ms for 2048 polynomials at n = 2048, NTT included; the same staging
// for decoding's gather was slower than gathering through L2).
__global__ void __launch_bounds__(STH) slots_to_ntt_lds_kernel(const uint32_t *slots, uint32_t *ntt, size_t P,
                                                               uint32_t logN, uint32_t p) {
    extern __shared__ uint32_t sh[];
    const uint32_t N = 1u << logN;
    for (size_t poly = blockIdx.x; poly < P; poly += gridDim.x) {
        const uint4 *src = reinterpret_cast<const uint4 *>(slots + (poly << logN));
        for (uint32_t c = threadIdx.x; c < N / 4; c += STH) {
            const uint4 v = src[c];
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int u = 0; u < 4; u++) sh[slot_to_ntt(4 * c + u, logN)] = w[u] < p ? w[u] : w[u] % p;
        }
        __syncthreads();
        uint4 *dst = reinterpret_cast<uint4 *>(ntt + (poly << logN));
        for (uint32_t c = threadIdx.x; c < N / 4; c += STH) dst[c] = reinterpret_cast<const uint4 *>(sh)[c];
        __syncthreads();   // the stores' LDS reads precede the next polynomial's writes
    }
}

// out = in(X^g) per limb-polynomial, gathered: output coefficient i comes from
// j = i g^-1 mod 2N (sign + if j < N, else from j - N with sign -)
__global__ void __launch_bounds__(STH) automorphism_kernel(const uint32_t *in, uint32_t *out, size_t polys,
                                                           uint32_t logN, uint32_t L, uint32_t ginv, LimbTable lt) {
    const uint32_t N = 1u << logN, mask = 2 * N - 1;
    const uint32_t chunks = (uint32_t)(polys << (logN - 8));   // < 2^31 (checked on the host)
    for (uint32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const uint32_t poly = c >> (logN - 8);   // limb-polynomial index, limb = poly mod L
        const uint32_t q = lt.c[poly % L].q;
        const uint32_t i = ((c & ((1u << (logN - 8)) - 1)) << 8) + threadIdx.x;
        const uint32_t j = (i * ginv) & mask;
        const size_t base = (size_t)poly << logN;
        uint32_t v;
        if (j < N) {
            v = in[base + j];
        } else {
            const uint32_t a = in[base + j - N];
            v = a ? q - a : 0;
        }
        out[base + i] = v;
    }
}

// The same permutation with the limb-polynomial staged in LDS: a block takes
// whole limb-polynomials (grid-stride), reads one with 16-byte loads
// contiguous across lanes, gathers the permuted coefficients from LDS and
// writes them back with 16-byte stores contiguous across lanes, so HBM sees
// one plain read and one plain write of every word. N words of dynamic LDS.
__global__ void __launch_bounds__(STH) automorphism_lds_kernel(const uint32_t *in, uint32_t *out, size_t polys,
                                                               uint32_t logN, uint32_t L, uint32_t ginv,
                                                               LimbTable lt) {
    extern __shared__ uint32_t sh[];
    const uint32_t N = 1u << logN, mask = 2 * N - 1;
    for (size_t poly = blockIdx.x; poly < polys; poly += gridDim.x) {
        const uint32_t q = lt.c[poly % L].q;
        const uint4 *src = reinterpret_cast<const uint4 *>(in + (poly << logN));
        uint4 *dst = reinterpret_cast<uint4 *>(out + (poly << logN));
        for (uint32_t c = threadIdx.x; c < N / 4; c += STH) reinterpret_cast<uint4 *>(sh)[c] = src[c];
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < N / 4; c += STH) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint32_t j = ((4 * c + u) * ginv) & mask;
                const uint32_t a = sh[j & (N - 1)];
                v[u] = (j < N || a == 0) ? a : q - a;
            }
            dst[c] = make_uint4(v[0], v[1], v[2], v[3]);
        }
        __syncthreads();   // the gathers precede the next polynomial's loads
    }
}

struct Sparse {
    uint32_t n;                       // monomials
    uint32_t e[MAX_TERMS];            // exponents, < 2N
    uint32_t cm[HYENA_MAX_LIMBS][MAX_TERMS];   // c_t 2^32 mod q_i (Montgomery form)
};

// out = sum_t c_t X^{e_t} in, per limb-polynomial: coefficient i takes
// +c_t in[d] for d = i - e_t mod 2N below N, -c_t in[d - N] otherwise
__global__ void __launch_bounds__(STH) pmult_sparse_kernel(const uint32_t *in, uint32_t *out, size_t polys,
                                                           uint32_t logN, uint32_t L, LimbTable lt, Sparse sp) {
    const uint32_t N = 1u << logN, mask = 2 * N - 1;
    const uint32_t chunks = (uint32_t)(polys << (logN - 8));   // < 2^31 (checked on the host)
    for (uint32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const uint32_t poly = c >> (logN - 8);
        const uint32_t limb = poly % L;
        const uint32_t q = lt.c[limb].q, qn = lt.c[limb].qinv_neg;
        const uint32_t i = ((c & ((1u << (logN - 8)) - 1)) << 8) + threadIdx.x;
        const size_t base = (size_t)poly << logN;
        uint32_t acc = 0;
        for (uint32_t t = 0; t < sp.n; t++) {
            const uint32_t d = (i - sp.e[t]) & mask;
            uint32_t a = in[base + (d & (N - 1))];
            if (d >= N) a = a ? q - a : 0;
            acc = scsub(acc + smont(a, sp.cm[limb][t], q, qn), q);
        }
        out[base + i] = acc;
    }
}

// The same sparse product with the limb-polynomial staged in LDS (16-byte
// loads and stores contiguous across lanes; the shifted reads hit LDS).
__global__ void __launch_bounds__(STH) pmult_sparse_lds_kernel(const uint32_t *in, uint32_t *out, size_t polys,
                                                               uint32_t logN, uint32_t L, LimbTable lt, Sparse sp) {
    extern __shared__ uint32_t sh[];
    const uint32_t N = 1u << logN, mask = 2 * N - 1;
    for (size_t poly = blockIdx.x; poly < polys; poly += gridDim.x) {
        const uint32_t limb = (uint32_t)(poly % L);
        const uint32_t q = lt.c[limb].q, qn = lt.c[limb].qinv_neg;
        const uint4 *src = reinterpret_cast<const uint4 *>(in + (poly << logN));
        uint4 *dst = reinterpret_cast<uint4 *>(out + (poly << logN));
        for (uint32_t c = threadIdx.x; c < N / 4; c += STH) reinterpret_cast<uint4 *>(sh)[c] = src[c];
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < N / 4; c += STH) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint32_t i = 4 * c + u;
                uint32_t acc = 0;
                for (uint32_t t = 0; t < sp.n; t++) {
                    const uint32_t d = (i - sp.e[t]) & mask;
                    uint32_t a = sh[d & (N - 1)];
                    if (d >= N) a = a ? q - a : 0;
                    acc = scsub(acc + smont(a, sp.cm[limb][t], q, qn), q);
                }
                v[u] = acc;
            }
            dst[c] = make_uint4(v[0], v[1], v[2], v[3]);
        }
        __syncthreads();
    }
}

// x <- x 2^32 mod q (a Montgomery product by 2^64 mod q), [polys][L][N]
__global__ void __launch_bounds__(STH) scale_montgomery_kernel(uint32_t *x, size_t polys, uint32_t logN, uint32_t L,
                                                               LimbTable lt) {
    const size_t chunks = polys << (logN - 8);
    for (size_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const LimbConst &lc = lt.c[(uint32_t)((c >> (logN - 8)) % L)];
        uint32_t *p = x + (c << 8) + threadIdx.x;
        *p = smont(*p, lc.r64, lc.q, lc.qinv_neg);
    }
}

constexpr uint32_t MAX_ROT = 64;

struct RotArgs {
    uint32_t n_rot, D, b;
    uint32_t g[MAX_ROT];
};

// work[m][i D + j][k] <- digit j (base 2^b) of c1's residues on limb i, the
// same integer on every limb k; work[m][L D][k] <- c0 on limb k
__global__ void __launch_bounds__(STH) decompose_kernel(const uint32_t *ct, uint32_t *work, size_t n_ct,
                                                        uint32_t logN, uint32_t L, RotArgs ra) {
    const uint32_t N = 1u << logN, mask = (1u << ra.b) - 1, T = L * ra.D + 1;
    const size_t LN = (size_t)L << logN;
    const uint32_t chunks = (uint32_t)((n_ct * L) << (logN - 8));   // < 2^31 (checked on the host)
    for (uint32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const uint32_t mk = c >> (logN - 8);                 // m L + k
        const uint32_t m = mk / L, k = mk % L;
        const uint32_t x = ((c & ((1u << (logN - 8)) - 1)) << 8) + threadIdx.x;
        const uint32_t *c0 = ct + (size_t)m * 2 * LN, *c1 = c0 + LN;
        uint32_t *w = work + (size_t)m * T * LN + (size_t)k * N + x;
        for (uint32_t i = 0; i < L; i++) {
            const uint32_t v = c1[(size_t)i * N + x];
            for (uint32_t j = 0; j < ra.D; j++) w[(size_t)(i * ra.D + j) * LN] = (v >> (ra.b * j)) & mask;
        }
        w[(size_t)(T - 1) * LN] = c0[(size_t)k * N + x];
    }
}

// NTT domain: out[m][r][0][k][s] = c0^[s_r] + sum_t d_t^[s_r] K_r,t,0[k][s],
//             out[m][r][1][k][s] = sum_t d_t^[s_r] K_r,t,1[k][s],
// s_r the NTT index of the exponent (2 brv(s) + 1) g_r mod 2N (the
// automorphism X -> X^g_r permutes evaluation points); K in Montgomery form
__global__ void __launch_bounds__(STH) keyswitch_kernel(const uint32_t *work, const uint32_t *ksk, uint32_t *out,
                                                        size_t n_ct, uint32_t logN, uint32_t L, LimbTable lt,
                                                        RotArgs ra) {
    const uint32_t N = 1u << logN, mask = 2 * N - 1, TD = L * ra.D;
    const size_t LN = (size_t)L << logN;
    // (m n_rot + r) L + k < 2^31 (checked on the host): 32-bit index arithmetic
    const uint32_t chunks = (uint32_t)(((n_ct * ra.n_rot) * L) << (logN - 8));
    for (uint32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const uint32_t mrk = c >> (logN - 8);                // (m n_rot + r) L + k
        const uint32_t k = mrk % L, mr = mrk / L;
        const uint32_t r = mr % ra.n_rot, m = mr / ra.n_rot;
        const uint32_t s = ((c & ((1u << (logN - 8)) - 1)) << 8) + threadIdx.x;
        const uint32_t e = ((2 * brev(s, logN) + 1) * ra.g[r]) & mask;
        const uint32_t sr = brev(e >> 1, logN);
        const LimbConst &lc = lt.c[k];
        const uint32_t q = lc.q, qn = lc.qinv_neg;
        const uint32_t *wm = work + (size_t)m * (TD + 1) * LN + (size_t)k * N + sr;
        const uint32_t *kr = ksk + (size_t)r * TD * 2 * LN + (size_t)k * N + s;
        uint32_t acc0 = wm[(size_t)TD * LN], acc1 = 0;
        uint32_t t = 0;
        for (; t + 4 <= TD; t += 4) {   // the twelve loads of four digit terms first
            uint32_t d[4], k0[4], k1[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                d[u] = wm[(size_t)(t + u) * LN];
                k0[u] = kr[(size_t)(2 * (t + u)) * LN];
                k1[u] = kr[(size_t)(2 * (t + u) + 1) * LN];
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                acc0 = scsub(acc0 + smont(d[u], k0[u], q, qn), q);
                acc1 = scsub(acc1 + smont(d[u], k1[u], q, qn), q);
            }
        }
        for (; t < TD; t++) {
            const uint32_t d = wm[(size_t)t * LN];
            acc0 = scsub(acc0 + smont(d, kr[(size_t)(2 * t) * LN], q, qn), q);
            acc1 = scsub(acc1 + smont(d, kr[(size_t)(2 * t + 1) * LN], q, qn), q);
        }
        uint32_t *o = out + (size_t)mr * 2 * LN + (size_t)k * N + s;
        o[0] = acc0;
        o[LN] = acc1;
    }
}

// The same key switching with TD = L D known at compile time: a thread keeps
// the 2 TD key words of its (rotation, limb, slot) in registers and serves
// KS_M ciphertexts with them, so keys are read once per KS_M ciphertexts.
constexpr uint32_t KS_M = 8;

template <uint32_t TD>
__global__ void __launch_bounds__(STH) keyswitch_keys_kernel(const uint32_t *work, const uint32_t *ksk, uint32_t *out,
                                                             uint32_t n_ct, uint32_t logN, uint32_t L, LimbTable lt,
                                                             RotArgs ra) {
    const uint32_t N = 1u << logN, mask = 2 * N - 1, cpl = 1u << (logN - 8);
    const size_t LN = (size_t)L << logN;
    const uint32_t groups = (n_ct + KS_M - 1) / KS_M;
    const uint32_t chunks = groups * ra.n_rot * L * cpl;   // < 2^31 (checked on the host)
    for (uint32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const uint32_t sch = c % cpl, rest = c / cpl;
        const uint32_t k = rest % L, rr = rest / L;
        const uint32_t r = rr % ra.n_rot, mg = rr / ra.n_rot;
        const uint32_t s = (sch << 8) + threadIdx.x;
        const uint32_t e = ((2 * brev(s, logN) + 1) * ra.g[r]) & mask;
        const uint32_t sr = brev(e >> 1, logN);
        const LimbConst &lc = lt.c[k];
        const uint32_t q = lc.q;
        const uint32_t *kr = ksk + (size_t)r * TD * 2 * LN + (size_t)k * N + s;
        uint32_t k0[TD], k1[TD];
#pragma unroll
        for (uint32_t t = 0; t < TD; t++) {
            k0[t] = kr[(size_t)(2 * t) * LN];
            k1[t] = kr[(size_t)(2 * t + 1) * LN];
        }
        const uint32_t m_end = min(n_ct, (mg + 1) * KS_M);
        for (uint32_t m = mg * KS_M; m < m_end; m++) {
            const uint32_t *wm = work + (size_t)m * (TD + 1) * LN + (size_t)k * N + sr;
            uint32_t d[TD + 1];
#pragma unroll
            for (uint32_t t = 0; t <= TD; t++) d[t] = wm[(size_t)t * LN];
            uint32_t *o = out + ((size_t)m * ra.n_rot + r) * 2 * LN + (size_t)k * N + s;
            o[0] = scsub(ks_dot<TD>(d, k0, lc) + d[TD], q);
            o[LN] = ks_dot<TD>(d, k1, lc);
        }
    }
}

// The same key switching with the rotations in the inner loop: a thread owns
// one digit slot sd of KS_R ciphertexts and one limb, loads their TD digits
// and c0 there once, and for every rotation r sums the output slot s whose
// permuted source is sd (s = brv((e_d g_r^-1 mod 2N - 1) / 2) for
// e_d = 2 brv(sd) + 1) with that rotation's keys at s. The digits are read
// once for all rotations instead of once per rotation; the keys of a
// rotation are read once per KS_R ciphertexts. The permutation maps the
// wave's aligned block of 64 source slots onto one aligned block of output
// slots, so keys are loaded and sums stored in slot order (lane j at slot
// block + j, 256 contiguous bytes per access) and moved between the wave's
// lanes by ds_bpermute (a cross-lane read that takes no LDS space).
constexpr uint32_t KS_R = 8;

struct RotInv {
    uint32_t ginv[MAX_ROT];   // g_r^-1 mod 2N
};

template <uint32_t TD>
__global__ void __launch_bounds__(STH) keyswitch_rot_kernel(const uint32_t *work, const uint32_t *ksk, uint32_t *out,
                                                            uint32_t n_ct, uint32_t logN, uint32_t L, LimbTable lt,
                                                            RotArgs ra, RotInv ri) {
    const uint32_t N = 1u << logN, mask = 2 * N - 1, cpl = 1u << (logN - 8);
    const size_t LN = (size_t)L << logN;
    const uint32_t groups = (n_ct + KS_R - 1) / KS_R;
    const uint32_t chunks = groups * L * cpl;   // < 2^31 (checked on the host)
    for (uint32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const uint32_t sch = c % cpl, rest = c / cpl;
        const uint32_t k = rest % L, mg = rest / L;
        const uint32_t sd = (sch << 8) + threadIdx.x;
        const uint32_t ed = 2 * brev(sd, logN) + 1;
        const LimbConst &lc = lt.c[k];
        const uint32_t q = lc.q;
        const uint32_t m0 = mg * KS_R, nm = min(KS_R, n_ct - m0);
        uint32_t d[KS_R][TD + 1];
#pragma unroll
        for (uint32_t u = 0; u < KS_R; u++) {
            if (u >= nm) break;
            const uint32_t *wm = work + (size_t)(m0 + u) * (TD + 1) * LN + (size_t)k * N + sd;
#pragma unroll
            for (uint32_t t = 0; t <= TD; t++) d[u][t] = wm[(size_t)t * LN];
        }
        const uint32_t lane = threadIdx.x & 63, sbase = sd - lane;
        for (uint32_t r = 0; r < ra.n_rot; r++) {
            // output slot of this lane's source slot; the wave's 64 source
            // slots fill the aligned output block at obase
            const uint32_t s = brev((((ed * ri.ginv[r]) & mask) - 1) >> 1, logN);
            const uint32_t obase = __builtin_amdgcn_readfirstlane(s & ~63u);
            // the lane stores output slot so, whose source slot is sr; keys
            // are read and sums stored at so (whole 256-byte rows), and moved
            // between lanes by ds_bpermute
            const uint32_t so = obase + lane;
            const uint32_t sr = brev((((2 * brev(so, logN) + 1) * ra.g[r]) & mask) >> 1, logN);
            const int kaddr = (int)((s - obase) << 2);   // lane that read the keys of slot s
            const int oaddr = (int)((sr - sbase) << 2);  // lane that summed slot so
            const uint32_t *kr = ksk + (size_t)r * TD * 2 * LN + (size_t)k * N + so;
            uint32_t k0[TD], k1[TD];
#pragma unroll
            for (uint32_t t = 0; t < TD; t++) {
                k0[t] = (uint32_t)__builtin_amdgcn_ds_bpermute(kaddr, (int)kr[(size_t)(2 * t) * LN]);
                k1[t] = (uint32_t)__builtin_amdgcn_ds_bpermute(kaddr, (int)kr[(size_t)(2 * t + 1) * LN]);
            }
#pragma unroll
            for (uint32_t u = 0; u < KS_R; u++) {
                if (u >= nm) break;
                const uint32_t v0 = scsub(ks_dot<TD>(d[u], k0, lc) + d[u][TD], q), v1 = ks_dot<TD>(d[u], k1, lc);
                uint32_t *o = out + ((size_t)(m0 + u) * ra.n_rot + r) * 2 * LN + (size_t)k * N + so;
                o[0] = (uint32_t)__builtin_amdgcn_ds_bpermute(oaddr, (int)v0);
                o[LN] = (uint32_t)__builtin_amdgcn_ds_bpermute(oaddr, (int)v1);
            }
        }
    }
}

// out[o] = sum_r W[o][r] in[r] mod q_i for ciphertexts [R][2][L][N]: products
// of residues by small signed integers summed exactly in a signed 64-bit word
// (|W| <= 2^16, R <= 4096: |sum| < 2^59 <= q 2^30), one reduction per output
// coefficient (CMult and HAdd without reduction, "Lazy Reduction")
__global__ void __launch_bounds__(STH) cmult_acc_kernel(const uint32_t *__restrict__ in, const int32_t *__restrict__ W,
                                                        uint32_t *__restrict__ out, uint32_t R, uint32_t O,
                                                        uint32_t logN, uint32_t L, LimbTable lt) {
    const size_t PLN = (size_t)2 * L << logN;               // words per ciphertext
    const uint32_t chunks = (uint32_t)(((size_t)O * 2 * L) << (logN - 8));   // < 2^31 (checked on the host)
    for (uint32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const uint32_t op = c >> (logN - 8);                // o (2 L) + part L + limb
        const uint32_t o = op / (2 * L), limb = op % L;
        const size_t idx = ((size_t)(op % (2 * L)) << logN) + ((c & ((1u << (logN - 8)) - 1)) << 8) + threadIdx.x;
        // the weight row is the same for every lane (scalar loads); residues are
        // below 2^31, so as signed 32-bit words their products with the
        // weights are single v_mad_i64_i32 instructions
        const int32_t *w = W + (size_t)__builtin_amdgcn_readfirstlane(o) * R;
        int64_t acc = 0;
#pragma unroll 8
        for (uint32_t r = 0; r < R; r++) acc += (int64_t)w[r] * (int64_t)(int32_t)in[(size_t)r * PLN + idx];
        const LimbConst &lc = lt.c[limb];
        const uint64_t t = (uint64_t)(acc + ((int64_t)lc.q << 30));          // in [0, q 2^31)
        // t 2^-32 mod q by one Montgomery reduction, then times 2^64 mod q
        const uint32_t m = (uint32_t)t * lc.qinv_neg;
        const uint32_t y = scsub((uint32_t)(((uint64_t)m * lc.q + t) >> 32), lc.q);
        out[(size_t)o * PLN + idx] = smont(y, lc.r64, lc.q, lc.qinv_neg);
    }
}

// Two weight sets over the same inputs (the A and B Walsh components of the
// SIMD convolution): every input word is read once for both sums.
__device__ __forceinline__ uint32_t lazy_result(int64_t acc, const LimbConst &lc) {
    const uint64_t t = (uint64_t)(acc + ((int64_t)lc.q << 30));          // in [0, q 2^31)
    const uint32_t m = (uint32_t)t * lc.qinv_neg;
    const uint32_t y = scsub((uint32_t)(((uint64_t)m * lc.q + t) >> 32), lc.q);   // t 2^-32 mod q
    return smont(y, lc.r64, lc.q, lc.qinv_neg);                                    // t mod q
}

// OPT outputs per thread: each input word read from L2 once per OPT outputs
template <uint32_t OPT>
__global__ void __launch_bounds__(STH) cmult_acc2_kernel(const uint32_t *__restrict__ in,
                                                         const int32_t *__restrict__ WA,
                                                         const int32_t *__restrict__ WB, uint32_t *__restrict__ outA,
                                                         uint32_t *__restrict__ outB, uint32_t R, uint32_t O,
                                                         uint32_t logN, uint32_t L, LimbTable lt) {
    const size_t PLN = (size_t)2 * L << logN;
    const uint32_t og = (O + OPT - 1) / OPT;
    const uint32_t chunks = (uint32_t)(((size_t)og * 2 * L) << (logN - 8));   // < 2^31 (checked on the host)
    for (uint32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const uint32_t op = c >> (logN - 8);
        const uint32_t o0 = (op / (2 * L)) * OPT, limb = op % L;
        const size_t idx = ((size_t)(op % (2 * L)) << logN) + ((c & ((1u << (logN - 8)) - 1)) << 8) + threadIdx.x;
        const uint32_t no = min(OPT, O - o0);
        int64_t a[OPT], b[OPT];
        // the weight rows are the same for every lane: scalar pointers, so
        // that the weights come through scalar loads (rows past O repeat the
        // last and are not stored)
        const int32_t *wa[OPT], *wb[OPT];
#pragma unroll
        for (uint32_t u = 0; u < OPT; u++) {
            const uint32_t o = __builtin_amdgcn_readfirstlane(min(o0 + u, O - 1));
            wa[u] = WA + (size_t)o * R, wb[u] = WB + (size_t)o * R;
            a[u] = 0, b[u] = 0;
        }
#pragma unroll 4
        for (uint32_t r = 0; r < R; r++) {
            const int32_t x = (int32_t)in[(size_t)r * PLN + idx];   // < 2^31: one v_mad_i64_i32 per product
#pragma unroll
            for (uint32_t u = 0; u < OPT; u++) {
                a[u] += (int64_t)wa[u][r] * (int64_t)x;
                b[u] += (int64_t)wb[u][r] * (int64_t)x;
            }
        }
        const LimbConst &lc = lt.c[limb];
#pragma unroll
        for (uint32_t u = 0; u < OPT; u++) {
            if (u >= no) break;
            outA[(size_t)(o0 + u) * PLN + idx] = lazy_result(a[u], lc);
            outB[(size_t)(o0 + u) * PLN + idx] = lazy_result(b[u], lc);
        }
    }
}

// The [k, -k] plaintext kh (X^(N/4) + X^(3N/4)) at the NTT's evaluation point
// psi^e (e = 2 brv(s) + 1 odd) is kh (w^e + w^(3e)) with w = psi^(N/4) of order
// 8, so it takes four values per limb, chosen by e mod 8: in the NTT domain
// PMult by it is a product by one of four constants.
struct PmConst {
    uint32_t c[HYENA_MAX_LIMBS][4];   // kh (w^e + w^3e) 2^32 mod q_i for e = 1, 3, 5, 7
};

// Z = A + B . NTT(w_pm) (NTT domain), ciphertext arrays [..][L][N]
__global__ void __launch_bounds__(STH) pm_madd_ntt_kernel(const uint32_t *A, const uint32_t *B, uint32_t *Z,
                                                          uint32_t polys, uint32_t logN, uint32_t L, LimbTable lt,
                                                          PmConst pc) {
    const uint32_t chunks = polys << (logN - 8);   // < 2^31 (checked on the host)
    for (uint32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const uint32_t limb = (c >> (logN - 8)) % L;
        const LimbConst &lc = lt.c[limb];
        const uint32_t s = ((c & ((1u << (logN - 8)) - 1)) << 8) + threadIdx.x;
        const uint32_t e = 2 * brev(s, logN) + 1;
        const size_t i = ((size_t)c << 8) + threadIdx.x;
        Z[i] = scsub(A[i] + smont(B[i], pc.c[limb][(e >> 1) & 3], lc.q, lc.qinv_neg), lc.q);
    }
}

// HAdd: out = a + b mod q_i for ciphertext arrays [..][L][N] of `polys` limb-polynomials
__global__ void __launch_bounds__(STH) hadd_kernel(const uint32_t *a, const uint32_t *b, uint32_t *out,
                                                   uint32_t polys, uint32_t logN, uint32_t L, LimbTable lt) {
    const uint32_t chunks = polys << (logN - 8);   // < 2^31 (checked on the host)
    for (uint32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const uint32_t q = lt.c[(c >> (logN - 8)) % L].q;
        const size_t i = ((size_t)c << 8) + threadIdx.x;
        out[i] = scsub(a[i] + b[i], q);
    }
}

unsigned sgrid(size_t chunks) { return (unsigned)std::min<size_t>(chunks, 8192); }

bool soverlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return na && nb && a0 < b0 + nb && b0 < a0 + na;
}

int slaunched(const char *who) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string(who) + ": " + hipGetErrorString(e));
    return HYENA_OK;
}

int device_ctx(const hyena_ctx *c, const char *who) {
    if (!c->d_fw) return set_error(HYENA_EINVAL, std::string(who) + ": context was created host-only");
    return HYENA_OK;
}

bool is_prime_small(uint32_t x) {
    if (x < 2) return false;
    for (uint64_t f = 2; f * f <= x; f++)
        if (x % f == 0) return false;
    return true;
}

}  // namespace

extern "C" int hyena_simd_params(uint32_t n, uint32_t p, uint32_t kmax, uint32_t *h_out, uint32_t *k_out,
                                 uint32_t *kh_out) {
    if (n < 8 || (n & (n - 1)) || n > (1u << 20)) return set_error(HYENA_EINVAL, "hyena_simd_params: n must be a power of two >= 8");
    if (p >= (1u << 31) || (p - 1) % (2 * n) != 0 || !is_prime_small(p))
        return set_error(HYENA_EINVAL, "hyena_simd_params: p must be a prime below 2^31 with p = 1 mod 2n");
    if (kmax < 1) return set_error(HYENA_EINVAL, "hyena_simd_params: kmax must be at least 1");
    // zeta: the least primitive 2n-th root of unity; w = zeta^(n/4) has order 8 and
    // the [1, -1] plaintext is h (X^(n/4) + X^(3n/4)) with h (w + w^3) = 1
    uint32_t z = 2;
    while (h_powmod(z, n, p) != p - 1) z++;
    const uint32_t w = h_powmod(z, n / 4, p);
    const uint32_t s = (uint32_t)(((uint64_t)w + h_powmod(w, 3, p)) % p);
    const uint32_t h = h_powmod(s, p - 2, p);
    uint32_t bk = 1, bkh = h;
    for (uint32_t k = 2; k <= kmax; k++) {
        const uint32_t v = (uint32_t)((uint64_t)k * h % p);
        if (v < bkh) bk = k, bkh = v;
    }
    if (h_out) *h_out = h;
    if (k_out) *k_out = bk;
    if (kh_out) *kh_out = bkh;
    return HYENA_OK;
}

extern "C" int hyena_simd_encode(const hyena_ctx *c, const uint32_t *d_slots, size_t P, uint32_t *d_coef,
                                 hyena_stream_t stream) {
    static const char *who = "hyena_simd_encode";
    if (!c || (P && (!d_slots || !d_coef))) return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = device_ctx(c, who)) return rc;
    if (c->L != 1) return set_error(HYENA_EINVAL, std::string(who) + ": the context must hold the plaintext prime alone");
    if (P == 0) return HYENA_OK;
    if (P > 0x7fffffffull) return set_error(HYENA_EINVAL, std::string(who) + ": too many polynomials");
    const size_t bytes = P * c->N * 4;
    if (soverlap(d_slots, bytes, d_coef, bytes)) return set_error(HYENA_EINVAL, std::string(who) + ": d_coef overlaps d_slots");
    const hipStream_t s = (hipStream_t)stream;
    if ((((uintptr_t)d_slots | (uintptr_t)d_coef) & 15u) == 0)
        hipLaunchKernelGGL(slots_to_ntt_lds_kernel, dim3((unsigned)P), dim3(STH), c->N * 4, s, d_slots, d_coef, P,
                           c->logN, c->q[0]);
    else
        hipLaunchKernelGGL(slots_to_ntt_kernel, dim3(sgrid(P << (c->logN - 8))), dim3(STH), 0, s, d_slots, d_coef, P,
                           c->logN, c->q[0]);
    if (int rc = slaunched(who)) return rc;
    return launch_ntt(c, d_coef, P, true, s);
}

extern "C" int hyena_simd_decode(const hyena_ctx *c, uint32_t *d_coef, size_t P, uint32_t *d_slots,
                                 hyena_stream_t stream) {
    static const char *who = "hyena_simd_decode";
    if (!c || (P && (!d_slots || !d_coef))) return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = device_ctx(c, who)) return rc;
    if (c->L != 1) return set_error(HYENA_EINVAL, std::string(who) + ": the context must hold the plaintext prime alone");
    if (P == 0) return HYENA_OK;
    if (P > 0x7fffffffull) return set_error(HYENA_EINVAL, std::string(who) + ": too many polynomials");
    const size_t bytes = P * c->N * 4;
    if (soverlap(d_slots, bytes, d_coef, bytes)) return set_error(HYENA_EINVAL, std::string(who) + ": d_slots overlaps d_coef");
    const hipStream_t s = (hipStream_t)stream;
    if (int rc = launch_ntt(c, d_coef, P, false, s)) return rc;
    hipLaunchKernelGGL(ntt_to_slots_kernel, dim3(sgrid(P << (c->logN - 8))), dim3(STH), 0, s, d_coef, d_slots, P,
                       c->logN);
    return slaunched(who);
}

extern "C" int hyena_automorphism(const hyena_ctx *c, const uint32_t *d_in, size_t P, uint32_t g, uint32_t *d_out,
                                  hyena_stream_t stream) {
    static const char *who = "hyena_automorphism";
    if (!c || (P && (!d_in || !d_out))) return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = device_ctx(c, who)) return rc;
    if (!(g & 1)) return set_error(HYENA_EINVAL, std::string(who) + ": g must be odd");
    if (P == 0) return HYENA_OK;
    const size_t polys = P * c->L;
    if (polys > (0x7fffffffull >> (c->logN - 8))) return set_error(HYENA_EINVAL, std::string(who) + ": too many polynomials");
    const size_t bytes = polys * c->N * 4;
    if (soverlap(d_in, bytes, d_out, bytes)) return set_error(HYENA_EINVAL, std::string(who) + ": d_out overlaps d_in");
    // g^-1 mod 2N (g odd): Newton's iteration x <- x (2 - g x) doubles the correct low bits
    const uint32_t mask = 2 * c->N - 1;
    uint32_t x = g;   // correct to 3 bits (g g = 1 mod 8)
    for (int it = 0; it < 5; it++) x *= 2u - g * x;
    const uint32_t ginv = x & mask;
    if ((((uintptr_t)d_in | (uintptr_t)d_out) & 15u) == 0) {
        // whole limb-polynomials through LDS, one block each (the hardware
        // overlaps one block's loads with another's gathers and stores:
        // 5.7 against 5.2-5.4 TB/s with a grid of 4096 looping blocks)
        hipLaunchKernelGGL(automorphism_lds_kernel, dim3((unsigned)polys), dim3(STH),
                           c->N * 4, (hipStream_t)stream, d_in, d_out, polys, c->logN, c->L, ginv, c->lt);
    } else {
        hipLaunchKernelGGL(automorphism_kernel, dim3(sgrid(polys << (c->logN - 8))), dim3(STH), 0,
                           (hipStream_t)stream, d_in, d_out, polys, c->logN, c->L, ginv, c->lt);
    }
    return slaunched(who);
}

extern "C" int hyena_pmult_sparse(const hyena_ctx *c, const uint32_t *d_in, size_t P, uint32_t n_terms,
                                  const uint32_t *exps, const uint32_t *coefs, uint32_t *d_out, hyena_stream_t stream) {
    static const char *who = "hyena_pmult_sparse";
    if (!c || (P && (!d_in || !d_out)) || (n_terms && (!exps || !coefs)))
        return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = device_ctx(c, who)) return rc;
    if (n_terms > MAX_TERMS) return set_error(HYENA_EINVAL, std::string(who) + ": more than 16 monomials");
    if (P == 0) return HYENA_OK;
    const size_t polys = P * c->L;
    if (polys > (0x7fffffffull >> (c->logN - 8))) return set_error(HYENA_EINVAL, std::string(who) + ": too many polynomials");
    const size_t bytes = polys * c->N * 4;
    if (soverlap(d_in, bytes, d_out, bytes)) return set_error(HYENA_EINVAL, std::string(who) + ": d_out overlaps d_in");
    Sparse sp{};
    sp.n = n_terms;
    for (uint32_t t = 0; t < n_terms; t++) {
        if (exps[t] >= 2 * c->N) return set_error(HYENA_EINVAL, std::string(who) + ": exponent not below 2N");
        sp.e[t] = exps[t];
        for (uint32_t i = 0; i < c->L; i++) sp.cm[i][t] = to_montgomery(coefs[t] % c->q[i], c->q[i]);
    }
    if ((((uintptr_t)d_in | (uintptr_t)d_out) & 15u) == 0) {
        hipLaunchKernelGGL(pmult_sparse_lds_kernel, dim3((unsigned)polys), dim3(STH),
                           c->N * 4, (hipStream_t)stream, d_in, d_out, polys, c->logN, c->L, c->lt, sp);
    } else {
        hipLaunchKernelGGL(pmult_sparse_kernel, dim3(sgrid(polys << (c->logN - 8))), dim3(STH), 0,
                           (hipStream_t)stream, d_in, d_out, polys, c->logN, c->L, c->lt, sp);
    }
    return slaunched(who);
}

extern "C" int hyena_ksk_prepare(const hyena_ctx *c, uint32_t *d_ksk, size_t n_polys, hyena_stream_t stream) {
    static const char *who = "hyena_ksk_prepare";
    if (!c || (n_polys && !d_ksk)) return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = device_ctx(c, who)) return rc;
    if (n_polys == 0) return HYENA_OK;
    const hipStream_t s = (hipStream_t)stream;
    if (int rc = launch_ntt(c, d_ksk, n_polys, false, s)) return rc;
    const size_t polys = n_polys * c->L;
    hipLaunchKernelGGL(scale_montgomery_kernel, dim3(sgrid(polys << (c->logN - 8))), dim3(STH), 0, s, d_ksk, polys,
                       c->logN, c->L, c->lt);
    return slaunched(who);
}

// intt_out = false leaves the rotated ciphertexts in the NTT domain
static int hrot_impl(const hyena_ctx *c, const uint32_t *d_ct, size_t n_ct, uint32_t n_rot, const uint32_t *gs,
                     uint32_t log2_base, const uint32_t *d_ksk, uint32_t *d_work, uint32_t *d_out,
                     hyena_stream_t stream, bool intt_out) {
    static const char *who = "hyena_hrot_hoisted";
    if (!c || (n_ct && n_rot && (!d_ct || !gs || !d_ksk || !d_work || !d_out)))
        return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = device_ctx(c, who)) return rc;
    if (n_rot > MAX_ROT) return set_error(HYENA_EINVAL, std::string(who) + ": more than 64 rotations");
    if (log2_base < 1 || log2_base > 29) return set_error(HYENA_EINVAL, std::string(who) + ": log2_base must be in [1, 29]");
    if (n_ct == 0 || n_rot == 0) return HYENA_OK;
    RotArgs ra{};
    ra.n_rot = n_rot;
    ra.b = log2_base;
    ra.D = (31 + log2_base - 1) / log2_base;
    for (uint32_t r = 0; r < n_rot; r++) {
        if (!(gs[r] & 1)) return set_error(HYENA_EINVAL, std::string(who) + ": every g must be odd");
        ra.g[r] = gs[r] & (2 * c->N - 1);
    }
    const size_t LN = (size_t)c->L * c->N, T = (size_t)c->L * ra.D + 1;
    if (n_ct * T > 0x7fffffffull / c->L || n_ct * n_rot * 2 > 0x7fffffffull / c->L ||
        ((n_ct * n_rot * c->L) << (c->logN - 8)) > 0x7fffffffull)
        return set_error(HYENA_EINVAL, std::string(who) + ": too many ciphertexts");
    const size_t ct_b = n_ct * 2 * LN * 4, work_b = n_ct * T * LN * 4, out_b = n_ct * n_rot * 2 * LN * 4,
                 ksk_b = (size_t)n_rot * (T - 1) * 2 * LN * 4;
    if (soverlap(d_work, work_b, d_ct, ct_b) || soverlap(d_work, work_b, d_out, out_b) ||
        soverlap(d_work, work_b, d_ksk, ksk_b) || soverlap(d_out, out_b, d_ct, ct_b) ||
        soverlap(d_out, out_b, d_ksk, ksk_b))
        return set_error(HYENA_EINVAL, std::string(who) + ": d_work or d_out overlaps another array");
    const hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(decompose_kernel, dim3(sgrid((n_ct * c->L) << (c->logN - 8))), dim3(STH), 0, s, d_ct, d_work,
                       n_ct, c->logN, c->L, ra);
    if (int rc = slaunched(who)) return rc;
    if (int rc = launch_ntt(c, d_work, n_ct * T, false, s)) return rc;
    const uint32_t TD = c->L * ra.D;
    const size_t kchunks = (((n_ct + KS_M - 1) / KS_M) * n_rot * c->L) << (c->logN - 8);
    const size_t rchunks = (((n_ct + KS_R - 1) / KS_R) * c->L) << (c->logN - 8);
    RotInv ri{};
    for (uint32_t r = 0; r < n_rot; r++) {
        // g^-1 mod 2N for odd g: Newton's iteration x <- x (2 - g x) doubles the correct low bits
        uint32_t x = ra.g[r];
        for (int it = 0; it < 5; it++) x *= 2u - ra.g[r] * x;
        ri.ginv[r] = x & (2 * c->N - 1);
    }
    // with several rotations and few enough digit terms to hold KS_R
    // ciphertexts' digits in registers, the rotation-looping kernel
#define HY_KR(td)                                                                                                  \
    case td:                                                                                                       \
        hipLaunchKernelGGL(keyswitch_rot_kernel<td>, dim3(sgrid(rchunks)), dim3(STH), 0, s, d_work, d_ksk, d_out, \
                           (uint32_t)n_ct, c->logN, c->L, c->lt, ra, ri);                                          \
        looped = true;                                                                                             \
        break;
#define HY_KS(td)                                                                                               \
    case td:                                                                                                    \
        hipLaunchKernelGGL(keyswitch_keys_kernel<td>, dim3(sgrid(kchunks)), dim3(STH), 0, s, d_work, d_ksk, d_out, \
                           (uint32_t)n_ct, c->logN, c->L, c->lt, ra);                                           \
        break;
    bool looped = false;
    // (only when it still gives every CU several blocks: it has n_rot times
    // fewer than the per-rotation kernel)
    if (n_rot >= 2 && rchunks >= 2048) switch (TD) {
            HY_KR(1) HY_KR(2) HY_KR(3) HY_KR(4) HY_KR(6) HY_KR(8)
            default: break;
        }
    if (!looped) switch (TD) {
        HY_KS(1) HY_KS(2) HY_KS(3) HY_KS(4) HY_KS(6) HY_KS(8) HY_KS(9) HY_KS(12)
        default:
            hipLaunchKernelGGL(keyswitch_kernel, dim3(sgrid(((n_ct * n_rot) * c->L) << (c->logN - 8))), dim3(STH), 0,
                               s, d_work, d_ksk, d_out, n_ct, c->logN, c->L, c->lt, ra);
    }
#undef HY_KS
#undef HY_KR
    if (int rc = slaunched(who)) return rc;
    return intt_out ? launch_ntt(c, d_out, n_ct * n_rot * 2, true, s) : HYENA_OK;
}

extern "C" int hyena_hrot_hoisted(const hyena_ctx *c, const uint32_t *d_ct, size_t n_ct, uint32_t n_rot,
                                  const uint32_t *gs, uint32_t log2_base, const uint32_t *d_ksk, uint32_t *d_work,
                                  uint32_t *d_out, hyena_stream_t stream) {
    return hrot_impl(c, d_ct, n_ct, n_rot, gs, log2_base, d_ksk, d_work, d_out, stream, true);
}

// constants of the [k, -k] plaintext in the NTT domain
static PmConst pm_constants(const hyena_ctx *c, uint32_t kh) {
    PmConst pc{};
    for (uint32_t i = 0; i < c->L; i++) {
        const uint32_t q = c->q[i], w = h_powmod(c->psi[i], c->N / 4, q);
        for (uint32_t j = 0; j < 4; j++) {
            const uint32_t e = 2 * j + 1;
            const uint64_t v = ((uint64_t)h_powmod(w, e, q) + h_powmod(w, 3 * e, q)) % q;
            pc.c[i][j] = to_montgomery(h_mulmod((uint32_t)v, kh % q, q), q);
        }
    }
    return pc;
}

extern "C" int hyena_cmult_accumulate(const hyena_ctx *c, const uint32_t *d_in, uint32_t R, const int32_t *d_w,
                                      uint32_t O, uint32_t *d_out, hyena_stream_t stream) {
    static const char *who = "hyena_cmult_accumulate";
    if (!c || (O && !d_out) || (R && O && (!d_in || !d_w)))   // with R = 0 the outputs are still written (zeros)
        return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = device_ctx(c, who)) return rc;
    if (R > 4096) return set_error(HYENA_EINVAL, std::string(who) + ": more than 4096 inputs");
    for (uint32_t q : c->q)   // the bias q 2^30 must cover sums up to 2^59
        if (q <= (1u << 29)) return set_error(HYENA_EINVAL, std::string(who) + ": primes must exceed 2^29");
    if (O == 0) return HYENA_OK;
    if ((size_t)O * 2 * c->L > (0x7fffffffull >> (c->logN - 8)))
        return set_error(HYENA_EINVAL, std::string(who) + ": too many outputs");
    const size_t PLNb = (size_t)2 * c->L * c->N * 4;
    if (soverlap(d_out, O * PLNb, d_in, R * PLNb) || soverlap(d_out, O * PLNb, d_w, (size_t)O * R * 4))
        return set_error(HYENA_EINVAL, std::string(who) + ": d_out overlaps an input");
    hipLaunchKernelGGL(cmult_acc_kernel, dim3(sgrid(((size_t)O * 2 * c->L) << (c->logN - 8))), dim3(STH), 0,
                       (hipStream_t)stream, d_in, d_w, d_out, R, O, c->logN, c->L, c->lt);
    return slaunched(who);
}

// A = sum wa in, B = sum wb in over R ciphertexts (the checks of hyena_cmult_accumulate)
static int cmult_accumulate2(const hyena_ctx *c, const uint32_t *d_in, uint32_t R, const int32_t *d_wa,
                             const int32_t *d_wb, uint32_t O, uint32_t *A, uint32_t *B, hipStream_t s) {
    static const char *who = "hyena_simd_conv";
    if (R > 4096) return set_error(HYENA_EINVAL, std::string(who) + ": more than 4096 rotations");
    for (uint32_t q : c->q)
        if (q <= (1u << 29)) return set_error(HYENA_EINVAL, std::string(who) + ": primes must exceed 2^29");
    if ((size_t)O * 2 * c->L > (0x7fffffffull >> (c->logN - 8)))
        return set_error(HYENA_EINVAL, std::string(who) + ": too many outputs");
    // the most outputs per thread (4, 2, 1) that still leave two blocks per CU: fewer
    // outputs per thread cost L2 re-reads of the inputs, fewer blocks cost occupancy
    // (64 outputs at N = 2048, L = 3: 4 per thread, 768 blocks, 0.168 ms against 0.178
    // at 2; 8 per thread, 384 blocks, 0.20 ms)
    constexpr size_t kMinBlocks = 512;
    auto blocks = [&](size_t opt) { return ((O + opt - 1) / opt * 2 * c->L) << (c->logN - 8); };
#define HY_CMA(opt)                                                                                              \
    hipLaunchKernelGGL(cmult_acc2_kernel<opt>, dim3(sgrid(blocks(opt))), dim3(STH), 0, s, d_in, d_wa, d_wb, A, B, \
                       R, O, c->logN, c->L, c->lt)
    if (blocks(4) >= kMinBlocks) HY_CMA(4);
    else if (blocks(2) >= kMinBlocks) HY_CMA(2);
    else HY_CMA(1);
#undef HY_CMA
    return slaunched(who);
}

extern "C" int hyena_simd_conv_weights(uint32_t Ci, uint32_t Co, const int8_t *f, uint32_t k, int32_t *wa,
                                       int32_t *wb) {
    if (!f || !wa || !wb) return set_error(HYENA_EINVAL, "hyena_simd_conv_weights: NULL argument");
    if (Ci == 0 || Ci % 2 || Co == 0) return set_error(HYENA_EINVAL, "hyena_simd_conv_weights: Ci must be even and positive, Co positive");
    if (k > 255) return set_error(HYENA_EINVAL, "hyena_simd_conv_weights: k above 255 (the scalars must stay within 2^16)");
    const uint32_t G = Ci / 2;
    for (uint32_t o = 0; o < Co; o++)
        for (uint32_t g = 0; g < G; g++)
            for (uint32_t r = 0; r < 9; r++) {
                const int32_t f0 = f[((size_t)o * Ci + 2 * g) * 9 + r], f1 = f[((size_t)o * Ci + 2 * g + 1) * 9 + r];
                wa[((size_t)o * G + g) * 9 + r] = (int32_t)k * (f0 + f1);
                wb[((size_t)o * G + g) * 9 + r] = f0 - f1;
            }
    return HYENA_OK;
}

extern "C" size_t hyena_simd_conv_workspace(const hyena_ctx *c, uint32_t n_in, uint32_t Co, uint32_t log2_base) {
    if (!c || log2_base < 1 || log2_base > 29) return 0;
    const size_t LN = (size_t)c->L * c->N, D = (31 + log2_base - 1) / log2_base;
    const size_t hw = (size_t)std::max(n_in, Co) * (c->L * D + 1) * LN;
    return (size_t)n_in * 9 * 2 * LN + hw + 3 * (size_t)Co * 2 * LN;
}

extern "C" int hyena_simd_conv_cn2(const hyena_ctx *c, const uint32_t *d_ct, uint32_t n_in, uint32_t frame_w,
                                   const int32_t *d_wa, const int32_t *d_wb, uint32_t Co, uint32_t kh,
                                   uint32_t log2_base, const uint32_t *d_rot_ksk, const uint32_t *d_swap_ksk,
                                   uint32_t *d_work, size_t work_words, uint32_t *d_out, hyena_stream_t stream) {
    static const char *who = "hyena_simd_conv_cn2";
    if (!c || !d_ct || !d_wa || !d_wb || !d_rot_ksk || !d_swap_ksk || !d_work || !d_out)
        return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = device_ctx(c, who)) return rc;
    if (n_in == 0 || Co == 0) return set_error(HYENA_EINVAL, std::string(who) + ": no inputs or outputs");
    if (n_in * 9 > 4096) return set_error(HYENA_EINVAL, std::string(who) + ": more than 455 input ciphertexts");
    if (frame_w == 0 || frame_w >= c->N / 2) return set_error(HYENA_EINVAL, std::string(who) + ": frame width must be in [1, N/2)");
    const size_t need = hyena_simd_conv_workspace(c, n_in, Co, log2_base);
    if (need == 0) return set_error(HYENA_EINVAL, std::string(who) + ": log2_base must be in [1, 29]");
    if (work_words < need) return set_error(HYENA_EINVAL, std::string(who) + ": workspace too small");
    if ((size_t)Co * 2 * c->L > (0x7fffffffull >> (c->logN - 8)))
        return set_error(HYENA_EINVAL, std::string(who) + ": too many outputs");
    const size_t LN = (size_t)c->L * c->N, CT = 2 * LN;
    if (soverlap(d_out, Co * CT * 4, d_work, work_words * 4) || soverlap(d_out, Co * CT * 4, d_ct, n_in * CT * 4))
        return set_error(HYENA_EINVAL, std::string(who) + ": d_out overlaps an input or the workspace");
    // the nine rotations: slot s + (di - 1) frame_w + (dj - 1) moves to slot s, X -> X^(3^off)
    uint32_t gs[9];
    const uint32_t half = c->N / 2, mask = 2 * c->N - 1;
    for (uint32_t di = 0; di < 3; di++)
        for (uint32_t dj = 0; dj < 3; dj++) {
            const int64_t off = ((int64_t)di - 1) * frame_w + ((int64_t)dj - 1);
            const uint32_t e = (uint32_t)(((off % half) + half) % half);
            uint32_t g = 1, b = 3;
            for (uint32_t x = e; x; x >>= 1) {
                if (x & 1) g = (g * b) & mask;
                b = (b * b) & mask;
            }
            gs[di * 3 + dj] = g;
        }
    uint32_t *rots = d_work;                                   // [n_in][9][2][L][N]
    uint32_t *hwork = rots + (size_t)n_in * 9 * CT;            // HRot workspace
    const size_t D = (31 + log2_base - 1) / log2_base;
    uint32_t *A = hwork + (size_t)std::max(n_in, Co) * (c->L * D + 1) * LN;
    uint32_t *B = A + Co * CT, *PB = B + Co * CT;
    const hipStream_t s = (hipStream_t)stream;
    const uint32_t polys = Co * 2 * c->L;
    // 1. hoisted HRot of every input by the nine offsets, left in the NTT domain
    if (int rc = hrot_impl(c, d_ct, n_in, 9, gs, log2_base, d_rot_ksk, hwork, rots, stream, false)) return rc;
    // 2. CMult + HAdd of the Walsh components over every rotation (linear: either domain)
    if (int rc = cmult_accumulate2(c, rots, n_in * 9, d_wa, d_wb, Co, A, B, s)) return rc;
    // 3. Z = A + PMult(B, [k, -k]): a product by one of four constants per slot; then Z's inverse NTT
    hipLaunchKernelGGL(pm_madd_ntt_kernel, dim3(sgrid((size_t)polys << (c->logN - 8))), dim3(STH), 0, s, A, B, B,
                       polys, c->logN, c->L, c->lt, pm_constants(c, kh));
    if (int rc = slaunched(who)) return rc;
    if (int rc = launch_ntt(c, B, 2 * (size_t)Co, true, s)) return rc;
    // 4. row-swap HRot (into PB's buffer) and HAdd
    const uint32_t swap = 2 * c->N - 1;
    if (int rc = hyena_hrot_hoisted(c, B, Co, 1, &swap, log2_base, d_swap_ksk, hwork, PB, stream)) return rc;
    hipLaunchKernelGGL(hadd_kernel, dim3(sgrid((size_t)polys << (c->logN - 8))), dim3(STH), 0, s, B, PB, d_out, polys,
                       c->logN, c->L, c->lt);
    return slaunched(who);
}

extern "C" int hyena_simd_conv_weights_packed(uint32_t Ci, uint32_t Co, const int8_t *f, uint32_t k, int32_t *wa,
                                              int32_t *wb) {
    if (!f || !wa || !wb) return set_error(HYENA_EINVAL, "hyena_simd_conv_weights_packed: NULL argument");
    if (Ci == 0 || Ci % 2 || Co == 0 || Co % 2)
        return set_error(HYENA_EINVAL, "hyena_simd_conv_weights_packed: Ci and Co must be even and positive");
    if (k > 255) return set_error(HYENA_EINVAL, "hyena_simd_conv_weights_packed: k above 255 (the scalars must stay within 2^16)");
    const uint32_t G = Ci / 2, R = 2 * G * 9;
    auto tap = [&](uint32_t o, uint32_t c, uint32_t r) { return (int32_t)f[((size_t)o * Ci + c) * 9 + r]; };
    for (uint32_t o2 = 0; o2 < Co / 2; o2++)
        for (uint32_t h = 0; h < 2; h++)          // h = 0: the input, h = 1: its row swap
            for (uint32_t g = 0; g < G; g++)
                for (uint32_t r = 0; r < 9; r++) {
                    const uint32_t o = 2 * o2;
                    const int32_t a = h ? tap(o, 2 * g + 1, r) : tap(o, 2 * g, r);
                    const int32_t b = h ? tap(o + 1, 2 * g, r) : tap(o + 1, 2 * g + 1, r);
                    const size_t i = (size_t)o2 * R + ((size_t)h * G + g) * 9 + r;
                    wa[i] = (int32_t)k * (a + b);
                    wb[i] = a - b;
                }
    return HYENA_OK;
}

extern "C" size_t hyena_simd_conv_packed_workspace(const hyena_ctx *c, uint32_t n_in, uint32_t Co,
                                                   uint32_t log2_base) {
    if (!c || log2_base < 1 || log2_base > 29) return 0;
    const size_t LN = (size_t)c->L * c->N, CT = 2 * LN, D = (31 + log2_base - 1) / log2_base;
    return 2 * (size_t)n_in * CT + 2 * (size_t)n_in * 9 * CT + 2 * (size_t)n_in * (c->L * D + 1) * LN +
           2 * (size_t)(Co / 2) * CT;
}

extern "C" int hyena_simd_conv_packed(const hyena_ctx *c, const uint32_t *d_ct, uint32_t n_in, uint32_t frame_w,
                                      const int32_t *d_wa, const int32_t *d_wb, uint32_t Co, uint32_t kh,
                                      uint32_t log2_base, const uint32_t *d_rot_ksk, const uint32_t *d_swap_ksk,
                                      uint32_t *d_work, size_t work_words, uint32_t *d_out, hyena_stream_t stream) {
    static const char *who = "hyena_simd_conv_packed";
    if (!c || !d_ct || !d_wa || !d_wb || !d_rot_ksk || !d_swap_ksk || !d_work || !d_out)
        return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = device_ctx(c, who)) return rc;
    if (n_in == 0 || Co == 0 || Co % 2) return set_error(HYENA_EINVAL, std::string(who) + ": need inputs and an even Co");
    if (2 * n_in * 9 > 4096) return set_error(HYENA_EINVAL, std::string(who) + ": more than 227 input ciphertexts");
    if (frame_w == 0 || frame_w >= c->N / 2) return set_error(HYENA_EINVAL, std::string(who) + ": frame width must be in [1, N/2)");
    const size_t need = hyena_simd_conv_packed_workspace(c, n_in, Co, log2_base);
    if (need == 0) return set_error(HYENA_EINVAL, std::string(who) + ": log2_base must be in [1, 29]");
    if (work_words < need) return set_error(HYENA_EINVAL, std::string(who) + ": workspace too small");
    const uint32_t P2 = Co / 2;
    if ((size_t)P2 * 2 * c->L > (0x7fffffffull >> (c->logN - 8)))
        return set_error(HYENA_EINVAL, std::string(who) + ": too many outputs");
    const size_t LN = (size_t)c->L * c->N, CT = 2 * LN;
    if (soverlap(d_out, P2 * CT * 4, d_work, work_words * 4) || soverlap(d_out, P2 * CT * 4, d_ct, n_in * CT * 4) ||
        soverlap(d_work, work_words * 4, d_ct, n_in * CT * 4))
        return set_error(HYENA_EINVAL, std::string(who) + ": d_out, d_work and d_ct must not overlap");
    uint32_t gs[9];
    const uint32_t half = c->N / 2, mask = 2 * c->N - 1;
    for (uint32_t di = 0; di < 3; di++)
        for (uint32_t dj = 0; dj < 3; dj++) {
            const int64_t off = ((int64_t)di - 1) * frame_w + ((int64_t)dj - 1);
            const uint32_t e = (uint32_t)(((off % half) + half) % half);
            uint32_t g = 1, b = 3;
            for (uint32_t x = e; x; x >>= 1) {
                if (x & 1) g = (g * b) & mask;
                b = (b * b) & mask;
            }
            gs[di * 3 + dj] = g;
        }
    const size_t D = (31 + log2_base - 1) / log2_base;
    uint32_t *X = d_work;                                      // [2 n_in] ciphertexts: inputs, then their row swaps
    uint32_t *rots = X + 2 * (size_t)n_in * CT;                // [2 n_in][9]
    uint32_t *hwork = rots + 2 * (size_t)n_in * 9 * CT;
    uint32_t *A = hwork + 2 * (size_t)n_in * (c->L * D + 1) * LN;
    uint32_t *B = A + P2 * CT;
    const hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(X, d_ct, (size_t)n_in * CT * 4, hipMemcpyDeviceToDevice, s));
    // 1. the row swap of every input
    const uint32_t swap = 2 * c->N - 1;
    if (int rc = hyena_hrot_hoisted(c, d_ct, n_in, 1, &swap, log2_base, d_swap_ksk, hwork, X + (size_t)n_in * CT, stream))
        return rc;
    // 2. hoisted HRot of the inputs and their swaps by the nine offsets, left in the NTT domain
    if (int rc = hrot_impl(c, X, 2 * (size_t)n_in, 9, gs, log2_base, d_rot_ksk, hwork, rots, stream, false)) return rc;
    // 3. CMult + HAdd of the Walsh components; out = A + PMult(B, [k, -k]) pointwise; its inverse NTT
    if (int rc = cmult_accumulate2(c, rots, 2 * n_in * 9, d_wa, d_wb, P2, A, B, s)) return rc;
    const uint32_t polys = P2 * 2 * c->L;
    hipLaunchKernelGGL(pm_madd_ntt_kernel, dim3(sgrid((size_t)polys << (c->logN - 8))), dim3(STH), 0, s, A, B, d_out,
                       polys, c->logN, c->L, c->lt, pm_constants(c, kh));
    if (int rc = slaunched(who)) return rc;
    return launch_ntt(c, d_out, 2 * (size_t)P2, true, s);
}

// Worst-case noise (infinity norm of v - Delta m over the coefficients) of the
// c_n = 2 convolution's output for base 2^b, as a double; fresh noise and key
// errors at most B = 32, q mod p < p:
//   key switching KS = L D N (2^b - 1) B per HRot; an automorphism negates
//   coefficients, which adds q mod p once; a CMult-and-HAdd by scalars w adds
//   (sum |w|) times the input noise plus (q mod p) per unit of sum |w| (the
//   carries of the plaintext sum past p); PMult by kh (X^(N/4) + X^(3N/4))
//   multiplies noise by 2 kh and adds 2 kh (q mod p); HAdd adds q mod p.
static double simd_conv_noise(const hyena_ctx *c, double p, double kh, double sa, double sb, uint32_t b, bool packed) {
    const double B = 32.0, D = (31 + b - 1) / b;
    const double KS = (double)c->L * D * c->N * (std::ldexp(1.0, (int)b) - 1.0) * B;
    const double in = packed ? B + KS + p : B;               // packed: half the inputs went through the row swap
    const double rot = in + KS + p;
    const double A = sa * rot + p * sa, Bn = sb * rot + p * sb;
    const double PB = 2 * kh * Bn + 2 * kh * p;
    const double Z = A + PB + p;
    return packed ? Z : Z + (Z + KS + p) + p;                 // unpacked: Z + HRot(Z, row swap)
}

extern "C" int hyena_simd_conv_choose_base(const hyena_ctx *c, uint32_t p, uint32_t kh, const int32_t *wa,
                                           const int32_t *wb, uint32_t O, uint32_t R, int packed,
                                           uint32_t *log2_base, double *margin_bits) {
    static const char *who = "hyena_simd_conv_choose_base";
    if (!c || !wa || !wb || !log2_base || !O || !R) return set_error(HYENA_EINVAL, std::string(who) + ": NULL or empty argument");
    if (p < 3) return set_error(HYENA_EINVAL, std::string(who) + ": p must be an odd prime");
    double sa = 0, sb = 0;   // the largest sum |w| over the outputs
    for (uint32_t o = 0; o < O; o++) {
        double a = 0, b = 0;
        for (uint32_t r = 0; r < R; r++) {
            a += std::fabs((double)wa[(size_t)o * R + r]);
            b += std::fabs((double)wb[(size_t)o * R + r]);
        }
        sa = std::max(sa, a);
        sb = std::max(sb, b);
    }
    double logq = 0;
    for (uint32_t q : c->q) logq += std::log2((double)q);
    // decryption is exact while |noise| < q / (2p) - p (the rounding also absorbs (q mod p) m / q < p)
    const double limit = std::exp2(logq - std::log2(2.0 * p)) - p;
    for (uint32_t b = 29; b >= 1; b--) {
        const double bound = simd_conv_noise(c, p, kh, sa, sb, b, packed != 0);
        if (bound < limit) {
            *log2_base = b;
            if (margin_bits) *margin_bits = std::log2(limit) - std::log2(bound);
            return HYENA_OK;
        }
    }
    return set_error(HYENA_ENOISE, std::string(who) + ": no base keeps the worst-case noise below q / 2p");
}
