// Evaluation-domain weight synthesis for gfx950.
//
// The cloud keeps each layer's kernels as small integers (the "Enabling Output
// Channel Packing" section) and needs them as evaluations at the NTT points.
// The kernel polynomial of output o and input group g is a sparse sum of
// monomials gw X^e (one per tap: e = O - c'*Bt - di*Wp - dj, gw the
// Walsh-combined integer weight), so its value at the point of NTT slot k,
// r = psi^(2 brv(k) + 1), is sum gw r^e: ci*k*k multiply-adds per word, with
// no coefficient array and no transform. hyena_encode_weights reaches the
// same words by scattering the taps and running the forward NTT.
//
// A block owns 256 slots of one limb for kSynthPolys consecutive polynomials
// (o, g). Each thread looks up r^O, r^-Bt, r^-Wp and r^-1 in the context's
// table of psi powers (r^E = psi^((2 brv(k) + 1) E mod 2N), and
// psi^(m + N) = -psi^m) and walks the tap powers with one Montgomery product
// per tap; the block
// stages the Walsh-combined weights of up to kSynthTaps taps of all its
// polynomials in LDS (read back as broadcasts); every tap adds power times
// weight into one 64-bit accumulator per polynomial. The weights are stored
// offset by 2^13 (|gw| <= 64 * 128, so gw + 2^13 is in [0, 2^14]), which makes
// each product one unsigned 32 x 32 -> 64 multiply-add; the offset's share,
// 2^13 times the sum of the powers (one accumulator for all polynomials), is
// taken off at the end. Fewer than 2^17 taps of powers below 2^31 keep the
// unsigned sums below 2^62 and the signed result below 2^61 <= q 2^32, so
// adding q 2^32 makes it a non-negative 64-bit value that one fold and one
// Montgomery reduction take.
#include <string>

#include "internal.h"

namespace {

constexpr uint32_t kSynthPolys = 32, kSynthTaps = 256;

struct SynthArgs {
    const int8_t *w;
    uint32_t *out;
    const uint32_t *fw;                // [L][N]: fw[i][j] = psi_i^brv(j) 2^32 mod q_i
    uint32_t N, L, logN, Co, Ci, k, ci, Bt, Wp, O, w_groups, c_n, kchunks;
    uint32_t wscale[HYENA_MAX_LIMBS];  // c_n^{-1} 2^64 mod q_i
    LimbTable lt;
};

// Montgomery reduction: y 2^-32 mod q for y < q 2^32
__device__ __forceinline__ uint32_t redc(uint64_t y, const LimbConst &lc) {
    const uint32_t m = (uint32_t)y * lc.qinv_neg;
    const uint32_t t = (uint32_t)(((uint64_t)m * lc.q + y) >> 32);
    return min(t, t - lc.q);
}

__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, const LimbConst &lc) {
    return redc((uint64_t)a * b, lc);  // a, b < q: a b < q 2^32
}

// psi^e 2^32 mod q for e < 2N, from the bit-reversed table of psi^j, j < N
__device__ __forceinline__ uint32_t psi_pow(const uint32_t *fw, uint32_t e, uint32_t N, uint32_t logN,
                                            const LimbConst &lc) {
    const uint32_t v = fw[__brev(e & (N - 1)) >> (32 - logN)];
    return (e & N) ? lc.q - v : v;  // v != 0: psi^j is a unit
}

__global__ void __launch_bounds__(256) synth_weights_kernel(SynthArgs a) {
    __shared__ __align__(16) uint32_t gs[kSynthTaps][kSynthPolys];  // gw + 2^13
    const uint32_t chunk = blockIdx.x % a.kchunks, pblk = blockIdx.x / a.kchunks, limb = blockIdx.y;
    const uint32_t slot = chunk * 256 + threadIdx.x;
    const LimbConst lc = a.lt.c[limb];
    const uint32_t mask = 2 * a.N - 1;  // psi has order 2N, a power of two
    // exponent of r = psi^(2 brv(slot) + 1); exponents are taken mod 2N
    const uint32_t re = 2 * (__brev(slot) >> (32 - a.logN)) + 1;
    const uint32_t *fw = a.fw + (size_t)limb * a.N;
    auto rpow = [&](uint32_t e) { return psi_pow(fw, (re * e) & mask, a.N, a.logN, lc); };
    const uint32_t step_c = rpow(0u - a.Bt), step_r = rpow(0u - a.Wp), step_j = rpow(0u - 1u);
    const uint32_t polys = a.Co * a.w_groups, p0 = pblk * kSynthPolys, kk = a.k * a.k;
    const uint32_t cpb = kSynthTaps / kk > 0 ? kSynthTaps / kk : 1;
    uint64_t acc[kSynthPolys], psum = 0;
#pragma unroll
    for (uint32_t pb = 0; pb < kSynthPolys; pb++) acc[pb] = 0;
    // the walk starts from c_n^{-1} 2^64 r^O (Montgomery form of
    // c_n^{-1} 2^32 r^O), so every tap power carries the output scale
    uint32_t pc = mont_mul(rpow(a.O), a.wscale[limb], lc);
    for (uint32_t cp0 = 0; cp0 < a.ci; cp0 += cpb) {
        const uint32_t nc = min(cpb, a.ci - cp0), nt = nc * kk;
        __syncthreads();  // the previous chunk's weights are no longer read
        // consecutive threads take consecutive taps of one polynomial: the
        // int8 weights of (cw, di, dj) are contiguous for a fixed output
        for (uint32_t idx = threadIdx.x; idx < nt * kSynthPolys; idx += 256) {
            const uint32_t t = idx % nt, pb = idx / nt, p = p0 + pb;
            int32_t gsum = 0;
            if (p < polys) {
                const uint32_t o = p / a.w_groups, g = p % a.w_groups, cw = g * a.ci + cp0 + t / kk;
                if (cw < a.Ci) {
                    const uint32_t G = o / a.c_n, j = o % a.c_n, tap = t % kk;
                    for (uint32_t b = 0; b < a.c_n; b++) {
                        const int v = a.w[((size_t)(G * a.c_n + b) * a.Ci + cw) * kk + tap];
                        gsum += (__popc(j & b) & 1) ? -v : v;
                    }
                }
            }
            gs[t][pb] = (uint32_t)(gsum + (1 << 13));
        }
        __syncthreads();
        uint32_t t = 0;
        for (uint32_t c = 0; c < nc; c++, pc = mont_mul(pc, step_c, lc)) {
            uint32_t pr = pc;
            for (uint32_t di = 0; di < a.k; di++, pr = mont_mul(pr, step_r, lc)) {
                uint32_t pw = pr;
                for (uint32_t dj = 0; dj < a.k; dj++, pw = mont_mul(pw, step_j, lc), t++) {
                    const uint4 *row = reinterpret_cast<const uint4 *>(gs[t]);
                    psum += pw;
#pragma unroll
                    for (uint32_t v4 = 0; v4 < kSynthPolys / 4; v4++) {
                        const uint4 v = row[v4];
                        acc[4 * v4 + 0] += (uint64_t)v.x * pw;
                        acc[4 * v4 + 1] += (uint64_t)v.y * pw;
                        acc[4 * v4 + 2] += (uint64_t)v.z * pw;
                        acc[4 * v4 + 3] += (uint64_t)v.w * pw;
                    }
                }
            }
        }
    }
#pragma unroll
    for (uint32_t pb = 0; pb < kSynthPolys; pb++) {
        const uint32_t p = p0 + pb;
        if (p >= polys) break;
        // y = sum gw pw + q 2^32, in [0, 2^64) (the unsigned wrap-around of
        // the subtraction cancels because the true value is in range); the
        // powers are c_n^{-1} 2^64 r^e, so the reduction leaves
        // c_n^{-1} 2^32 sum gw r^e
        const uint64_t y = acc[pb] - (psum << 13) + ((uint64_t)lc.q << 32);
        // fold the high word (hi 2^32 = hi r32 mod q), then reduce:
        // hi r32 + lo <= (2^32 - 1) q < q 2^32
        a.out[((size_t)p * a.L + limb) * a.N + slot] =
            redc((uint64_t)(uint32_t)(y >> 32) * lc.r32 + (uint32_t)y, lc);
    }
}

}  // namespace

extern "C" int hyena_synth_weights(const hyena_ctx *c, const hyena_conv_desc *d, const int8_t *d_w,
                                   uint32_t *d_wntt, hyena_stream_t s) {
    if (!c || !d || !d_w || !d_wntt) return set_error(HYENA_EINVAL, "hyena_synth_weights: NULL argument");
    if (!d->Bt) return set_error(HYENA_EINVAL, "hyena_synth_weights: descriptor not planned");
    // the signs popc(j & b) of the Walsh combination form the Sylvester
    // matrix only for a power of two
    if (d->c_n & (d->c_n - 1)) return set_error(HYENA_EINVAL, "hyena_synth_weights: c_n must be a power of two");
    if (d->depthwise) return set_error(HYENA_EUNSUPPORTED, "hyena_synth_weights: depthwise layers use hyena_encode_weights");
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_synth_weights: context was created host-only");
    if (c->N % 256) return set_error(HYENA_EUNSUPPORTED, "hyena_synth_weights: N must be a multiple of 256");
    const uint32_t cn = d->c_n ? d->c_n : 1;
    if (d->k * d->k > kSynthTaps || cn > 64 || d->Co % cn || !d->ci || (size_t)d->ci * d->w_groups < d->Ci ||
        (uint64_t)d->ci * d->k * d->k >= (1u << 17))
        return set_error(HYENA_EINVAL, "hyena_synth_weights: descriptor fields inconsistent with a plan");
    const size_t polys = (size_t)d->Co * d->w_groups;
    if (polys == 0) return HYENA_OK;
    const size_t blocks = (polys + kSynthPolys - 1) / kSynthPolys * (c->N / 256);
    if (blocks > 0x7fffffffu / 256) return set_error(HYENA_EINVAL, "hyena_synth_weights: layer too large for one launch");
    SynthArgs a{};
    a.w = d_w;
    a.out = d_wntt;
    a.fw = c->d_fw;
    a.N = c->N;
    a.L = c->L;
    a.logN = c->logN;
    a.Co = d->Co;
    a.Ci = d->Ci;
    a.k = d->k;
    a.ci = d->ci;
    a.Bt = d->Bt;
    a.Wp = d->Wp;
    a.O = d->O;
    a.w_groups = d->w_groups;
    a.c_n = cn;
    a.kchunks = c->N / 256;
    a.lt = c->lt;
    for (uint32_t i = 0; i < c->L; i++) {
        a.wscale[i] = to_montgomery(to_montgomery(h_powmod(a.c_n, c->q[i] - 2, c->q[i]), c->q[i]), c->q[i]);
    }
    hipLaunchKernelGGL(synth_weights_kernel, dim3((unsigned)blocks, c->L), dim3(256), 0, (hipStream_t)s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_synth_weights: ") + hipGetErrorString(e));
    return HYENA_OK;
}
