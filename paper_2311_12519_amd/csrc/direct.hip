// Coefficient-domain direct convolution for gfx950.
//
// Y_{o,tau} = sum_g ct_{tau,g} * K_{o,g} in Z_q[X]/(X^N + 1), computed straight
// from the integer kernel taps: K_{o,g} has one monomial f X^e per tap, and
// X^e * a is a negacyclic shift (coefficient j - e, negated where it wraps).
// This is the regime of the "Lazy Reduction" passage of the "Latency
// Optimization" section: products of ciphertext coefficients by small
// plaintext integers taken without reduction, summed in wide words, one
// reduction per output coefficient. It needs no NTT of inputs, weights or
// outputs, so for layers with few taps per output (depthwise, and c_i = 1
// layers with few input ciphertexts) it does less work than NTT + pointwise
// product + inverse NTT.
//
// Arithmetic: |f| <= 128 and residues < 2^31, so every product is below 2^38
// in magnitude and up to 2^20 taps sum exactly in a signed 64-bit word. Adding
// q 2^29 (a multiple of q, at least the largest magnitude) makes the sum
// non-negative and below q 2^32; one Montgomery reduction gives sum 2^-32 mod
// q and a Montgomery product by 2^64 mod q restores the factor 2^32.
#include <type_traits>

#include "internal.h"

namespace {

constexpr int DSLICE = 4;                     // coefficients per thread, 256 apart
constexpr uint32_t DCHUNK = 256u * DSLICE;    // coefficients per block

struct DirectArgs {
    const uint32_t *ct;   // [rows][n_groups][2][L][N], coefficient domain
    const int8_t *w;      // [Co][wch][k][k]
    uint32_t *out;        // [rows][Co][2][L][N], coefficient domain
    uint32_t N, L, Co, Ci, k, ci, Bt, Wp, O, n_groups, depthwise, wch;
    LimbTable lt;
};

__device__ __forceinline__ uint32_t dcsub(uint32_t x, uint32_t q) { return min(x, x - q); }

__device__ __forceinline__ uint32_t dmont(uint64_t t, uint32_t q, uint32_t qn) {
    // t < q 2^32 -> t 2^-32 mod q in [0, 2q)
    const uint32_t m = (uint32_t)t * qn;
    return (uint32_t)(((uint64_t)m * q + t) >> 32);
}

// Add tap (w, e) of one input polynomial pair (parts 0 and 1 at src, src + LN)
// to the thread's DSLICE coefficients k = k0 + s 256 + tid of both parts. The
// coefficient read is k - e, or k - e + N with the weight negated where k < e;
// both lie in [0, N).
__device__ __forceinline__ void direct_tap(int64_t (&acc)[2][DSLICE], const uint32_t *src, size_t LN,
                                           int32_t w, uint32_t e, uint32_t k0, uint32_t N, uint32_t tid) {
#pragma unroll
    for (int s = 0; s < DSLICE; s++) {
        const uint32_t kb = k0 + (uint32_t)s * 256u;   // block-uniform, kb + 256 <= N
        uint32_t idx;
        int32_t ws;
        if (kb >= e) {                  // no lane wraps
            idx = kb - e + tid;
            ws = w;
        } else if (kb + 256u <= e) {    // every lane wraps
            idx = kb + N - e + tid;
            ws = -w;
        } else {                        // the range straddles e: per lane
            const uint32_t kk = kb + tid;
            const bool wrap = kk < e;
            idx = wrap ? kk + N - e : kk - e;
            ws = wrap ? -w : w;
        }
        acc[0][s] += (int64_t)ws * (int64_t)(int32_t)src[idx];
        acc[1][s] += (int64_t)ws * (int64_t)(int32_t)src[LN + idx];
    }
}

__global__ void __launch_bounds__(256) direct_kernel(DirectArgs a) {
    extern __shared__ int8_t lw[];   // this output channel's taps, [wch][k][k]
    const uint32_t tid = threadIdx.x;
    const uint32_t k0 = blockIdx.x * DCHUNK;
    const uint32_t limb = blockIdx.y % a.L, o = blockIdx.y / a.L;
    const uint32_t row = blockIdx.z;     // image x tile
    const uint32_t kk2 = a.k * a.k, nw = a.wch * kk2;
    for (uint32_t i = tid; i < nw; i += 256) lw[i] = a.w[(size_t)o * nw + i];
    __syncthreads();

    const size_t LN = (size_t)a.L * a.N;
    int64_t acc[2][DSLICE];
#pragma unroll
    for (int p = 0; p < 2; p++)
#pragma unroll
        for (int s = 0; s < DSLICE; s++) acc[p][s] = 0;

    if (a.depthwise) {
        // channel o sits at position o mod ci of input group o / ci
        const uint32_t g = o / a.ci, cp = o % a.ci;
        const uint32_t *src = a.ct + ((size_t)row * a.n_groups + g) * 2 * LN + (size_t)limb * a.N;
        for (uint32_t di = 0; di < a.k; di++)
            for (uint32_t dj = 0; dj < a.k; dj++) {
                const int32_t w = lw[di * a.k + dj];
                if (w == 0) continue;
                const uint32_t e = a.O - cp * a.Bt - di * a.Wp - dj;
                direct_tap(acc, src, LN, w, e, k0, a.N, tid);
            }
    } else {
        for (uint32_t g = 0; g < a.n_groups; g++) {
            const uint32_t *src = a.ct + ((size_t)row * a.n_groups + g) * 2 * LN + (size_t)limb * a.N;
            for (uint32_t cp = 0; cp < a.ci; cp++) {
                const uint32_t ch = g * a.ci + cp;
                if (ch >= a.Ci) break;   // short last group
                for (uint32_t di = 0; di < a.k; di++)
                    for (uint32_t dj = 0; dj < a.k; dj++) {
                        const int32_t w = lw[(ch * a.k + di) * a.k + dj];
                        if (w == 0) continue;
                        const uint32_t e = a.O - cp * a.Bt - di * a.Wp - dj;
                        direct_tap(acc, src, LN, w, e, k0, a.N, tid);
                    }
            }
        }
    }

    const LimbConst lc = a.lt.c[limb];
    const uint32_t q = lc.q, qn = lc.qinv_neg;
    const int64_t bias = (int64_t)q << 29;
    uint32_t *dst = a.out + ((size_t)row * a.Co + o) * 2 * LN + (size_t)limb * a.N;
#pragma unroll
    for (int p = 0; p < 2; p++)
#pragma unroll
        for (int s = 0; s < DSLICE; s++) {
            const uint64_t t = (uint64_t)(acc[p][s] + bias);          // in [0, q 2^32)
            const uint32_t z = dcsub(dmont(t, q, qn), q);             // t 2^-32 mod q
            const uint32_t y = dcsub(dmont((uint64_t)z * lc.r64, q, qn), q);   // z 2^32 = t mod q
            dst[(size_t)p * LN + k0 + (uint32_t)s * 256u + tid] = y;
        }
}

}  // namespace

extern "C" int hyena_conv_direct(const hyena_ctx *c, const hyena_conv_desc *d, const uint32_t *d_ct,
                                 const int8_t *d_w, uint32_t *d_out, hyena_stream_t s) {
    if (!c || !d || !d_ct || !d_w || !d_out) return set_error(HYENA_EINVAL, "hyena_conv_direct: NULL argument");
    if (!d->Bt || !d->n_groups) return set_error(HYENA_EINVAL, "hyena_conv_direct: descriptor not planned");
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_conv_direct: context was created host-only");
    if (c->N % DCHUNK) return set_error(HYENA_EUNSUPPORTED, "hyena_conv_direct: N must be a multiple of 1024");
    if (d->O >= c->N) return set_error(HYENA_EINVAL, "hyena_conv_direct: kernel exponents exceed N");
    const uint32_t batch = d->batch ? d->batch : 1;
    const size_t rows = (size_t)batch * d->tiles;
    const size_t taps = d->depthwise ? (size_t)d->k * d->k : (size_t)d->n_groups * d->ci * d->k * d->k;
    if (taps > (1u << 20)) return set_error(HYENA_EINVAL, "hyena_conv_direct: more than 2^20 taps per output");
    if ((size_t)c->L * d->Co > 65535 || rows > 65535)
        return set_error(HYENA_EINVAL, "hyena_conv_direct: grid too large");
    const size_t LN = (size_t)c->L * c->N;
    const uintptr_t in_lo = (uintptr_t)d_ct, in_hi = in_lo + rows * d->n_groups * 2 * LN * 4;
    const uintptr_t out_lo = (uintptr_t)d_out, out_hi = out_lo + rows * d->Co * 2 * LN * 4;
    if (out_lo < in_hi && in_lo < out_hi) return set_error(HYENA_EINVAL, "hyena_conv_direct: d_out overlaps d_ct");
    DirectArgs a{};
    a.ct = d_ct;
    a.w = d_w;
    a.out = d_out;
    a.N = c->N;
    a.L = c->L;
    a.Co = d->Co;
    a.Ci = d->Ci;
    a.k = d->k;
    a.ci = d->ci;
    a.Bt = d->Bt;
    a.Wp = d->Wp;
    a.O = d->O;
    a.n_groups = d->n_groups;
    a.depthwise = d->depthwise;
    a.wch = d->depthwise ? 1 : d->Ci;
    a.lt = c->lt;
    const size_t lds = ((size_t)a.wch * a.k * a.k + 3) & ~(size_t)3;
    const dim3 grid(c->N / DCHUNK, c->L * d->Co, (unsigned)rows);
    hipLaunchKernelGGL(direct_kernel, grid, dim3(256), lds, (hipStream_t)s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_conv_direct: ") + hipGetErrorString(e));
    return HYENA_OK;
}
