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
    uint32_t wwords;      // 32-bit words of LDS holding the taps
    uint32_t win_len;     // DCHUNK + (k - 1)(Wp + 1): window length per part
    LimbTable lt;
};

__device__ __forceinline__ uint32_t dcsub(uint32_t x, uint32_t q) { return min(x, x - q); }

__device__ __forceinline__ uint32_t dmont(uint64_t t, uint32_t q, uint32_t qn) {
    // t < q 2^32 -> t 2^-32 mod q in [0, 2q)
    const uint32_t m = (uint32_t)t * qn;
    return (uint32_t)(((uint64_t)m * q + t) >> 32);
}

// One block: DCHUNK consecutive output coefficients k0 ... k0 + DCHUNK - 1 of
// both parts of one (row, output channel, limb). For every input channel the
// block stages in LDS the window of input coefficients its taps read: with the
// channel's largest exponent e_hi and tap span `span` (taps have exponents
// e_hi - d, 0 <= d <= span), raw indices j = k - e run over
// [k0 - e_hi, k0 + DCHUNK - 1 - e_hi + span]; the window holds a[j] for j >= 0
// and -a[j + N] for j < 0 (the negacyclic wrap), so tap e = e_hi - d reads
// window position k - k0 + d with no per-lane branch.
__global__ void __launch_bounds__(256) direct_kernel(DirectArgs a) {
    extern __shared__ int32_t smem[];
    int8_t *lw = reinterpret_cast<int8_t *>(smem);   // this output channel's taps, [wch][k][k]
    int32_t *win = smem + a.wwords;                   // [2][win_len] signed window
    const uint32_t tid = threadIdx.x;
    const uint32_t k0 = blockIdx.x * DCHUNK;
    const uint32_t limb = blockIdx.y % a.L, o = blockIdx.y / a.L;
    const uint32_t row = blockIdx.z;     // image x tile
    const uint32_t kk2 = a.k * a.k, nw = a.wch * kk2;
    for (uint32_t i = tid; i < nw; i += 256) lw[i] = a.w[(size_t)o * nw + i];

    const size_t LN = (size_t)a.L * a.N;
    const uint32_t wl = a.win_len;       // DCHUNK + span
    int64_t acc[2][DSLICE];
#pragma unroll
    for (int p = 0; p < 2; p++)
#pragma unroll
        for (int s = 0; s < DSLICE; s++) acc[p][s] = 0;

    // input channels of this output: all of them, or channel o alone if depthwise
    const uint32_t ch_first = a.depthwise ? o : 0, ch_end = a.depthwise ? o + 1 : a.Ci;
    for (uint32_t ch = ch_first; ch < ch_end; ch++) {
        const uint32_t g = ch / a.ci, cp = ch % a.ci;
        const int8_t *wt = lw + (a.depthwise ? 0 : ch * kk2);
        const uint32_t e_hi = a.O - cp * a.Bt;          // >= span: O = (ci-1) Bt + span
        const int32_t j0 = (int32_t)k0 - (int32_t)e_hi;  // >= -(N - 1)
        const uint32_t *src = a.ct + ((size_t)row * a.n_groups + g) * 2 * LN + (size_t)limb * a.N;
        __syncthreads();   // the taps (first pass) or the previous window are no longer read
        for (uint32_t i = tid; i < wl; i += 256) {
            const int32_t j = j0 + (int32_t)i;             // in [-(N-1), N-1]
            const uint32_t jj = j >= 0 ? (uint32_t)j : (uint32_t)(j + (int32_t)a.N);
            const int32_t v0 = (int32_t)src[jj], v1 = (int32_t)src[LN + jj];
            win[i] = j >= 0 ? v0 : -v0;
            win[wl + i] = j >= 0 ? v1 : -v1;
        }
        __syncthreads();
        for (uint32_t di = 0; di < a.k; di++)
            for (uint32_t dj = 0; dj < a.k; dj++) {
                const int32_t w = wt[di * a.k + dj];
                if (w == 0) continue;
                const uint32_t d = di * a.Wp + dj;           // e = e_hi - d, d <= span
#pragma unroll
                for (int s = 0; s < DSLICE; s++) {
                    const uint32_t pos = (uint32_t)s * 256u + tid + d;   // < DCHUNK + span
                    acc[0][s] += (int64_t)w * (int64_t)win[pos];
                    acc[1][s] += (int64_t)w * (int64_t)win[wl + pos];
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
    for (uint32_t q : c->q)   // the bias q 2^29 must cover every signed sum
        if (q <= (1u << 29)) return set_error(HYENA_EINVAL, "hyena_conv_direct: primes must exceed 2^29");
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
    const uint32_t span = (d->k - 1) * (d->Wp + 1);
    if (d->O != (d->ci - 1) * d->Bt + span) return set_error(HYENA_EINVAL, "hyena_conv_direct: inconsistent descriptor");
    a.wwords = (a.wch * a.k * a.k + 3) / 4;
    a.win_len = DCHUNK + span;
    const size_t lds = 4 * ((size_t)a.wwords + 2 * (size_t)a.win_len);
    if (lds > 64 * 1024) return set_error(HYENA_EINVAL, "hyena_conv_direct: layer needs more than 64 KiB of LDS");
    const dim3 grid(c->N / DCHUNK, c->L * d->Co, (unsigned)rows);
    hipLaunchKernelGGL(direct_kernel, grid, dim3(256), lds, (hipStream_t)s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_conv_direct: ") + hipGetErrorString(e));
    return HYENA_OK;
}
