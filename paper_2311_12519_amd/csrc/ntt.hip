// Negacyclic NTT / inverse NTT for gfx950.
//
// Forward: A[k] = sum_j a[j] psi^((2 brv(k) + 1) j) mod q (bit-reversed output),
// computed with Cooley-Tukey butterflies whose twiddles are psi powers in
// bit-reversed order. Inverse: Gentleman-Sande butterflies with psi^-1 powers,
// natural-order output, times N^{-1} (folded into the last stage). The NTT is
// what turns the ciphertext-by-kernel-polynomial products of the padded
// convolution into pointwise products; q = 1 mod 2N makes it exist.
//
// Design: one workgroup of T = 2^LOGT threads transforms one limb of one
// polynomial (N = 2^LOGN residues, 16..64 KiB) resident in LDS. Each thread
// keeps E = N/T residues in registers and runs e <= LOGE consecutive butterfly
// stages on them (a radix-2^e pass) between LDS exchanges. The first pass
// reads HBM directly with unit stride across lanes; the last pass writes
// through LDS so that the HBM store is coalesced too. LDS words are padded
// by one per 32 to break the bank conflicts of the strided passes.
#include "internal.h"

namespace {

__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t q) {
    // x in [0, 2q) -> [0, q): x - q wraps above x exactly when x < q
    return min(x, x - q);
}

// Shoup multiplication: a * w mod q with ws = floor(w 2^32 / q), a < 2^32.
__device__ __forceinline__ uint32_t shoup(uint32_t a, uint32_t w, uint32_t ws, uint32_t q) {
    uint32_t qh = __umulhi(a, ws);
    return csub(a * w - qh * q, q);
}

__device__ __forceinline__ uint32_t lds_idx(uint32_t j) { return j + (j >> 5); }

template <int LOGN>
struct Sched;
// pass widths (stages per pass); the first entry is the register radix
template <> struct Sched<10> { static constexpr int LOGT = 6, NP = 3; static constexpr int e[3] = {4, 3, 3}; };
template <> struct Sched<11> { static constexpr int LOGT = 7, NP = 3; static constexpr int e[3] = {4, 4, 3}; };
template <> struct Sched<12> { static constexpr int LOGT = 8, NP = 3; static constexpr int e[3] = {4, 4, 4}; };
template <> struct Sched<13> { static constexpr int LOGT = 8, NP = 3; static constexpr int e[3] = {5, 4, 4}; };
template <> struct Sched<14> { static constexpr int LOGT = 9, NP = 3; static constexpr int e[3] = {5, 5, 4}; };

// One pass of forward stages [s0, s0+e) on the thread's E registers.
// Group gi of the pass holds indices b*(N>>s0) + o + r*(N>>(s0+e)), r < 2^e,
// with o = gi mod (N>>(s0+e)), b = gi div (N>>(s0+e)); thread tid owns groups
// gi = tid + k*T, k < E>>e, stored at registers x[k*2^e + r].
template <int LOGN, int LOGT, int E_LOG, int S0, int EP>
__device__ __forceinline__ void fwd_pass(uint32_t (&x)[1 << E_LOG], const uint2 *__restrict__ tw,
                                         uint32_t q, uint32_t tid) {
    constexpr int GE = 1 << EP;
    constexpr int NG = (1 << E_LOG) >> EP;          // groups per thread
    constexpr uint32_t OSPAN = 1u << (LOGN - S0 - EP);
#pragma unroll
    for (int kg = 0; kg < NG; kg++) {
        const uint32_t gi = tid + (uint32_t)kg * (1u << LOGT);
        const uint32_t b = gi / OSPAN;
#pragma unroll
        for (int u = 0; u < EP; u++) {
            const int half = GE >> (u + 1);
#pragma unroll
            for (int r = 0; r < GE; r++) {
                if (r & half) continue;
                const uint32_t widx = (1u << (S0 + u)) + (b << u) + ((uint32_t)r >> (EP - u));
                const uint2 w = tw[widx];
                uint32_t &lo = x[kg * GE + r];
                uint32_t &hi = x[kg * GE + r + half];
                const uint32_t t = shoup(hi, w.x, w.y, q);
                const uint32_t s = lo + t;
                hi = csub(lo - t + q, q);
                lo = csub(s, q);
            }
        }
    }
}

template <int LOGN, int LOGT, int E_LOG, int S0, int EP>
__device__ __forceinline__ void to_lds(const uint32_t (&x)[1 << E_LOG], uint32_t *lds, uint32_t tid) {
    constexpr int GE = 1 << EP;
    constexpr int NG = (1 << E_LOG) >> EP;
    constexpr uint32_t OSPAN = 1u << (LOGN - S0 - EP);
#pragma unroll
    for (int kg = 0; kg < NG; kg++) {
        const uint32_t gi = tid + (uint32_t)kg * (1u << LOGT);
        const uint32_t o = gi % OSPAN, b = gi / OSPAN;
#pragma unroll
        for (int r = 0; r < GE; r++) lds[lds_idx(b * (OSPAN << EP) + o + (uint32_t)r * OSPAN)] = x[kg * GE + r];
    }
}

template <int LOGN, int LOGT, int E_LOG, int S0, int EP>
__device__ __forceinline__ void from_lds(uint32_t (&x)[1 << E_LOG], const uint32_t *lds, uint32_t tid) {
    constexpr int GE = 1 << EP;
    constexpr int NG = (1 << E_LOG) >> EP;
    constexpr uint32_t OSPAN = 1u << (LOGN - S0 - EP);
#pragma unroll
    for (int kg = 0; kg < NG; kg++) {
        const uint32_t gi = tid + (uint32_t)kg * (1u << LOGT);
        const uint32_t o = gi % OSPAN, b = gi / OSPAN;
#pragma unroll
        for (int r = 0; r < GE; r++) x[kg * GE + r] = lds[lds_idx(b * (OSPAN << EP) + o + (uint32_t)r * OSPAN)];
    }
}

template <int LOGN>
__global__ void __launch_bounds__(1 << Sched<LOGN>::LOGT)
ntt_fwd_kernel(uint32_t *__restrict__ poly, const uint2 *__restrict__ tw_all, LimbTable lt, uint32_t L) {
    constexpr int LOGT = Sched<LOGN>::LOGT;
    constexpr int E_LOG = LOGN - LOGT;
    constexpr int N = 1 << LOGN, T = 1 << LOGT, E = 1 << E_LOG;
    constexpr int E0 = Sched<LOGN>::e[0], E1 = Sched<LOGN>::e[1], E2 = Sched<LOGN>::e[2];
    static_assert(E0 + E1 + E2 == LOGN, "schedule must cover every stage");
    static_assert(E0 == E_LOG, "first pass uses the full register radix");
    __shared__ uint32_t lds[N + N / 32];
    const uint32_t tid = threadIdx.x;
    const uint32_t limb = blockIdx.x % L;
    uint32_t *a = poly + (size_t)blockIdx.x * N;
    const uint2 *tw = tw_all + (size_t)limb * N;
    const uint32_t q = lt.c[limb].q;
    uint32_t x[E];
    // pass 0: stages [0, E0); group of thread tid: indices tid + r*T
#pragma unroll
    for (int r = 0; r < E; r++) x[r] = a[tid + r * T];
    fwd_pass<LOGN, LOGT, E_LOG, 0, E0>(x, tw, q, tid);
    to_lds<LOGN, LOGT, E_LOG, 0, E0>(x, lds, tid);
    __syncthreads();
    from_lds<LOGN, LOGT, E_LOG, E0, E1>(x, lds, tid);
    fwd_pass<LOGN, LOGT, E_LOG, E0, E1>(x, tw, q, tid);
    __syncthreads();
    to_lds<LOGN, LOGT, E_LOG, E0, E1>(x, lds, tid);
    __syncthreads();
    from_lds<LOGN, LOGT, E_LOG, E0 + E1, E2>(x, lds, tid);
    fwd_pass<LOGN, LOGT, E_LOG, E0 + E1, E2>(x, tw, q, tid);
    __syncthreads();
    to_lds<LOGN, LOGT, E_LOG, E0 + E1, E2>(x, lds, tid);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; r++) a[tid + r * T] = lds[lds_idx(tid + r * T)];
}

// Inverse: Gentleman-Sande stages run in the reverse order of the forward
// ones (len = 1, 2, ..., N/2). Stage with m = 2^s blocks (s from LOGN-1 down
// to 0) pairs j and j + (N >> (s+1)) in block j >> (LOGN - s) with twiddle
// psi^-brv(m + block). Passes are the forward passes taken in reverse.
template <int LOGN, int LOGT, int E_LOG, int S0, int EP, bool LAST>
__device__ __forceinline__ void inv_pass(uint32_t (&x)[1 << E_LOG], const uint2 *__restrict__ tw,
                                         const LimbConst &lc, uint32_t tid) {
    constexpr int GE = 1 << EP;
    constexpr int NG = (1 << E_LOG) >> EP;
    constexpr uint32_t OSPAN = 1u << (LOGN - S0 - EP);
    const uint32_t q = lc.q;
#pragma unroll
    for (int kg = 0; kg < NG; kg++) {
        const uint32_t gi = tid + (uint32_t)kg * (1u << LOGT);
        const uint32_t b = gi / OSPAN;
#pragma unroll
        for (int u = EP - 1; u >= 0; u--) {
            const int half = GE >> (u + 1);
#pragma unroll
            for (int r = 0; r < GE; r++) {
                if (r & half) continue;
                const uint32_t widx = (1u << (S0 + u)) + (b << u) + ((uint32_t)r >> (EP - u));
                const uint2 w = tw[widx];
                uint32_t &lo = x[kg * GE + r];
                uint32_t &hi = x[kg * GE + r + half];
                const uint32_t s = csub(lo + hi, q);
                const uint32_t d = csub(lo - hi + q, q);
                if (LAST && S0 + u == 0) {
                    // last stage: fold N^{-1} into both outputs
                    (void)w;
                    lo = shoup(s, lc.ninv, lc.ninvs, q);
                    hi = shoup(d, lc.w1n, lc.w1ns, q);
                } else {
                    lo = s;
                    hi = shoup(d, w.x, w.y, q);
                }
            }
        }
    }
}

template <int LOGN>
__global__ void __launch_bounds__(1 << Sched<LOGN>::LOGT)
ntt_inv_kernel(uint32_t *__restrict__ poly, const uint2 *__restrict__ tw_all, LimbTable lt, uint32_t L) {
    constexpr int LOGT = Sched<LOGN>::LOGT;
    constexpr int E_LOG = LOGN - LOGT;
    constexpr int N = 1 << LOGN, T = 1 << LOGT, E = 1 << E_LOG;
    constexpr int E0 = Sched<LOGN>::e[0], E1 = Sched<LOGN>::e[1], E2 = Sched<LOGN>::e[2];
    __shared__ uint32_t lds[N + N / 32];
    const uint32_t tid = threadIdx.x;
    const uint32_t limb = blockIdx.x % L;
    uint32_t *a = poly + (size_t)blockIdx.x * N;
    const uint2 *tw = tw_all + (size_t)limb * N;
    const LimbConst lc = lt.c[limb];
    uint32_t x[E];
#pragma unroll
    for (int r = 0; r < E; r++) lds[lds_idx(tid + r * T)] = a[tid + r * T];
    __syncthreads();
    from_lds<LOGN, LOGT, E_LOG, E0 + E1, E2>(x, lds, tid);
    inv_pass<LOGN, LOGT, E_LOG, E0 + E1, E2, false>(x, tw, lc, tid);
    __syncthreads();
    to_lds<LOGN, LOGT, E_LOG, E0 + E1, E2>(x, lds, tid);
    __syncthreads();
    from_lds<LOGN, LOGT, E_LOG, E0, E1>(x, lds, tid);
    inv_pass<LOGN, LOGT, E_LOG, E0, E1, false>(x, tw, lc, tid);
    __syncthreads();
    to_lds<LOGN, LOGT, E_LOG, E0, E1>(x, lds, tid);
    __syncthreads();
    from_lds<LOGN, LOGT, E_LOG, 0, E0>(x, lds, tid);
    inv_pass<LOGN, LOGT, E_LOG, 0, E0, true>(x, tw, lc, tid);
#pragma unroll
    for (int r = 0; r < E; r++) a[tid + r * T] = x[r];
}

template <int LOGN>
hipError_t launch(uint32_t *d, size_t P, const hyena_ctx *c, bool inv, hipStream_t s) {
    const dim3 grid((unsigned)(P * c->L)), block(1u << Sched<LOGN>::LOGT);
    if (inv)
        hipLaunchKernelGGL(ntt_inv_kernel<LOGN>, grid, block, 0, s, d, (const uint2 *)c->d_iw, c->lt, c->L);
    else
        hipLaunchKernelGGL(ntt_fwd_kernel<LOGN>, grid, block, 0, s, d, (const uint2 *)c->d_fw, c->lt, c->L);
    return hipGetLastError();
}

}  // namespace

int launch_ntt(const hyena_ctx *c, uint32_t *d, size_t P, bool inv, hipStream_t s) {
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_ntt: context was created host-only");
    if (P == 0) return HYENA_OK;
    if (P * c->L > 0x7fffffffull) return set_error(HYENA_EINVAL, "hyena_ntt: too many polynomials");
    hipError_t e;
    switch (c->logN) {
        case 10: e = launch<10>(d, P, c, inv, s); break;
        case 11: e = launch<11>(d, P, c, inv, s); break;
        case 12: e = launch<12>(d, P, c, inv, s); break;
        case 13: e = launch<13>(d, P, c, inv, s); break;
        case 14: e = launch<14>(d, P, c, inv, s); break;
        default: return set_error(HYENA_EUNSUPPORTED, "hyena_ntt: unsupported N");
    }
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_ntt: ") + hipGetErrorString(e));
    return HYENA_OK;
}

extern "C" int hyena_ntt(const hyena_ctx *c, uint32_t *d_poly, size_t P, hyena_stream_t s) {
    if (!c || (P && !d_poly)) return set_error(HYENA_EINVAL, "hyena_ntt: NULL argument");
    return launch_ntt(c, d_poly, P, false, (hipStream_t)s);
}

extern "C" int hyena_intt(const hyena_ctx *c, uint32_t *d_poly, size_t P, hyena_stream_t s) {
    if (!c || (P && !d_poly)) return set_error(HYENA_EINVAL, "hyena_intt: NULL argument");
    return launch_ntt(c, d_poly, P, true, (hipStream_t)s);
}
