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
// stages on them (a radix-2^e pass) between LDS exchanges. The passes at the
// two ends touch HBM directly: the one over the first stages with unit stride
// across lanes, the one over the last stages with runs of 2^e consecutive
// residues per thread (16-byte accesses), so a transform of P passes needs
// P - 1 LDS exchanges. LDS words are padded by one per 32 to break the bank
// conflicts of the strided passes. Polynomials must be 16-byte aligned.
#include <algorithm>

#include "bfv.h"

namespace {

__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t q) {
    // x in [0, 2q) -> [0, q): x - q wraps above x exactly when x < q
    return min(x, x - q);
}

// Montgomery multiplication: a * wm * 2^-32 mod q, left in [0, 2q), for any
// a < 2^32 and wm < q (wm = w 2^32 mod q gives a * w mod q). With
// t = a wm < q 2^32 and m = t (-q^-1) mod 2^32, t + m q is divisible by
// 2^32 and (t + m q) / 2^32 < 2q. Both words of each 64-bit product are used,
// so it compiles to two v_mad_u64_u32 and one v_mul_lo_u32 (the fast forms on
// gfx950), and the twiddle tables need no companion words.
__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t wm, uint32_t q, uint32_t qn) {
    const uint64_t t = (uint64_t)a * wm;
    const uint32_t m = (uint32_t)t * qn;
    return (uint32_t)(((uint64_t)m * q + t) >> 32);
}

// (lo, hi) -> (lo + w hi, lo - w hi). Exact variant (any q < 2^31): values
// in [0, 2q) between stages (2q < 2^32), canonical inputs to the first stage
// and canonical outputs of the last (first, last: the butterfly's stage, known
// once the stage loops are unrolled). Lazy variant (Harvey's butterfly,
// q < 2^30): values in [0, 4q) between stages, reduced after the transform.
template <bool LAZY>
__device__ __forceinline__ void ct_bfly(uint32_t &lo, uint32_t &hi, uint32_t w, uint32_t q, uint32_t qn, bool first,
                                        bool last) {
    if (LAZY) {
        const uint32_t x = min(lo, lo - 2 * q);           // [0, 2q)
        const uint32_t t = mont_mul(hi, w, q, qn);        // [0, 2q)
        lo = x + t;                                       // [0, 4q)
        hi = x - t + 2 * q;                               // (0, 4q)
    } else {
        const uint32_t x = first ? lo : csub(lo, q);      // [0, q)
        const uint32_t t = csub(mont_mul(hi, w, q, qn), q);
        if (last) {
            const uint32_t d = x - t;
            hi = min(d, d + q);   // x - t wraps above 2q exactly when x < t
            lo = csub(x + t, q);
        } else {
            lo = x + t;           // [0, 2q)
            hi = x - t + q;       // (0, 2q)
        }
    }
}

// (lo, hi) -> (lo + hi, w (lo - hi)). Exact: canonical in and out. Lazy:
// [0, 2q) in and out.
template <bool LAZY>
__device__ __forceinline__ void gs_bfly(uint32_t &lo, uint32_t &hi, uint32_t w, uint32_t q, uint32_t qn) {
    if (LAZY) {
        const uint32_t s = lo + hi;                       // [0, 4q)
        const uint32_t t = lo - hi + 2 * q;               // (0, 4q)
        lo = min(s, s - 2 * q);
        hi = mont_mul(t, w, q, qn);
    } else {
        const uint32_t s = lo + hi;
        const uint32_t d = lo - hi + q;                   // (0, 2q)
        lo = csub(s, q);
        hi = csub(mont_mul(d, w, q, qn), q);
    }
}

__device__ __forceinline__ uint32_t lds_idx(uint32_t j) { return j + (j >> 5); }

// Which waves an exchange between two passes connects. In the pass over
// stages [S0, S0 + EP), thread tid holds the groups gi = tid + kg T, whose
// residues have the index bits [b | r | o]: b = gi's high S0 bits, r the
// register index, o = gi's low LOGN - S0 - EP bits. The wave number sits in
// bits [6, LOGT) of gi, so bit p of it lands on residue bit p when
// p < LOGN - S0 - EP and on residue bit p + EP otherwise. When the two passes
// put every wave bit on the same residue bit, each wave writes to LDS exactly
// the residues it reads back: the exchange needs no workgroup barrier, only
// the wave's own LDS accesses kept in order.
template <int LOGN, int LOGT, int SA, int EA, int SB, int EB>
constexpr bool exchange_in_wave() {
    for (int p = 6; p < LOGT; p++) {
        const int fa = p < LOGN - SA - EA ? p : p + EA;
        const int fb = p < LOGN - SB - EB ? p : p + EB;
        if (fa != fb) return false;
    }
    return true;
}

// The wave's earlier LDS writes are complete before its later LDS reads
// issue, and the compiler keeps LDS accesses on their side.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <bool IN_WAVE>
__device__ __forceinline__ void exchange_sync() {
    if constexpr (IN_WAVE) wave_lds_sync();
    else __syncthreads();
}

// One pass of forward stages [s0, s0+e) on the thread's E registers.
// Group gi of the pass holds indices b*(N>>s0) + o + r*(N>>(s0+e)), r < 2^e,
// with o = gi mod (N>>(s0+e)), b = gi div (N>>(s0+e)); thread tid owns groups
// gi = tid + k*T, k < E>>e, stored at registers x[k*2^e + r].
template <int LOGN, int LOGT, int E_LOG, int S0, int EP, bool LAZY>
__device__ __forceinline__ void fwd_pass(uint32_t (&x)[1 << E_LOG], const uint32_t *__restrict__ tw,
                                         uint32_t q, uint32_t qn, uint32_t tid) {
    constexpr int GE = 1 << EP;
    constexpr int NG = (1 << E_LOG) >> EP;          // groups per thread
    constexpr uint32_t OSPAN = 1u << (LOGN - S0 - EP);
#pragma unroll
    for (int kg = 0; kg < NG; kg++) {
        const uint32_t gi = tid + (uint32_t)kg * (1u << LOGT);
        // the first pass has one block (b = 0): its twiddles are uniform
        const uint32_t b = (S0 == 0) ? 0u : gi / OSPAN;
#pragma unroll
        for (int u = 0; u < EP; u++) {
            const int half = GE >> (u + 1);
#pragma unroll
            for (int r = 0; r < GE; r++) {
                if (r & half) continue;
                const uint32_t widx = (1u << (S0 + u)) + (b << u) + ((uint32_t)r >> (EP - u));
                ct_bfly<LAZY>(x[kg * GE + r], x[kg * GE + r + half], tw[widx], q, qn, S0 + u == 0,
                              S0 + u == LOGN - 1);
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

// A pass that ends at the last stage (S0 + EP == LOGN) gives group gi the
// 2^EP consecutive residues [gi 2^EP, (gi + 1) 2^EP): the thread moves them
// between HBM and registers with 16-byte (or, for 2^EP = 2, 8-byte) accesses,
// and the wave as a whole covers one contiguous span.
template <int LOGT, int E_LOG, int EP>
__device__ __forceinline__ void load_runs(uint32_t (&x)[1 << E_LOG], const uint32_t *__restrict__ a, uint32_t tid) {
    constexpr int GE = 1 << EP, NG = (1 << E_LOG) >> EP;
    static_assert(GE >= 2, "runs of at least two residues");
#pragma unroll
    for (int kg = 0; kg < NG; kg++) {
        const uint32_t *p = a + ((size_t)(tid + (uint32_t)kg * (1u << LOGT)) << EP);
        if constexpr (GE >= 4) {
#pragma unroll
            for (int r = 0; r < GE; r += 4) {
                const uint4 v = *reinterpret_cast<const uint4 *>(p + r);
                x[kg * GE + r] = v.x, x[kg * GE + r + 1] = v.y, x[kg * GE + r + 2] = v.z, x[kg * GE + r + 3] = v.w;
            }
        } else {
            const uint2 v = *reinterpret_cast<const uint2 *>(p);
            x[kg * GE] = v.x, x[kg * GE + 1] = v.y;
        }
    }
}

template <int LOGT, int E_LOG, int EP>
__device__ __forceinline__ void store_runs(const uint32_t (&x)[1 << E_LOG], uint32_t *__restrict__ a, uint32_t tid) {
    constexpr int GE = 1 << EP, NG = (1 << E_LOG) >> EP;
    static_assert(GE >= 2, "runs of at least two residues");
#pragma unroll
    for (int kg = 0; kg < NG; kg++) {
        uint32_t *p = a + ((size_t)(tid + (uint32_t)kg * (1u << LOGT)) << EP);
        if constexpr (GE >= 4) {
#pragma unroll
            for (int r = 0; r < GE; r += 4)
                *reinterpret_cast<uint4 *>(p + r) =
                    make_uint4(x[kg * GE + r], x[kg * GE + r + 1], x[kg * GE + r + 2], x[kg * GE + r + 3]);
        } else {
            *reinterpret_cast<uint2 *>(p) = make_uint2(x[kg * GE], x[kg * GE + 1]);
        }
    }
}

// Forward transform of one limb-polynomial a (N residues) by the block:
// passes of E0, E1, E2 (, E3) stages; E0 = LOGN - LOGT is the register radix
// (every thread holds 2^E0 residues). The first pass reads HBM with unit
// stride across lanes, the last writes runs of consecutive residues; the
// passes between exchange residues through LDS.
template <int LOGN, int LOGT, int E0, int E1, int E2, int E3, bool LAZY>
__device__ __forceinline__ void fwd_front(uint32_t (&x)[1 << (LOGN - LOGT)], const uint32_t *__restrict__ tw,
                                          uint32_t q, uint32_t qn, uint32_t *lds, uint32_t tid) {
    constexpr int E_LOG = LOGN - LOGT;
    constexpr int E = 1 << E_LOG;
    static_assert(E0 + E1 + E2 + E3 == LOGN, "schedule must cover every stage");
    static_assert(E0 == E_LOG && E1 <= E_LOG && E2 <= E_LOG && E3 <= E_LOG, "pass wider than the registers");
    // Before each write to LDS, only this wave's own earlier reads have to be
    // done: a wave writes back exactly the residues it read for the pass it
    // just ran, which no other wave reads. So the barriers are those of the
    // exchanges that cross waves.
    constexpr bool X1 = exchange_in_wave<LOGN, LOGT, 0, E0, E0, E1>();
    constexpr bool X2 = exchange_in_wave<LOGN, LOGT, E0, E1, E0 + E1, E2>();
    constexpr bool X3 = exchange_in_wave<LOGN, LOGT, E0 + E1, E2, E0 + E1 + E2, E3>();
    fwd_pass<LOGN, LOGT, E_LOG, 0, E0, LAZY>(x, tw, q, qn, tid);
    to_lds<LOGN, LOGT, E_LOG, 0, E0>(x, lds, tid);
    exchange_sync<X1>();
    from_lds<LOGN, LOGT, E_LOG, E0, E1>(x, lds, tid);
    fwd_pass<LOGN, LOGT, E_LOG, E0, E1, LAZY>(x, tw, q, qn, tid);
    wave_lds_sync();
    to_lds<LOGN, LOGT, E_LOG, E0, E1>(x, lds, tid);
    exchange_sync<X2>();
    from_lds<LOGN, LOGT, E_LOG, E0 + E1, E2>(x, lds, tid);
    fwd_pass<LOGN, LOGT, E_LOG, E0 + E1, E2, LAZY>(x, tw, q, qn, tid);
    if constexpr (E3 > 0) {
        wave_lds_sync();
        to_lds<LOGN, LOGT, E_LOG, E0 + E1, E2>(x, lds, tid);
        exchange_sync<X3>();
        from_lds<LOGN, LOGT, E_LOG, E0 + E1 + E2, E3>(x, lds, tid);
        fwd_pass<LOGN, LOGT, E_LOG, E0 + E1 + E2, E3, LAZY>(x, tw, q, qn, tid);
    }
    if (LAZY) {
#pragma unroll
        for (int r = 0; r < E; r++) x[r] = csub(min(x[r], x[r] - 2 * q), q);  // [0, 4q) -> [0, q)
    }
}

// Store of the last pass's residues through LDS: each wave holds, per group
// round kg, the 64 * 2^EP consecutive residues starting at 2^EP (kg T + 64 w);
// it writes them to LDS where it read them and reads them back as 16-byte
// pieces contiguous across lanes, so every global store instruction covers
// 1 KiB contiguous (against 16-byte pieces 2^EP words apart when the runs are
// stored from registers). Only the wave's own LDS words move: no barrier.
template <int LOGN, int LOGT, int E_LOG, int EP>
__device__ __forceinline__ void store_staged(const uint32_t (&x)[1 << E_LOG], uint32_t *__restrict__ a,
                                             uint32_t *lds, uint32_t tid) {
    constexpr int GE = 1 << EP, NG = (1 << E_LOG) >> EP;
    static_assert(GE >= 4, "runs of at least four residues");
    wave_lds_sync();
    to_lds<LOGN, LOGT, E_LOG, LOGN - EP, EP>(x, lds, tid);
    wave_lds_sync();
    const uint32_t lane = tid & 63, w0 = tid & ~63u;
#pragma unroll
    for (int kg = 0; kg < NG; kg++) {
        const uint32_t base = (uint32_t)GE * ((uint32_t)kg * (1u << LOGT) + w0);
#pragma unroll
        for (int c = 0; c < GE / 4; c++) {
            const uint32_t j = base + 4 * ((uint32_t)c * 64 + lane);
            *reinterpret_cast<uint4 *>(a + j) =
                make_uint4(lds[lds_idx(j)], lds[lds_idx(j + 1)], lds[lds_idx(j + 2)], lds[lds_idx(j + 3)]);
        }
    }
}

// Forward transform of one limb-polynomial a (N residues) by the block:
// passes of E0, E1, E2 (, E3) stages; E0 = LOGN - LOGT is the register radix
// (every thread holds 2^E0 residues). The first pass reads HBM with unit
// stride across lanes, the last writes runs of consecutive residues (staged
// through the wave's LDS words into stores contiguous across lanes); the
// passes between exchange residues through LDS.
template <int LOGN, int LOGT, int E0, int E1, int E2, int E3, bool LAZY>
__device__ __forceinline__ void ntt_fwd_body(uint32_t *__restrict__ a, const uint32_t *__restrict__ tw,
                                             uint32_t q, uint32_t qn, uint32_t *lds) {
    constexpr int E_LOG = LOGN - LOGT;
    constexpr int T = 1 << LOGT, E = 1 << E_LOG;
    const uint32_t tid = threadIdx.x;
    uint32_t x[E];
#pragma unroll
    for (int r = 0; r < E; r++) x[r] = a[tid + r * T];
    fwd_front<LOGN, LOGT, E0, E1, E2, E3, LAZY>(x, tw, q, qn, lds, tid);
    constexpr int EF = E3 > 0 ? E3 : E2;
    if constexpr ((1 << EF) >= 4) store_staged<LOGN, LOGT, E_LOG, EF>(x, a, lds, tid);
    else store_runs<LOGT, E_LOG, EF>(x, a, tid);
}

// Inverse: Gentleman-Sande stages run in the reverse order of the forward
// ones (len = 1, 2, ..., N/2). Stage with m = 2^s blocks (s from LOGN-1 down
// to 0) pairs j and j + (N >> (s+1)) in block j >> (LOGN - s) with twiddle
// psi^-brv(m + block). Passes are the forward passes taken in reverse.
template <int LOGN, int LOGT, int E_LOG, int S0, int EP, bool LAST, bool LAZY>
__device__ __forceinline__ void inv_pass(uint32_t (&x)[1 << E_LOG], const uint32_t *__restrict__ tw,
                                         const LimbConst &lc, uint32_t tid) {
    constexpr int GE = 1 << EP;
    constexpr int NG = (1 << E_LOG) >> EP;
    constexpr uint32_t OSPAN = 1u << (LOGN - S0 - EP);
    const uint32_t q = lc.q, qn = lc.qinv_neg;
#pragma unroll
    for (int kg = 0; kg < NG; kg++) {
        const uint32_t gi = tid + (uint32_t)kg * (1u << LOGT);
        const uint32_t b = (S0 == 0) ? 0u : gi / OSPAN;
#pragma unroll
        for (int u = EP - 1; u >= 0; u--) {
            const int half = GE >> (u + 1);
#pragma unroll
            for (int r = 0; r < GE; r++) {
                if (r & half) continue;
                uint32_t &lo = x[kg * GE + r];
                uint32_t &hi = x[kg * GE + r + half];
                if (LAST && S0 + u == 0) {
                    // last stage (one block, twiddle psi^-brv(1)): fold N^{-1}
                    // into both outputs and leave them canonical
                    // (any input below 2^32 is valid: s, d < 4q)
                    const uint32_t s = lo + hi;
                    const uint32_t d = lo - hi + (LAZY ? 2 * q : q);
                    lo = csub(mont_mul(s, lc.ninv_m, q, qn), q);
                    hi = csub(mont_mul(d, lc.w1n_m, q, qn), q);
                } else {
                    const uint32_t widx = (1u << (S0 + u)) + (b << u) + ((uint32_t)r >> (EP - u));
                    gs_bfly<LAZY>(lo, hi, tw[widx], q, qn);
                }
            }
        }
    }
}

// Inverse transform in two parts. inv_front: from the first pass's registers
// (loaded by load_runs: the first inverse pass is the forward's last, over
// runs of consecutive residues) through every pass but the last, ending with
// the last pass's residues in registers. inv_back: the last pass (uniform
// twiddles, scalar loads; the N^{-1} factor) and the coalesced store.
template <int LOGN, int LOGT, int E0, int E1, int E2, int E3, bool LAZY>
__device__ __forceinline__ void inv_front(uint32_t (&x)[1 << (LOGN - LOGT)], const uint32_t *__restrict__ tw,
                                          const LimbConst &lc, uint32_t *lds, uint32_t tid) {
    constexpr int E_LOG = LOGN - LOGT;
    static_assert(E0 + E1 + E2 + E3 == LOGN, "schedule must cover every stage");
    // barriers only where an exchange crosses waves (see fwd_front)
    constexpr bool X1 = exchange_in_wave<LOGN, LOGT, 0, E0, E0, E1>();
    constexpr bool X2 = exchange_in_wave<LOGN, LOGT, E0, E1, E0 + E1, E2>();
    constexpr bool X3 = exchange_in_wave<LOGN, LOGT, E0 + E1, E2, E0 + E1 + E2, E3>();
    if constexpr (E3 > 0) {
        inv_pass<LOGN, LOGT, E_LOG, E0 + E1 + E2, E3, false, LAZY>(x, tw, lc, tid);
        to_lds<LOGN, LOGT, E_LOG, E0 + E1 + E2, E3>(x, lds, tid);
        exchange_sync<X3>();
        from_lds<LOGN, LOGT, E_LOG, E0 + E1, E2>(x, lds, tid);
    }
    inv_pass<LOGN, LOGT, E_LOG, E0 + E1, E2, false, LAZY>(x, tw, lc, tid);
    if constexpr (E3 > 0) wave_lds_sync();
    to_lds<LOGN, LOGT, E_LOG, E0 + E1, E2>(x, lds, tid);
    exchange_sync<X2>();
    from_lds<LOGN, LOGT, E_LOG, E0, E1>(x, lds, tid);
    inv_pass<LOGN, LOGT, E_LOG, E0, E1, false, LAZY>(x, tw, lc, tid);
    wave_lds_sync();
    to_lds<LOGN, LOGT, E_LOG, E0, E1>(x, lds, tid);
    exchange_sync<X1>();
    from_lds<LOGN, LOGT, E_LOG, 0, E0>(x, lds, tid);
}

template <int LOGN, int LOGT, int E0, bool LAZY>
__device__ __forceinline__ void inv_back(uint32_t (&x)[1 << (LOGN - LOGT)], uint32_t *__restrict__ a,
                                         const uint32_t *__restrict__ tw, const LimbConst &lc, uint32_t tid) {
    constexpr int E_LOG = LOGN - LOGT;
    constexpr int T = 1 << LOGT, E = 1 << E_LOG;
    inv_pass<LOGN, LOGT, E_LOG, 0, E0, true, LAZY>(x, tw, lc, tid);
#pragma unroll
    for (int r = 0; r < E; r++) a[tid + r * T] = x[r];
}

template <int LOGN, int LOGT, int E0, int E1, int E2, int E3, bool LAZY>
__device__ __forceinline__ void ntt_inv_body(uint32_t *__restrict__ a, const uint32_t *__restrict__ tw,
                                             const LimbConst &lc, uint32_t *lds) {
    constexpr int E_LOG = LOGN - LOGT;
    const uint32_t tid = threadIdx.x;
    uint32_t x[1 << E_LOG];
    load_runs<LOGT, E_LOG, (E3 > 0 ? E3 : E2)>(x, a, tid);
    inv_front<LOGN, LOGT, E0, E1, E2, E3, LAZY>(x, tw, lc, lds, tid);
    inv_back<LOGN, LOGT, E0, LAZY>(x, a, tw, lc, tid);
}

// Polynomial p of a launch: a contiguous [P][L][N] array (segments == 1) or
// the concatenation of several such arrays (one per layer of a batch).
struct NttSegs {
    uint32_t *ptr[HYENA_MAX_SEGS];
    uint32_t first[HYENA_MAX_SEGS + 1];  // prefix sums of limb-polynomial counts
    uint32_t n;
};

// Waves per SIMD that the LDS footprint allows (160 KiB per CU): the register
// budget the compiler may use without costing occupancy.
constexpr int ntt_waves_per_simd(int logn, int logt) {
    const int blocks = (160 * 1024) / (((1 << logn) + (1 << logn) / 32) * 4);
    const int w = blocks * ((1 << logt) / 64) / 4;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

template <int LOGN, int LOGT, int E0, int E1, int E2, int E3, bool LAZY, bool INV>
__global__ void __launch_bounds__(1 << LOGT) __attribute__((amdgpu_waves_per_eu(1, ntt_waves_per_simd(LOGN, LOGT))))
ntt_kernel(NttSegs sg, const uint32_t *__restrict__ tw_all, LimbTable lt, uint32_t L) {
    constexpr int N = 1 << LOGN;
    __shared__ uint32_t lds[N + N / 32];
    // blocks of one segment hold limb-polynomials in [P][L][N] order; every
    // segment starts at limb 0, so the limb is the block's index within it mod L
    uint32_t s = 0;
    while (s + 1 < sg.n && blockIdx.x >= sg.first[s + 1]) s++;
    const uint32_t local = blockIdx.x - sg.first[s];
    uint32_t *a = sg.ptr[s] + (size_t)local * N;
    const uint32_t limb = local % L;
    const uint32_t *tw = tw_all + (size_t)limb * N;
    if (INV) ntt_inv_body<LOGN, LOGT, E0, E1, E2, E3, LAZY>(a, tw, lt.c[limb], lds);
    else ntt_fwd_body<LOGN, LOGT, E0, E1, E2, E3, LAZY>(a, tw, lt.c[limb].q, lt.c[limb].qinv_neg, lds);
}

// x <- x . NTT(s) mod q, canonical, in the runs layout the forward transform
// ends in (group kg of thread tid: residues [(tid + kg T) 2^EF, + 2^EF));
// mul holds NTT(s) of the limb in Montgomery form, read 16 bytes at a time.
template <int LOGT, int E_LOG, int EF>
__device__ __forceinline__ void mul_runs(uint32_t (&x)[1 << E_LOG], const uint32_t *__restrict__ mul, uint32_t q,
                                         uint32_t qn, uint32_t tid) {
    constexpr int GE = 1 << EF, NG = (1 << E_LOG) >> EF;
    static_assert(GE >= 4, "16-byte loads of NTT(s) in the runs layout");
#pragma unroll
    for (int kg = 0; kg < NG; kg++) {
        const uint32_t *m = mul + ((size_t)(tid + (uint32_t)kg * (1u << LOGT)) << EF);
        uint32_t *xv = &x[kg * GE];
#pragma unroll
        for (int j = 0; j < GE; j += 4) {
            const uint4 u = *reinterpret_cast<const uint4 *>(m + j);
            xv[j] = csub(mont_mul(xv[j], u.x, q, qn), q);
            xv[j + 1] = csub(mont_mul(xv[j + 1], u.y, q, qn), q);
            xv[j + 2] = csub(mont_mul(xv[j + 2], u.z, q, qn), q);
            xv[j + 3] = csub(mont_mul(xv[j + 3], u.w, q, qn), q);
        }
    }
}

// Encryption's a s, with a drawn in the load: block p (limb p mod L of
// message p / L) takes a_j = floor(q sm64(seed, 2 (p N + j)) / 2^64), writes
// c1 = -a of that ciphertext ([n][2][L][N]), transforms a, multiplies by
// NTT(s) (mul [L][N], Montgomery form) in the runs layout the forward
// transform ends in and the inverse starts from, transforms back and stores
// a s mod q into dst [n][L][N]; the product never leaves the chip.
template <int LOGN, int LOGT, int E0, int E1, int E2, int E3, bool LAZY>
__global__ void __launch_bounds__(1 << LOGT) __attribute__((amdgpu_waves_per_eu(1, ntt_waves_per_simd(LOGN, LOGT))))
ntt_sample_as_kernel(uint32_t *ct, uint32_t *dst, const uint32_t *__restrict__ mul, uint64_t seed,
                     const uint32_t *__restrict__ fw_all, const uint32_t *__restrict__ iw_all, LimbTable lt,
                     uint32_t L) {
    constexpr int N = 1 << LOGN, T = 1 << LOGT, E_LOG = LOGN - LOGT, E = 1 << E_LOG;
    constexpr int EF = E3 > 0 ? E3 : E2;
    __shared__ uint32_t lds[N + N / 32];
    const uint32_t p = blockIdx.x, limb = p % L, m = p / L, tid = threadIdx.x;
    const size_t LN = (size_t)L * N;
    uint32_t *c1 = ct + (size_t)m * 2 * LN + LN + (size_t)limb * N;
    const LimbConst lc = lt.c[limb];
    const uint32_t q = lc.q, qn = lc.qinv_neg;
    uint32_t x[E];
#pragma unroll
    for (int r = 0; r < E; r++) {
        const uint32_t j = tid + r * T;
        const uint32_t a = (uint32_t)__umul64hi(hy_sm64(seed, 2 * ((uint64_t)p * N + j)), (uint64_t)q);
        x[r] = a;
        c1[j] = a ? q - a : 0;
    }
    fwd_front<LOGN, LOGT, E0, E1, E2, E3, LAZY>(x, fw_all + (size_t)limb * N, q, qn, lds, tid);
    const uint32_t *sh = mul + (size_t)limb * N;
    mul_runs<LOGT, E_LOG, EF>(x, sh, q, qn, tid);
    __syncthreads();   // every wave's reads of the forward exchanges are done
    const uint32_t *iw = iw_all + (size_t)limb * N;
    inv_front<LOGN, LOGT, E0, E1, E2, E3, LAZY>(x, iw, lc, lds, tid);
    inv_back<LOGN, LOGT, E0, LAZY>(x, dst + (size_t)p * N, iw, lc, tid);
}

template <int LOGN, int LOGT, int E0, int E1, int E2, int E3>
hipError_t launch_sample_as(const hyena_ctx *c, uint32_t *ct, size_t n, uint32_t *dst, const uint32_t *mul,
                            uint64_t seed, hipStream_t s) {
    const dim3 grid((unsigned)(n * c->L)), block(1u << LOGT);
    if (c->lazy_ntt)
        hipLaunchKernelGGL((ntt_sample_as_kernel<LOGN, LOGT, E0, E1, E2, E3, true>), grid, block, 0, s, ct, dst, mul,
                           seed, c->d_fw, c->d_iw, c->lt, c->L);
    else
        hipLaunchKernelGGL((ntt_sample_as_kernel<LOGN, LOGT, E0, E1, E2, E3, false>), grid, block, 0, s, ct, dst,
                           mul, seed, c->d_fw, c->d_iw, c->lt, c->L);
    return hipGetLastError();
}


// Decryption's c0 + c1 s in one pass over each limb-polynomial: block p
// (limb p mod L of ciphertext p / L of ct [n][2][L][N]) transforms c1 (the
// forward passes), multiplies by NTT(s) (mul [L][N], Montgomery form) in the
// runs layout the forward transform ends in and the inverse starts from,
// transforms back and stores INTT(NTT(c1) . NTT(s)) + c0 mod q into
// v [n][L][N]; the product never leaves the chip.
template <int LOGN, int LOGT, int E0, int E1, int E2, int E3, bool LAZY>
__global__ void __launch_bounds__(1 << LOGT) __attribute__((amdgpu_waves_per_eu(1, ntt_waves_per_simd(LOGN, LOGT))))
ntt_c1s_add_kernel(const uint32_t *__restrict__ ct, uint32_t *__restrict__ v, const uint32_t *__restrict__ mul,
                   const uint32_t *__restrict__ fw_all, const uint32_t *__restrict__ iw_all, LimbTable lt,
                   uint32_t L) {
    constexpr int N = 1 << LOGN, T = 1 << LOGT, E_LOG = LOGN - LOGT, E = 1 << E_LOG;
    constexpr int EF = E3 > 0 ? E3 : E2;
    __shared__ uint32_t lds[N + N / 32];
    const uint32_t p = blockIdx.x, limb = p % L, m = p / L, tid = threadIdx.x;
    const size_t LN = (size_t)L * N;
    const uint32_t *c0 = ct + (size_t)m * 2 * LN + (size_t)limb * N, *c1 = c0 + LN;
    const LimbConst lc = lt.c[limb];
    const uint32_t q = lc.q, qn = lc.qinv_neg;
    uint32_t x[E];
#pragma unroll
    for (int r = 0; r < E; r++) x[r] = c1[tid + r * T];
    fwd_front<LOGN, LOGT, E0, E1, E2, E3, LAZY>(x, fw_all + (size_t)limb * N, q, qn, lds, tid);
    const uint32_t *sh = mul + (size_t)limb * N;
    mul_runs<LOGT, E_LOG, EF>(x, sh, q, qn, tid);
    __syncthreads();   // every wave's reads of the forward exchanges are done
    const uint32_t *iw = iw_all + (size_t)limb * N;
    inv_front<LOGN, LOGT, E0, E1, E2, E3, LAZY>(x, iw, lc, lds, tid);
    inv_pass<LOGN, LOGT, E_LOG, 0, E0, true, LAZY>(x, iw, lc, tid);
    uint32_t *o = v + (size_t)p * N;
#pragma unroll
    for (int r = 0; r < E; r++) o[tid + r * T] = csub(x[r] + c0[tid + r * T], q);
}

template <int LOGN, int LOGT, int E0, int E1, int E2, int E3>
hipError_t launch_c1s_add(const hyena_ctx *c, const uint32_t *ct, size_t n, uint32_t *v, const uint32_t *mul,
                          hipStream_t s) {
    const dim3 grid((unsigned)(n * c->L)), block(1u << LOGT);
    if (c->lazy_ntt)
        hipLaunchKernelGGL((ntt_c1s_add_kernel<LOGN, LOGT, E0, E1, E2, E3, true>), grid, block, 0, s, ct, v, mul,
                           c->d_fw, c->d_iw, c->lt, c->L);
    else
        hipLaunchKernelGGL((ntt_c1s_add_kernel<LOGN, LOGT, E0, E1, E2, E3, false>), grid, block, 0, s, ct, v, mul,
                           c->d_fw, c->d_iw, c->lt, c->L);
    return hipGetLastError();
}

// Persistent inverse transform: a grid of a few blocks per CU (a multiple of
// L, so a block keeps one limb); block b transforms limb-polynomials b,
// b + grid, ... and loads the next one's first-pass residues into registers
// while it runs the current one's last pass and store. The last pass reads
// only uniform (scalar) twiddles, so no vector-memory wait in it has to cover
// the prefetch; the wait comes when the next polynomial starts.
__device__ __forceinline__ uint32_t *seg_poly(const NttSegs &sg, uint32_t &s, uint32_t p, uint32_t N) {
    while (s + 1 < sg.n && p >= sg.first[s + 1]) s++;
    return sg.ptr[s] + (size_t)(p - sg.first[s]) * N;
}

template <int LOGN, int LOGT, int E0, int E1, int E2, int E3, bool LAZY>
__global__ void __launch_bounds__(1 << LOGT) __attribute__((amdgpu_waves_per_eu(1, ntt_waves_per_simd(LOGN, LOGT))))
ntt_inv_persist_kernel(NttSegs sg, const uint32_t *__restrict__ tw_all, LimbTable lt, uint32_t L) {
    constexpr int N = 1 << LOGN, E_LOG = LOGN - LOGT, E = 1 << E_LOG;
    constexpr int EF = E3 > 0 ? E3 : E2;
    __shared__ uint32_t lds[N + N / 32];
    const uint32_t tid = threadIdx.x, total = sg.first[sg.n];
    uint32_t p = blockIdx.x, s = 0;
    if (p >= total) return;
    uint32_t x[E], nx[E];
    load_runs<LOGT, E_LOG, EF>(nx, seg_poly(sg, s, p, N), tid);
    for (;;) {
        // every segment starts at limb 0, so the limb is p mod L; looked up
        // per polynomial so that the twiddle loads stay in the loop rather
        // than holding registers across it
        const uint32_t limb = __builtin_amdgcn_readfirstlane(p % L);
        const uint32_t *tw = tw_all + (size_t)limb * N;
        const LimbConst lc = lt.c[limb];
        uint32_t *a = sg.ptr[s] + (size_t)(p - sg.first[s]) * N;
#pragma unroll
        for (int r = 0; r < E; r++) x[r] = nx[r];
        const uint32_t pn = p + gridDim.x;
        inv_front<LOGN, LOGT, E0, E1, E2, E3, LAZY>(x, tw, lc, lds, tid);
        if (pn < total) load_runs<LOGT, E_LOG, EF>(nx, seg_poly(sg, s, pn, N), tid);
        inv_back<LOGN, LOGT, E0, LAZY>(x, a, tw, lc, tid);
        if (pn >= total) break;
        p = pn;
        __syncthreads();  // the last pass's LDS reads precede the next exchange
    }
}

// Streaming transform (either direction): a persistent grid whose size is a
// multiple of L, so every block keeps one limb. The block copies that limb's
// twiddles into LDS once; the passes then read twiddles from LDS (counted on
// lgkmcnt), so the only vector-memory traffic is the polynomials themselves
// and the next polynomial's residues can be loaded into registers as soon as
// the current one's have arrived: its loads overlap the whole transform of the
// current one, not only its last pass.
template <int LOGN, int LOGT, int E0, int E1, int E2, int E3, bool LAZY, bool INV>
__global__ void __launch_bounds__(1 << LOGT)
ntt_stream_kernel(NttSegs sg, const uint32_t *__restrict__ tw_all, LimbTable lt, uint32_t L) {
    constexpr int N = 1 << LOGN, E_LOG = LOGN - LOGT, T = 1 << LOGT, E = 1 << E_LOG;
    constexpr int EF = E3 > 0 ? E3 : E2;   // the pass over the last (forward) stages
    __shared__ uint32_t lds[N + N / 32];
    __shared__ uint32_t tws[N];
    const uint32_t tid = threadIdx.x, total = sg.first[sg.n];
    uint32_t p = blockIdx.x, s = 0;
    if (p >= total) return;
    // every segment starts at limb 0 and the grid is a multiple of L (or covers
    // every polynomial in one round), so p mod L is the same for all of this
    // block's polynomials
    const uint32_t limb = __builtin_amdgcn_readfirstlane(p % L);
    const uint32_t *tw = tw_all + (size_t)limb * N;
    for (int i = tid; i < N; i += T) tws[i] = tw[i];
    const LimbConst lc = lt.c[limb];
    uint32_t x[E], nx[E];
    auto load = [&](uint32_t (&v)[E], const uint32_t *a) {
        if (INV) {
            load_runs<LOGT, E_LOG, EF>(v, a, tid);
        } else {
#pragma unroll
            for (int r = 0; r < E; r++) v[r] = a[tid + r * T];
        }
    };
    load(nx, seg_poly(sg, s, p, N));
    __syncthreads();   // twiddles in LDS
    for (;;) {
        uint32_t *a = sg.ptr[s] + (size_t)(p - sg.first[s]) * N;
#pragma unroll
        for (int r = 0; r < E; r++) x[r] = nx[r];
        const uint32_t pn = p + gridDim.x;
        if (pn < total) load(nx, seg_poly(sg, s, pn, N));   // s now refers to pn
        if (INV) {
            inv_front<LOGN, LOGT, E0, E1, E2, E3, LAZY>(x, tws, lc, lds, tid);
            inv_back<LOGN, LOGT, E0, LAZY>(x, a, tws, lc, tid);
        } else {
            fwd_front<LOGN, LOGT, E0, E1, E2, E3, LAZY>(x, tws, lc.q, lc.qinv_neg, lds, tid);
            store_runs<LOGT, E_LOG, EF>(x, a, tid);
        }
        if (pn >= total) break;
        p = pn;
        __syncthreads();  // this polynomial's LDS reads precede the next one's exchange
    }
}

template <int LOGN, int LOGT, int E0, int E1, int E2, int E3>
hipError_t launch_sched(const NttSegs &sg, const hyena_ctx *c, bool inv, hipStream_t s) {
    const dim3 grid(sg.first[sg.n]), block(1u << LOGT);
    const uint32_t *tw = inv ? c->d_iw : c->d_fw;
    if (c->lazy_ntt) {  // Harvey's lazy butterflies need 4q < 2^32
        if (inv) hipLaunchKernelGGL((ntt_kernel<LOGN, LOGT, E0, E1, E2, E3, true, true>), grid, block, 0, s, sg, tw, c->lt, c->L);
        else hipLaunchKernelGGL((ntt_kernel<LOGN, LOGT, E0, E1, E2, E3, true, false>), grid, block, 0, s, sg, tw, c->lt, c->L);
    } else {
        if (inv) hipLaunchKernelGGL((ntt_kernel<LOGN, LOGT, E0, E1, E2, E3, false, true>), grid, block, 0, s, sg, tw, c->lt, c->L);
        else hipLaunchKernelGGL((ntt_kernel<LOGN, LOGT, E0, E1, E2, E3, false, false>), grid, block, 0, s, sg, tw, c->lt, c->L);
    }
    return hipGetLastError();
}

// Persistent schedule: forward transforms as launch_sched; inverse ones with
// ntt_inv_persist_kernel on a grid of as many blocks as fit on the chip.
template <int LOGN, int LOGT, int E0, int E1, int E2, int E3>
hipError_t launch_persist(const NttSegs &sg, const hyena_ctx *c, bool inv, hipStream_t s) {
    if (!inv) return launch_sched<LOGN, LOGT, E0, E1, E2, E3>(sg, c, false, s);
    const auto kern = c->lazy_ntt ? ntt_inv_persist_kernel<LOGN, LOGT, E0, E1, E2, E3, true>
                                  : ntt_inv_persist_kernel<LOGN, LOGT, E0, E1, E2, E3, false>;
    int n_cu = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, 1 << LOGT, 0);
    if (e != hipSuccess) return e;
    const uint32_t total = sg.first[sg.n];
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(total, (uint32_t)std::max(1, per_cu) * n_cu));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(1u << LOGT), 0, s, sg, inv ? c->d_iw : c->d_fw, c->lt, c->L);
    return hipGetLastError();
}

// Streaming schedule: both directions with ntt_stream_kernel on as many
// blocks as fit on the chip, rounded down to a multiple of L (one limb per
// block), or one block per polynomial when there are fewer.
template <int LOGN, int LOGT, int E0, int E1, int E2, int E3>
hipError_t launch_stream(const NttSegs &sg, const hyena_ctx *c, bool inv, hipStream_t s) {
    void (*kern)(NttSegs, const uint32_t *, LimbTable, uint32_t);
    if (c->lazy_ntt) kern = inv ? ntt_stream_kernel<LOGN, LOGT, E0, E1, E2, E3, true, true>
                                : ntt_stream_kernel<LOGN, LOGT, E0, E1, E2, E3, true, false>;
    else kern = inv ? ntt_stream_kernel<LOGN, LOGT, E0, E1, E2, E3, false, true>
                    : ntt_stream_kernel<LOGN, LOGT, E0, E1, E2, E3, false, false>;
    int n_cu = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, 1 << LOGT, 0);
    if (e != hipSuccess) return e;
    const uint32_t total = sg.first[sg.n], fit = (uint32_t)std::max(1, per_cu) * (uint32_t)n_cu;
    const uint32_t grid = total <= fit ? total : std::max<uint32_t>(c->L, fit / c->L * c->L);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(1u << LOGT), 0, s, sg, inv ? c->d_iw : c->d_fw, c->lt, c->L);
    return hipGetLastError();
}

// NTT schedules per ring degree: threads per polynomial, stages per pass and
// how the launch runs: 0 one block per limb-polynomial, 1 persistent inverse
// (next polynomial prefetched during the last pass), 2 streaming, both
// directions (twiddles in LDS, next polynomial prefetched for the whole
// transform).
struct NttSched {
    int logn, logt, e0, e1, e2, e3, persist;
};
const NttSched kNtt[] = {
    {10, 6, 4, 3, 3, 0, 0},
    {11, 7, 4, 4, 3, 0, 0}, {11, 6, 5, 3, 3, 0, 0}, {11, 6, 5, 5, 1, 0, 0},
    {12, 8, 4, 4, 4, 0, 0}, {12, 7, 5, 5, 2, 0, 0}, {12, 6, 6, 3, 3, 0, 0},
    {12, 8, 4, 4, 4, 0, 1}, {12, 7, 5, 5, 2, 0, 1}, {12, 8, 4, 4, 4, 0, 2}, {12, 7, 5, 5, 2, 0, 2},
    {13, 8, 5, 4, 4, 0, 0}, {13, 9, 4, 4, 4, 1, 0}, {13, 7, 6, 6, 1, 0, 0},
    {13, 8, 5, 4, 4, 0, 1}, {13, 9, 4, 4, 4, 1, 1}, {13, 8, 5, 4, 4, 0, 2}, {13, 9, 4, 4, 4, 1, 2},
    {14, 9, 5, 5, 4, 0, 0}, {14, 10, 4, 4, 4, 2, 0}, {14, 8, 6, 6, 2, 0, 0},
    {14, 9, 5, 5, 4, 0, 1}, {14, 10, 4, 4, 4, 2, 1}, {14, 9, 5, 5, 4, 0, 2}, {14, 10, 4, 4, 4, 2, 2},
};
const int kNumNtt = sizeof(kNtt) / sizeof(kNtt[0]);

hipError_t launch_idx(int i, const NttSegs &d, const hyena_ctx *c, bool inv, hipStream_t s) {
    switch (i) {
        case 0: return launch_sched<10, 6, 4, 3, 3, 0>(d, c, inv, s);
        case 1: return launch_sched<11, 7, 4, 4, 3, 0>(d, c, inv, s);
        case 2: return launch_sched<11, 6, 5, 3, 3, 0>(d, c, inv, s);
        case 3: return launch_sched<11, 6, 5, 5, 1, 0>(d, c, inv, s);
        case 4: return launch_sched<12, 8, 4, 4, 4, 0>(d, c, inv, s);
        case 5: return launch_sched<12, 7, 5, 5, 2, 0>(d, c, inv, s);
        case 6: return launch_sched<12, 6, 6, 3, 3, 0>(d, c, inv, s);
        case 7: return launch_persist<12, 8, 4, 4, 4, 0>(d, c, inv, s);
        case 8: return launch_persist<12, 7, 5, 5, 2, 0>(d, c, inv, s);
        case 9: return launch_stream<12, 8, 4, 4, 4, 0>(d, c, inv, s);
        case 10: return launch_stream<12, 7, 5, 5, 2, 0>(d, c, inv, s);
        case 11: return launch_sched<13, 8, 5, 4, 4, 0>(d, c, inv, s);
        case 12: return launch_sched<13, 9, 4, 4, 4, 1>(d, c, inv, s);
        case 13: return launch_sched<13, 7, 6, 6, 1, 0>(d, c, inv, s);
        case 14: return launch_persist<13, 8, 5, 4, 4, 0>(d, c, inv, s);
        case 15: return launch_persist<13, 9, 4, 4, 4, 1>(d, c, inv, s);
        case 16: return launch_stream<13, 8, 5, 4, 4, 0>(d, c, inv, s);
        case 17: return launch_stream<13, 9, 4, 4, 4, 1>(d, c, inv, s);
        case 18: return launch_sched<14, 9, 5, 5, 4, 0>(d, c, inv, s);
        case 19: return launch_sched<14, 10, 4, 4, 4, 2>(d, c, inv, s);
        case 20: return launch_sched<14, 8, 6, 6, 2, 0>(d, c, inv, s);
        case 21: return launch_persist<14, 9, 5, 5, 4, 0>(d, c, inv, s);
        case 22: return launch_persist<14, 10, 4, 4, 4, 2>(d, c, inv, s);
        case 23: return launch_stream<14, 9, 5, 5, 4, 0>(d, c, inv, s);
        case 24: return launch_stream<14, 10, 4, 4, 4, 2>(d, c, inv, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int ntt_default_schedule(uint32_t logN) {
    switch (logN) {
        case 10: return 0;
        case 11: return 1;
        case 12: return 4;
        case 13: return 11;
        case 14: return 19;
        default: return -1;
    }
}

int launch_ntt_segs(const hyena_ctx *c, uint32_t *const *ptrs, const size_t *P, uint32_t nseg, bool inv,
                    int sched, hipStream_t s) {
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_ntt: context was created host-only");
    for (uint32_t i = 0; i < nseg; i++)
        if (P[i] && ((uintptr_t)ptrs[i] & 15u))
            return set_error(HYENA_EINVAL, "hyena_ntt: polynomial array is not 16-byte aligned");
    if (sched < 0) sched = ntt_default_schedule(c->logN);
    if (sched < 0 || sched >= kNumNtt || kNtt[sched].logn != (int)c->logN)
        return set_error(HYENA_EINVAL, "hyena_ntt: schedule does not exist for this N");
    // launches of at most HYENA_MAX_SEGS segments and 2^31 blocks each
    uint32_t i = 0;
    while (i < nseg) {
        NttSegs sg{};
        uint64_t total = 0;
        while (i < nseg && sg.n < HYENA_MAX_SEGS) {
            const uint64_t blocks = (uint64_t)P[i] * c->L;
            if (blocks == 0) { i++; continue; }
            if (total + blocks > 0x7fffffffull) {
                if (sg.n == 0) return set_error(HYENA_EINVAL, "hyena_ntt: too many polynomials");
                break;
            }
            if (!ptrs[i]) return set_error(HYENA_EINVAL, "hyena_ntt: NULL polynomial array");
            sg.ptr[sg.n] = ptrs[i];
            sg.first[sg.n] = (uint32_t)total;
            total += blocks;
            sg.n++;
            i++;
        }
        if (sg.n == 0) break;
        sg.first[sg.n] = (uint32_t)total;
        const hipError_t e = launch_idx(sched, sg, c, inv, s);
        if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_ntt: ") + hipGetErrorString(e));
    }
    return HYENA_OK;
}

int launch_ntt_sched(const hyena_ctx *c, uint32_t *d, size_t P, bool inv, int sched, hipStream_t s) {
    return launch_ntt_segs(c, &d, &P, 1, inv, sched, s);
}

int launch_ntt(const hyena_ctx *c, uint32_t *d, size_t P, bool inv, hipStream_t s) {
    return launch_ntt_sched(c, d, P, inv, -1, s);
}

int launch_ntt_sample_as(const hyena_ctx *c, uint32_t *ct, size_t n, uint32_t *dst, const uint32_t *mul,
                          uint64_t seed, hipStream_t s) {
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_ntt: context was created host-only");
    if (n == 0) return HYENA_OK;
    if (n * c->L > 0x7fffffffull) return set_error(HYENA_EINVAL, "hyena_ntt: too many polynomials");
    if (((uintptr_t)dst | (uintptr_t)mul) & 15u)
        return set_error(HYENA_EINVAL, "hyena_ntt: polynomial array is not 16-byte aligned");
    hipError_t e;
    switch (c->logN) {
        case 10: e = launch_sample_as<10, 6, 4, 3, 3, 0>(c, ct, n, dst, mul, seed, s); break;
        case 11: e = launch_sample_as<11, 7, 4, 4, 3, 0>(c, ct, n, dst, mul, seed, s); break;
        case 12: e = launch_sample_as<12, 8, 4, 4, 4, 0>(c, ct, n, dst, mul, seed, s); break;
        case 13: e = launch_sample_as<13, 8, 5, 4, 4, 0>(c, ct, n, dst, mul, seed, s); break;
        case 14: e = launch_sample_as<14, 10, 4, 4, 4, 2>(c, ct, n, dst, mul, seed, s); break;
        default: return set_error(HYENA_EUNSUPPORTED, "hyena_ntt: unsupported N");
    }
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_ntt: ") + hipGetErrorString(e));
    return HYENA_OK;
}

int launch_ntt_c1s_add(const hyena_ctx *c, const uint32_t *ct, size_t n, uint32_t *v, const uint32_t *mul,
                       hipStream_t s) {
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_ntt: context was created host-only");
    if (n == 0) return HYENA_OK;
    if (n * c->L > 0x7fffffffull) return set_error(HYENA_EINVAL, "hyena_ntt: too many polynomials");
    if ((uintptr_t)mul & 15u) return set_error(HYENA_EINVAL, "hyena_ntt: polynomial array is not 16-byte aligned");
    hipError_t e;
    switch (c->logN) {   // the default schedule of each N (one block per limb-polynomial)
        case 10: e = launch_c1s_add<10, 6, 4, 3, 3, 0>(c, ct, n, v, mul, s); break;
        case 11: e = launch_c1s_add<11, 7, 4, 4, 3, 0>(c, ct, n, v, mul, s); break;
        case 12: e = launch_c1s_add<12, 8, 4, 4, 4, 0>(c, ct, n, v, mul, s); break;
        case 13: e = launch_c1s_add<13, 8, 5, 4, 4, 0>(c, ct, n, v, mul, s); break;
        case 14: e = launch_c1s_add<14, 10, 4, 4, 4, 2>(c, ct, n, v, mul, s); break;
        default: return set_error(HYENA_EUNSUPPORTED, "hyena_ntt: unsupported N");
    }
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_ntt: ") + hipGetErrorString(e));
    return HYENA_OK;
}

extern "C" int hyena_ntt_schedules(uint32_t N, int *first, int *count) {
    int f = -1, n = 0;
    for (int i = 0; i < kNumNtt; i++)
        if ((1u << kNtt[i].logn) == N) {
            if (f < 0) f = i;
            n++;
        }
    if (first) *first = f;
    if (count) *count = n;
    return n ? HYENA_OK : set_error(HYENA_EUNSUPPORTED, "hyena_ntt_schedules: unsupported N");
}

extern "C" int hyena_ntt_sched(const hyena_ctx *c, uint32_t *d_poly, size_t P, int inverse, int sched,
                               hyena_stream_t s) {
    if (!c || (P && !d_poly)) return set_error(HYENA_EINVAL, "hyena_ntt_sched: NULL argument");
    return launch_ntt_sched(c, d_poly, P, inverse != 0, sched, (hipStream_t)s);
}

extern "C" int hyena_ntt(const hyena_ctx *c, uint32_t *d_poly, size_t P, hyena_stream_t s) {
    if (!c || (P && !d_poly)) return set_error(HYENA_EINVAL, "hyena_ntt: NULL argument");
    return launch_ntt(c, d_poly, P, false, (hipStream_t)s);
}

extern "C" int hyena_intt(const hyena_ctx *c, uint32_t *d_poly, size_t P, hyena_stream_t s) {
    if (!c || (P && !d_poly)) return set_error(HYENA_EINVAL, "hyena_intt: NULL argument");
    return launch_ntt(c, d_poly, P, true, (hipStream_t)s);
}
