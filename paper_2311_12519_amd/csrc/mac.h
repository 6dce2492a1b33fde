// Multiply-accumulate building blocks shared by the per-layer launches and
// the persistent batched kernel (device code; included by conv.hip and
// batch.hip only).
#pragma once
#include <type_traits>

#include "internal.h"

// Arguments of one layer's multiply-accumulate (also stored in device memory
// as the per-layer table of the persistent kernel).
constexpr int kSynthTapsMax = 18;   // taps per weight word a synthesizing schedule can take

struct MacArgs {
    const uint32_t *ct;   // [rows/2][n_groups][2][L][N]
    const uint32_t *w;    // [Co][w_groups][L][N] (schedules that stream the NTT-domain weights)
    uint32_t *out;        // [rows/2][Co][2][L][N]
    uint32_t N, L, logN, Co, n_groups, w_groups, rows, ci, c_n;
    uint32_t depthwise, fuse, n_ot, n_mt, kchunks;
    // schedules that synthesize the weight words from the integer taps:
    // taps [Co][w_groups][T4] (Walsh-combined, tap t = c' k^2 + di k + dj),
    // texp[t] = O - c' Bt - di Wp - dj the exponent of tap t's monomial,
    // fw [L][N] the psi powers psi^brv(j) 2^32 mod q_i
    const int32_t *taps;
    const uint32_t *fw;
    uint32_t T, T4;
    uint32_t texp[kSynthTapsMax];
    uint32_t wscale[HYENA_MAX_LIMBS];   // c_n^{-1} 2^64 mod q_i
    LimbTable lt;
};

namespace {

__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t q) { return min(x, x - q); }

__device__ __forceinline__ uint64_t mad64(uint32_t a, uint32_t b, uint64_t c) {
    return (uint64_t)a * b + c;  // one v_mad_u64_u32
}

// Exact reduction of a 64-bit accumulator to [0, q), times 2^-32. The encoded
// weights carry a factor 2^32 (Montgomery form, applied once when they are
// encoded), so for acc = sum ct * (w 2^32) this returns sum ct * w mod q.
// FOLD = false when acc is already below q 2^32 (at most lc.nofold products
// since the last fold).
template <bool FOLD = true>
__device__ __forceinline__ uint32_t reduce64(uint64_t acc, const LimbConst &lc) {
    const uint32_t q = lc.q;
    const uint32_t hi = (uint32_t)(acc >> 32), lo = (uint32_t)acc;
    // y = hi * 2^32 + lo = hi * r32 + lo (mod q); with r32 = 2^32 mod q <= q - 1,
    // y <= (r32 + 1)(2^32 - 1) < q * 2^32, the range Montgomery reduction takes
    const uint64_t y = FOLD ? mad64(hi, lc.r32, lo) : acc;
    // Montgomery REDC: y * 2^-32 mod q in [0, 2q)
    const uint32_t m = (uint32_t)y * lc.qinv_neg;
    const uint64_t t = mad64(m, q, y);
    return csub((uint32_t)(t >> 32), q);
}

__device__ __forceinline__ uint64_t fold(uint64_t acc, uint32_t r32) {
    return mad64((uint32_t)(acc >> 32), r32, (uint32_t)acc);
}

// a b 2^-32 mod q in [0, q) for a, b < q
__device__ __forceinline__ uint32_t mont_mul_red(uint32_t a, uint32_t b, const LimbConst &lc) {
    const uint64_t t = (uint64_t)a * b;
    const uint32_t m = (uint32_t)t * lc.qinv_neg;
    return csub((uint32_t)(mad64(m, lc.q, t) >> 32), lc.q);
}




// LDS-pipelined multiply-accumulate. A block of 256 threads (4 waves in a
// WR x WO grid) owns 64 consecutive NTT slots of one limb (lane = slot) and a
// tile of MB = WR*MT rows by OB = WO*OT outputs; wave (wr, wo) accumulates
// rows [wr*MT, +MT) x outputs [wo*OT, +OT). For every input group g the MB
// ciphertext rows and OB weight rows of the block (64 words each) are copied
// global -> LDS with direct-to-LDS 16-byte loads, NS groups ahead of the
// arithmetic, so each word is fetched once per block and the copies need no
// registers. One barrier per group separates a stage's reads from its reuse.
__device__ __forceinline__ void wait_vm(int n) {
    // s_waitcnt with vmcnt = n (n <= 15 here), expcnt and lgkmcnt left at max
    switch (n) {
        case 0: __builtin_amdgcn_s_waitcnt(0x0F70); break;
        case 1: __builtin_amdgcn_s_waitcnt(0x0F71); break;
        case 2: __builtin_amdgcn_s_waitcnt(0x0F72); break;
        case 3: __builtin_amdgcn_s_waitcnt(0x0F73); break;
        case 4: __builtin_amdgcn_s_waitcnt(0x0F74); break;
        case 5: __builtin_amdgcn_s_waitcnt(0x0F75); break;
        case 6: __builtin_amdgcn_s_waitcnt(0x0F76); break;
        case 7: __builtin_amdgcn_s_waitcnt(0x0F77); break;
        case 8: __builtin_amdgcn_s_waitcnt(0x0F78); break;
        case 9: __builtin_amdgcn_s_waitcnt(0x0F79); break;
        case 10: __builtin_amdgcn_s_waitcnt(0x0F7A); break;
        case 11: __builtin_amdgcn_s_waitcnt(0x0F7B); break;
        case 12: __builtin_amdgcn_s_waitcnt(0x0F7C); break;
        default: __builtin_amdgcn_s_waitcnt(0x0F70); break;
    }
}

// LDS layout of one pipeline stage: the copied rows (MB ciphertext rows, and
// the OB weight rows when they are streamed) in whole loader rounds, then,
// when the weights are synthesized (TM > 0), the OB synthesized weight rows;
// and, for schedules with more than 9 taps, the per-slot tap powers.
template <int MT, int OT, int WR, int WO, int NS, int TM = 0>
struct MacLdsShape {
    static constexpr int MB = WR * MT, OB = WO * OT;
    static constexpr int ROWS = MB + (TM ? 0 : OB);  // copied rows
    static constexpr int RND = (ROWS + 15) / 16;   // loader rounds: 256 threads x 16 B = 16 rows
    static constexpr int PROWS = RND * 16;
    static constexpr int WB = TM ? PROWS : MB;      // first weight row of a stage
    static constexpr int SROWS = PROWS + (TM ? OB : 0);
    static constexpr bool VP_LDS = TM > 9;          // tap powers in LDS rather than registers
    static constexpr int LDS_WORDS = NS * SROWS * 64 + (VP_LDS ? TM * 64 : 0);
    // resident blocks per CU the launch asks for: three (at most 168 VGPRs
    // per thread) unless the LDS stages of fewer blocks already fill the
    // CU's 160 KiB (64 bytes spared for the persistent kernel's claim words)
    static constexpr int FIT = (160 * 1024) / (LDS_WORDS * 4 + 64);
    static constexpr int MIN_BLOCKS = FIT < 1 ? 1 : (FIT > 3 ? 3 : FIT);
};

struct NoHook {
    __device__ void operator()() const {}
};

// One logical block (64-slot chunk x row tile x output tile) of a layer.
// `after_loop` runs once the last group's products are accumulated, before
// the reduction and the stores (the persistent kernel claims its next work
// item there).
// s_waitcnt with vmcnt = n and lgkmcnt = 0: this wave's LDS writes (and
// scalar loads) complete as well
__device__ __forceinline__ void wait_vm_lgkm0(int n) {
    switch (n) {
        case 0: __builtin_amdgcn_s_waitcnt(0x0070); break;
        case 1: __builtin_amdgcn_s_waitcnt(0x0071); break;
        case 2: __builtin_amdgcn_s_waitcnt(0x0072); break;
        case 3: __builtin_amdgcn_s_waitcnt(0x0073); break;
        case 4: __builtin_amdgcn_s_waitcnt(0x0074); break;
        case 5: __builtin_amdgcn_s_waitcnt(0x0075); break;
        case 6: __builtin_amdgcn_s_waitcnt(0x0076); break;
        case 7: __builtin_amdgcn_s_waitcnt(0x0077); break;
        case 8: __builtin_amdgcn_s_waitcnt(0x0078); break;
        default: __builtin_amdgcn_s_waitcnt(0x0070); break;
    }
}

// Montgomery reduction of 0 <= y < q 2^32: y 2^-32 mod q in [0, q)
__device__ __forceinline__ uint32_t redc64(uint64_t y, const LimbConst &lc) {
    const uint32_t m = (uint32_t)y * lc.qinv_neg;
    return csub((uint32_t)(mad64(m, lc.q, y) >> 32), lc.q);
}

// One logical block (64-slot chunk x row tile x output tile) of a layer.
// `after_loop` runs once the last group's products are accumulated, before
// the reduction and the stores (the persistent kernel claims its next work
// item there).
//
// TM > 0: the weight words are not read but synthesized in the block from the
// integer taps (the cloud keeps the kernels as small integers, "Enabling
// Output Channel Packing"): the word of output o, input group g at NTT slot s
// is sum_t taps[o][g][t] V_t(s) with V_t(s) = c_n^{-1} 2^64 r_s^texp[t] mod q,
// r_s = psi^(2 brv(s) + 1), the value the NTT of the Walsh kernel polynomial
// takes there in Montgomery form (the form hyena_encode_weights stores). Each
// lane computes the T powers of its slot once per block; per group every
// wave synthesizes OB/4 weight rows of the block (signed 64-bit sums of T
// products, one Montgomery reduction) into LDS, one group ahead of the
// multiply-accumulate that reads them.
template <int MT, int OT, int WR, int WO, int NS, int TM = 0, class Hook = NoHook>
__device__ __forceinline__ void mac_lds_block(const MacArgs &a, uint32_t logical, uint32_t *lds_flat,
                                              const Hook &after_loop = Hook()) {
    using S = MacLdsShape<MT, OT, WR, WO, NS, TM>;
    constexpr int MB = S::MB, OB = S::OB, RND = S::RND, WB = S::WB, SROWS = S::SROWS;
    static_assert(WR * WO == 4, "four waves per block");
    static_assert(RND * (NS - 2) <= 12, "vmcnt budget");
    static_assert(TM == 0 || (MB % 16 == 0 && OB % 4 == 0 && TM <= kSynthTapsMax && RND * (NS - 2) <= 8),
                  "synthesizing schedules copy whole rounds of ciphertext rows");
    uint32_t(*lds)[SROWS][64] = reinterpret_cast<uint32_t(*)[SROWS][64]>(lds_flat);
    const uint32_t mt = logical % a.n_mt;
    const uint32_t ot = (logical / a.n_mt) % a.n_ot;
    const uint32_t kc = logical / (a.n_mt * a.n_ot);       // 64-slot chunk
    const uint32_t chunks = a.N >> 6;
    const uint32_t limb = kc / chunks;
    const uint32_t slot0 = limb * a.N + (kc % chunks) * 64;
    const LimbConst lc = a.lt.c[limb];
    const uint32_t r32 = lc.r32;
    const size_t LN = (size_t)a.L * a.N;
    const uint32_t row0 = mt * MB, o0 = ot * OB;
    // the wave index is the same on every lane: read it into a scalar so that
    // everything derived from it (LDS bases, output rows and channels, bounds
    // checks, store addresses) is scalar arithmetic and uniform branches
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t wr = wave / WO, wo = wave % WO;

    // loader: in round rd thread tid copies 16 B of LDS row rd*16 + tid/16
    const uint32_t *src[RND];
    size_t stride[RND];
#pragma unroll
    for (int rd = 0; rd < RND; rd++) {
        const uint32_t lr = rd * 16 + (tid >> 4);
        const uint32_t col = (tid & 15) * 4;
        if (TM > 0 || lr < (uint32_t)MB) {
            const uint32_t row = min(row0 + lr, a.rows - 1);
            src[rd] = a.ct + ((size_t)(row >> 1) * a.n_groups * 2 + (row & 1)) * LN + slot0 + col;
            stride[rd] = 2 * LN;
        } else {
            const uint32_t o = min(o0 + min(lr - MB, (uint32_t)OB - 1), a.Co - 1);
            src[rd] = a.w + (size_t)o * a.w_groups * LN + slot0 + col;
            stride[rd] = LN;
        }
    }
    // the copies are issued for groups 0, 1, 2, ... in order, so each round
    // keeps a running source pointer, advanced by its stride per issue
    auto issue = [&](int st) {
#pragma unroll
        for (int rd = 0; rd < RND; rd++) {
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src[rd],
                                             (__attribute__((address_space(3))) void *)&lds[st][rd * 16 + wave * 4][0],
                                             16, 0, 0);
            src[rd] += stride[rd];
        }
    };

    // tap powers of this lane's slot (synthesizing schedules)
    constexpr int TV = (TM > 0 && !S::VP_LDS) ? TM : 1;
    uint32_t vp[TV];
    uint32_t *vpl = lds_flat + NS * SROWS * 64;   // [TM][64] when S::VP_LDS
    if constexpr (TM > 0) {
        const uint32_t s = (kc % chunks) * 64 + lane;
        const uint32_t re = 2 * (__brev(s) >> (32 - a.logN)) + 1;
        const uint32_t *fw = a.fw + (size_t)limb * a.N;
        const uint32_t wsc = a.wscale[limb];
#pragma unroll
        for (int t = 0; t < TM; t++) {
            uint32_t v = 0;
            if ((uint32_t)t < a.T) {
                // psi^E 2^32 mod q from the bit-reversed table (psi^(m + N) = -psi^m)
                const uint32_t E = (re * a.texp[t]) & (2 * a.N - 1);
                const uint32_t f = fw[__brev(E & (a.N - 1)) >> (32 - a.logN)];
                v = mont_mul_red((E & a.N) ? lc.q - f : f, wsc, lc);
            }
            if constexpr (S::VP_LDS) {
                if (wave == 0) vpl[t * 64 + lane] = v;
            } else {
                vp[t] = v;
            }
        }
    }
    // this wave's OB/4 weight rows of group g, synthesized into stage st
    auto synth = [&](uint32_t g, int st) {
        if constexpr (TM > 0) {
            constexpr int R = OB / 4;
            const uint32_t ob = wave * R;
            // the taps are read-only in the kernel and the same on every lane:
            // read through the constant address space, so that they arrive by
            // scalar loads rather than by vector loads of one address per lane
            typedef const __attribute__((address_space(4))) int32_t ctap;
            ctap *tp[R];
#pragma unroll
            for (int r = 0; r < R; r++) {
                const uint32_t o = min(o0 + ob + r, a.Co - 1);
                tp[r] = (ctap *)(a.taps + ((size_t)o * a.w_groups + g) * a.T4);
            }
            // |sum| < T 2^13 2^31 <= 2^49 < q 2^20: starting from q 2^20 the
            // signed sum stays positive and below q 2^32, and q 2^20 adds
            // nothing mod q
            int64_t acc_s[R];
#pragma unroll
            for (int r = 0; r < R; r++) acc_s[r] = (int64_t)lc.q << 20;
#pragma unroll
            for (int t = 0; t < TM; t++) {
                if ((uint32_t)t >= a.T) break;
                const int32_t v = (int32_t)(S::VP_LDS ? vpl[t * 64 + lane] : vp[t < TV ? t : 0]);
#pragma unroll
                for (int r = 0; r < R; r++) acc_s[r] += (int64_t)v * tp[r][t];
            }
#pragma unroll
            for (int r = 0; r < R; r++) lds[st][WB + ob + r][lane] = redc64((uint64_t)acc_s[r], lc);
        }
    };

    uint64_t acc[MT][OT];
#pragma unroll
    for (int r = 0; r < MT; r++)
#pragma unroll
        for (int j = 0; j < OT; j++) acc[r][j] = 0;

    const uint32_t g1 = a.n_groups;
    if constexpr (TM > 0 && S::VP_LDS) __syncthreads();   // the powers wave 0 wrote
#pragma unroll
    for (int i = 0; i < NS - 1; i++)
        if ((uint32_t)i < g1) issue(i);
    if constexpr (TM > 0) synth(0, 0);
    const uint32_t F = lc.fold;
    uint32_t since = 0;
    int st = 0;
    for (uint32_t g = 0; g < g1; g++) {
        // this thread's copies of group g have landed once at most the
        // copies of the groups issued after it are outstanding (and, when
        // synthesizing, this wave's weight rows of group g are written)
        const int pend = (g + NS - 2 < g1) ? RND * (NS - 2) : 0;
        if constexpr (TM > 0) wait_vm_lgkm0(pend);
        else wait_vm(pend);
        // workgroup barrier without a fence: the copies this stage needs are
        // complete per the wait above; later stages stay in flight
        asm volatile("s_barrier" ::: "memory");
        if (g + NS - 1 < g1) issue(st == 0 ? NS - 1 : st - 1);   // group g + NS - 1
        // the next group's weights go into the next stage, whose weight rows
        // were last read in an iteration that every wave finished before this
        // barrier
        if (TM > 0 && g + 1 < g1) synth(g + 1, st + 1 == NS ? 0 : st + 1);
        uint32_t x[MT], w[OT];
#pragma unroll
        for (int r = 0; r < MT; r++) x[r] = lds[st][wr * MT + r][lane];
#pragma unroll
        for (int j = 0; j < OT; j++) w[j] = lds[st][WB + wo * OT + j][lane];
#pragma unroll
        for (int r = 0; r < MT; r++)
#pragma unroll
            for (int j = 0; j < OT; j++) acc[r][j] = mad64(x[r], w[j], acc[r][j]);
        if (++since >= F) {
            since = 0;
#pragma unroll
            for (int r = 0; r < MT; r++)
#pragma unroll
                for (int j = 0; j < OT; j++) acc[r][j] = fold(acc[r][j], r32);
        }
        st = (st + 1 == NS) ? 0 : st + 1;
    }
    after_loop();

    const uint32_t q = lc.q;
    const uint32_t orow0 = row0 + wr * MT, oo0 = o0 + wo * OT;
    // the products since the last fold decide whether the reduction folds
    // first (a uniform branch around the whole epilogue)
    auto epilogue = [&](auto fold_first) {
#pragma unroll
        for (int r = 0; r < MT; r++) {
            uint32_t y[OT];
#pragma unroll
            for (int j = 0; j < OT; j++) y[j] = reduce64<decltype(fold_first)::value>(acc[r][j], lc);
            if (a.fuse) {
#pragma unroll
                for (int h = 1; h < OT; h <<= 1) {
                    if ((uint32_t)h >= a.c_n) break;
#pragma unroll
                    for (int j = 0; j < OT; j++) {
                        if (j & h) continue;
                        const uint32_t u = y[j], v = y[j + h];
                        y[j] = csub(u + v, q);
                        y[j + h] = csub(u - v + q, q);
                    }
                }
            }
            const uint32_t row = orow0 + r;
            if (row >= a.rows) break;
            // uniform base of output (row, oo0) at this block's first slot; the
            // lanes store 64 consecutive words from it
            typedef __attribute__((address_space(1))) uint32_t gword;
            gword *dst = (gword *)a.out + ((size_t)(row >> 1) * a.Co * 2 + (row & 1)) * LN + slot0;
#pragma unroll
            for (int j = 0; j < OT; j++)
                if (oo0 + j < a.Co) dst[(size_t)(oo0 + j) * 2 * LN + lane] = y[j];
        }
    };
    if (since > lc.nofold) epilogue(std::true_type{});
    else epilogue(std::false_type{});
}

template <int MT, int OT, int WR, int WO, int NS, int TM = 0>
__global__ void __launch_bounds__(256, (MacLdsShape<MT, OT, WR, WO, NS, TM>::MIN_BLOCKS)) mac_lds_kernel(MacArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[MacLdsShape<MT, OT, WR, WO, NS, TM>::LDS_WORDS];
    // blocks are dealt to the 8 XCDs round robin: give each XCD a contiguous
    // range of logical blocks so that the tiles of one slot chunk share an L2
    const uint32_t nb = gridDim.x;
    const uint32_t xcd = blockIdx.x & 7u, local = blockIdx.x >> 3;
    const uint32_t per = (nb + 7) >> 3;
    const uint32_t full = nb - (per - 1) * 8;
    const uint32_t logical = (xcd < full) ? xcd * per + local
                                          : full * per + (xcd - full) * (per - 1) + local;
    mac_lds_block<MT, OT, WR, WO, NS, TM>(a, logical, lds);
}

}  // namespace
