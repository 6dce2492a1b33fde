// NTT-domain homomorphic convolution for gfx950: weight encoding, the lazy
// multiply-accumulate over input ciphertexts and the Walsh-Hadamard butterflies.
//
// For NTT slot (limb i, coefficient k) the layer is a small dense product over
// input groups g:
//   A[row][o] = sum_g ct[row][g] * W[o][g]  (mod q_i),  row = (image, tile, part)
// (the padded convolution of the "Prior Art on Homomorphic Convolution" section
// with the Walsh kernel polynomials of "Enabling Output Channel Packing").
// Products are 62-bit; they are accumulated in 64-bit registers without
// reduction (the "Lazy Reduction" section). Because q_i is close to 2^31,
// 2^32 mod q_i is small, so one multiply-add folds the accumulator back to
// about 2^54 every F products: acc <- hi32(acc) * (2^32 mod q) + lo32(acc).
// One full reduction per output coefficient follows the sum, before the
// Walsh-Hadamard recombination (the reduction point the paper puts before the
// PMult by the +-1 pattern).
#include <algorithm>

#include "mac.h"

namespace {

// One thread = one NTT slot (limb, k) for MT rows x OT outputs. Blocks are
// 256 threads along k. The block index is remapped so that all o- and
// row-tiles of one k-chunk land on the same XCD (blocks are dealt to the 8
// XCDs round robin) and share its L2 for the ciphertext and weight reads.
// Row and output base addresses are block-uniform (scalar registers); each
// lane adds its slot. The loads of input group g+1 are issued before the
// multiply-adds of group g so that memory latency overlaps the arithmetic.
template <int MT, int OT>
__global__ void __launch_bounds__(256) mac_kernel(MacArgs a) {
    const uint32_t nb = gridDim.x;
    const uint32_t xcd = blockIdx.x & 7u, local = blockIdx.x >> 3;
    const uint32_t per = (nb + 7) >> 3;        // logical blocks per XCD (ceil)
    const uint32_t full = nb - (per - 1) * 8;  // XCDs that get `per` blocks
    uint32_t logical;
    if (xcd < full) logical = xcd * per + local;
    else logical = full * per + (xcd - full) * (per - 1) + local;
    const uint32_t mt = logical % a.n_mt;
    const uint32_t ot = (logical / a.n_mt) % a.n_ot;
    const uint32_t kc = logical / (a.n_mt * a.n_ot);
    const uint32_t limb = kc / a.kchunks;
    const uint32_t slot = limb * a.N + (kc % a.kchunks) * 256 + threadIdx.x;  // < L*N
    const LimbConst lc = a.lt.c[limb];
    const uint32_t r32 = lc.r32;
    const size_t LN = (size_t)a.L * a.N;
    const uint32_t row0 = mt * MT, o0 = ot * OT;

    uint32_t g0 = 0, g1 = a.n_groups;
    if (a.depthwise) {
        g0 = o0 / a.ci;
        g1 = g0 + 1;
    }
    // uniform bases
    const uint32_t *ctb[MT];
#pragma unroll
    for (int r = 0; r < MT; r++) {
        const uint32_t row = min(row0 + r, a.rows - 1);
        ctb[r] = a.ct + ((size_t)(row >> 1) * a.n_groups * 2 + (row & 1)) * LN;
    }
    const uint32_t *wb[OT];
#pragma unroll
    for (int j = 0; j < OT; j++) {
        const uint32_t o = min(o0 + j, a.Co - 1);
        wb[j] = a.w + (size_t)o * a.w_groups * LN;
    }
    const size_t gstride_ct = 2 * LN;
    const size_t gstride_w = a.depthwise ? 0 : LN;

    uint64_t acc[MT][OT];
#pragma unroll
    for (int r = 0; r < MT; r++)
#pragma unroll
        for (int j = 0; j < OT; j++) acc[r][j] = 0;

    // two register sets, ping-pong: group g+1 loads while group g computes
    uint32_t xa[MT], wa[OT], xb[MT], wb2[OT];
    auto load = [&](uint32_t (&x)[MT], uint32_t (&w)[OT], uint32_t g) {
        const size_t oc = (size_t)g * gstride_ct, ow = (size_t)g * gstride_w;
#pragma unroll
        for (int r = 0; r < MT; r++) x[r] = ctb[r][oc + slot];
#pragma unroll
        for (int j = 0; j < OT; j++) w[j] = wb[j][ow + slot];
    };
    const uint32_t F = lc.fold;
    uint32_t since = 0;
    auto compute = [&](const uint32_t (&x)[MT], const uint32_t (&w)[OT]) {
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
    };
    load(xa, wa, g0);
    for (uint32_t g = g0; g < g1; g += 2) {
        if (g + 1 < g1) load(xb, wb2, g + 1);
        compute(xa, wa);
        if (g + 1 >= g1) break;
        if (g + 2 < g1) load(xa, wa, g + 2);
        compute(xb, wb2);
    }

    const uint32_t q = lc.q;
    // the reduction folds first unless at most lc.nofold products were added
    // since the last fold (a depthwise output has one product: never)
    auto epilogue = [&](auto fold_first) {
#pragma unroll
        for (int r = 0; r < MT; r++) {
            uint32_t y[OT];
#pragma unroll
            for (int j = 0; j < OT; j++) y[j] = reduce64<decltype(fold_first)::value>(acc[r][j], lc);
            if (a.fuse) {
                // Walsh-Hadamard butterflies over each aligned group of c_n outputs
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
            const uint32_t row = row0 + r;
            if (row >= a.rows) break;
            typedef __attribute__((address_space(1))) uint32_t gword;
            gword *dst = (gword *)a.out + ((size_t)(row >> 1) * a.Co * 2 + (row & 1)) * LN;
#pragma unroll
            for (int j = 0; j < OT; j++) {
                if (o0 + j < a.Co) dst[(size_t)(o0 + j) * 2 * LN + slot] = y[j];
            }
        }
    };
    if (since > lc.nofold) epilogue(std::true_type{});
    else epilogue(std::false_type{});
}

// Standalone Walsh-Hadamard recombination: out[G][b] = sum_j H[b][j] in[G][j].
// One thread per (G, word of a [2][L][N] block); c_n <= 64 residues in registers.
// Walsh-Hadamard butterflies across groups of CN polynomials: block x covers
// 256 x VW words of one ciphertext (all groups share the word layout), block
// y strides over the groups, so no index needs a 64-bit division. Each thread
// moves VW consecutive words of each of the CN polynomials (16-byte accesses
// for CN <= 16; narrower for wider groups to bound registers).
template <int CN>
__global__ void __launch_bounds__(256) wht_kernel(const uint32_t *in, uint32_t *out, size_t G, uint32_t words,
                                                  uint32_t logN, uint32_t L, LimbTable lt) {
    constexpr int VW = CN <= 16 ? 4 : (CN <= 32 ? 2 : 1);
    const uint32_t w0 = (blockIdx.x * 256 + threadIdx.x) * VW;
    if (w0 >= words) return;
    const uint32_t p = w0 >> logN;                 // polynomial within the ciphertext: part * L + limb
    const uint32_t q = lt.c[p >= L ? p - L : p].q;
    for (size_t gg = blockIdx.y; gg < G; gg += gridDim.y) {
        const uint32_t *src = in + gg * CN * (size_t)words + w0;
        uint32_t y[CN][VW];
#pragma unroll
        for (int j = 0; j < CN; j++) {
            if constexpr (VW == 4) {
                const uint4 v = *reinterpret_cast<const uint4 *>(src + (size_t)j * words);
                y[j][0] = v.x, y[j][1] = v.y, y[j][2] = v.z, y[j][3] = v.w;
            } else if constexpr (VW == 2) {
                const uint2 v = *reinterpret_cast<const uint2 *>(src + (size_t)j * words);
                y[j][0] = v.x, y[j][1] = v.y;
            } else {
                y[j][0] = src[(size_t)j * words];
            }
        }
#pragma unroll
        for (int h = 1; h < CN; h <<= 1)
#pragma unroll
            for (int j = 0; j < CN; j++) {
                if (j & h) continue;
#pragma unroll
                for (int v = 0; v < VW; v++) {
                    const uint32_t a = y[j][v], b = y[j + h][v];
                    y[j][v] = csub(a + b, q);
                    y[j + h][v] = csub(a - b + q, q);
                }
            }
        uint32_t *dst = out + gg * CN * (size_t)words + w0;
#pragma unroll
        for (int j = 0; j < CN; j++) {
            if constexpr (VW == 4) {
                *reinterpret_cast<uint4 *>(dst + (size_t)j * words) = make_uint4(y[j][0], y[j][1], y[j][2], y[j][3]);
            } else if constexpr (VW == 2) {
                *reinterpret_cast<uint2 *>(dst + (size_t)j * words) = make_uint2(y[j][0], y[j][1]);
            } else {
                dst[(size_t)j * words] = y[j][0];
            }
        }
    }
}

__global__ void fill_zero_kernel(uint32_t *p, size_t n) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    for (; i < n; i += (size_t)gridDim.x * 256) p[i] = 0;
}

// Scatter the taps of every Walsh kernel polynomial into a zeroed
// [Co][w_groups][L][N] array (coefficient domain). Thread per (o, tap):
//   value = c_n^{-1} 2^32 * sum_b H[j][b] f[G*c_n+b][ch][di][dj]  mod q_i,
//   exponent O - c'*Bt - di*Wp - dj,  o = G*c_n + j,  ch = g*ci + c'.
// The factor 2^32 puts the kernel polynomials in Montgomery form (the NTT is
// linear, so their transforms carry it too): the multiply-accumulate's one
// Montgomery reduction per output then removes it and returns the plain sum.
struct EncArgs {
    const int8_t *w;
    uint32_t *out;
    uint32_t N, L, Co, Ci, k, ci, Bt, Wp, O, n_groups, w_groups, c_n, depthwise;
    uint32_t wscale[HYENA_MAX_LIMBS];   // c_n^{-1} 2^32 mod q_i
    LimbTable lt;
};

__global__ void encode_scatter_kernel(EncArgs a) {
    const uint32_t kk = a.k * a.k;
    // standard: thread per (o, input channel, di, dj), value sums the c_n
    // Walsh terms at one position; depthwise: thread per (o, b, di, dj), the
    // c_n terms of a Walsh kernel sit at the c_n channel positions of the group
    const uint32_t inner = a.depthwise ? a.c_n : a.Ci;
    const size_t total = (size_t)a.Co * inner * kk;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const uint32_t o = (uint32_t)(idx / ((size_t)inner * kk));
    const uint32_t rem = (uint32_t)(idx % ((size_t)inner * kk));
    const uint32_t cw = rem / kk, di = (rem % kk) / a.k, dj = rem % a.k;
    const uint32_t G = o / a.c_n, j = o % a.c_n;
    int32_t gsum = 0;
    uint32_t ch;
    if (a.depthwise) {
        const uint32_t b = cw;
        const int sgn = (__popc(j & b) & 1) ? -1 : 1;
        ch = G * a.c_n + b;
        gsum = sgn * (int32_t)a.w[((size_t)ch * a.k + di) * a.k + dj];
    } else {
        ch = cw;
        for (uint32_t b = 0; b < a.c_n; b++) {
            const int sgn = (__popc(j & b) & 1) ? -1 : 1;
            gsum += sgn * (int32_t)a.w[(((size_t)(G * a.c_n + b) * a.Ci + cw) * a.k + di) * a.k + dj];
        }
    }
    if (gsum == 0) return;
    const uint32_t g = ch / a.ci, cp = ch % a.ci;
    const uint32_t e = a.O - cp * a.Bt - di * a.Wp - dj;
    const uint32_t gslot = a.depthwise ? 0 : g;
    for (uint32_t i = 0; i < a.L; i++) {
        const uint32_t q = a.lt.c[i].q;
        const int64_t v = (int64_t)gsum % (int64_t)q;
        const uint32_t vr = (uint32_t)(v < 0 ? v + q : v);
        const uint32_t val = (uint32_t)((uint64_t)vr * a.wscale[i] % q);
        a.out[(((size_t)o * a.w_groups + gslot) * a.L + i) * a.N + e] = val;
    }
}

template <int MT, int OT>
hipError_t launch_mac(const MacArgs &base, hipStream_t s) {
    MacArgs a = base;
    a.n_ot = (a.Co + OT - 1) / OT;
    a.n_mt = (a.rows + MT - 1) / MT;
    a.kchunks = a.N / 256;
    const size_t nb = (size_t)a.n_ot * a.n_mt * a.kchunks * a.L;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((mac_kernel<MT, OT>), dim3((unsigned)nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int MT, int OT, int WR, int WO, int NS, int TM = 0>
hipError_t launch_mac_lds(const MacArgs &base, hipStream_t s) {
    MacArgs a = base;
    a.n_ot = (a.Co + WO * OT - 1) / (WO * OT);
    a.n_mt = (a.rows + WR * MT - 1) / (WR * MT);
    a.kchunks = a.N / 64;
    const size_t nb = (size_t)a.n_ot * a.n_mt * a.kchunks * a.L;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((mac_lds_kernel<MT, OT, WR, WO, NS, TM>), dim3((unsigned)nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Walsh-combined integer taps of a standard layer for the synthesizing MAC:
// taps[o][g][t] = sum_b H[j][b] f[G c_n + b][g ci + c'][di][dj] with
// o = G c_n + j, t = c' k^2 + di k + dj (0 past the last input channel and
// for T <= t < T4).
struct TapArgs {
    const int8_t *w;
    int32_t *taps;
    uint32_t Co, Ci, k, ci, w_groups, c_n, T, T4;
};

__global__ void synth_taps_kernel(TapArgs a) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = (size_t)a.Co * a.w_groups * a.T4;
    if (idx >= n) return;
    const uint32_t t = (uint32_t)(idx % a.T4);
    const uint32_t g = (uint32_t)((idx / a.T4) % a.w_groups);
    const uint32_t o = (uint32_t)(idx / ((size_t)a.T4 * a.w_groups));
    int32_t v = 0;
    const uint32_t kk = a.k * a.k;
    if (t < a.T) {
        const uint32_t cw = g * a.ci + t / kk, tap = t % kk;
        if (cw < a.Ci) {
            const uint32_t G = o / a.c_n, j = o % a.c_n;
            for (uint32_t b = 0; b < a.c_n; b++) {
                const int f = a.w[((size_t)(G * a.c_n + b) * a.Ci + cw) * kk + tap];
                v += (__popc(j & b) & 1) ? -f : f;
            }
        }
    }
    a.taps[idx] = v;
}

hipError_t launch_wht(const hyena_ctx *c, uint32_t cn, const uint32_t *in, uint32_t *out, size_t G,
                      hipStream_t s) {
    const uint32_t words = 2 * c->L * c->N;        // one ciphertext; N is a multiple of 256
    const uint32_t vw = cn <= 16 ? 4 : (cn <= 32 ? 2 : 1);
    const dim3 grid((words / vw + 255) / 256, (unsigned)std::min<size_t>(G, 65535)), block(256);
    switch (cn) {
        case 2: hipLaunchKernelGGL(wht_kernel<2>, grid, block, 0, s, in, out, G, words, c->logN, c->L, c->lt); break;
        case 4: hipLaunchKernelGGL(wht_kernel<4>, grid, block, 0, s, in, out, G, words, c->logN, c->L, c->lt); break;
        case 8: hipLaunchKernelGGL(wht_kernel<8>, grid, block, 0, s, in, out, G, words, c->logN, c->L, c->lt); break;
        case 16: hipLaunchKernelGGL(wht_kernel<16>, grid, block, 0, s, in, out, G, words, c->logN, c->L, c->lt); break;
        case 32: hipLaunchKernelGGL(wht_kernel<32>, grid, block, 0, s, in, out, G, words, c->logN, c->L, c->lt); break;
        case 64: hipLaunchKernelGGL(wht_kernel<64>, grid, block, 0, s, in, out, G, words, c->logN, c->L, c->lt); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

// Tile choice of the MAC: rows x outputs per thread.
// MAC schedules: the direct kernel (registers only) and the LDS-pipelined
// kernel, with their tiles. The autotuner searches this table.
struct MacSched {
    int lds;            // 0: mac_kernel, 1: mac_lds_kernel
    int mt, ot, wr, wo, ns;
    int syn;            // 0: streams the NTT-domain weights; > 0: synthesizes them
                        // from at most `syn` integer taps per word
};

static const MacSched kScheds[] = {
    {0, 2, 16, 0, 0, 0, 0}, {0, 4, 8, 0, 0, 0, 0}, {0, 4, 16, 0, 0, 0, 0}, {0, 8, 4, 0, 0, 0, 0},
    {0, 8, 8, 0, 0, 0, 0},  {0, 16, 4, 0, 0, 0, 0}, {0, 2, 8, 0, 0, 0, 0}, {0, 2, 4, 0, 0, 0, 0},
    {0, 2, 2, 0, 0, 0, 0},  {0, 2, 1, 0, 0, 0, 0},  {0, 4, 4, 0, 0, 0, 0}, {0, 4, 2, 0, 0, 0, 0},
    {0, 4, 1, 0, 0, 0, 0},  {0, 8, 2, 0, 0, 0, 0},  {0, 8, 1, 0, 0, 0, 0},
    {1, 8, 8, 2, 2, 4, 0},  {1, 8, 8, 2, 2, 3, 0},  {1, 4, 8, 2, 2, 4, 0},  {1, 8, 8, 1, 4, 4, 0},
    {1, 2, 16, 1, 4, 4, 0}, {1, 4, 16, 1, 4, 3, 0}, {1, 8, 4, 4, 1, 4, 0},  {1, 4, 8, 1, 4, 4, 0},
    {1, 8, 8, 2, 2, 5, 0},  {1, 8, 8, 2, 2, 6, 0},
    // weights synthesized in the block: 16 or 32 rows, up to 9 or 18 taps
    {1, 8, 8, 2, 2, 4, 9},  {1, 8, 8, 4, 1, 4, 9},  {1, 8, 8, 2, 2, 4, 18}, {1, 8, 8, 4, 1, 4, 18},
};
static const int kNumScheds = sizeof(kScheds) / sizeof(kScheds[0]);

static int find_sched(int lds, int mt, int ot) {
    for (int i = 0; i < kNumScheds; i++)
        if (kScheds[i].lds == lds && kScheds[i].mt == mt && kScheds[i].ot == ot && !kScheds[i].syn) return i;
    return -1;
}

static uint32_t taps_per_word(const hyena_conv_desc *d) { return d->ci * d->k * d->k; }

// the synthesizing schedule for a standard layer: the smallest tap bound that
// covers its taps per word, 32 rows per block when there are that many
static int default_synth_sched(const hyena_conv_desc *d) {
    const uint32_t T = taps_per_word(d), rows = 2 * (d->batch ? d->batch : 1) * d->tiles;
    const int syn = T <= 9 ? 9 : 18;
    const int wr = rows >= 32 ? 4 : 2;
    for (int i = 0; i < kNumScheds; i++)
        if (kScheds[i].syn == syn && kScheds[i].wr == wr) return i;
    return -1;
}

static int default_sched(const hyena_conv_desc *d) {
    const uint32_t rows = 2 * d->batch * d->tiles;
    if (d->depthwise) {
        // outputs of one tile must share the input group
        int ot = 1;
        while (ot < 8 && d->ci % (2 * ot) == 0 && d->Co % (2 * ot) == 0) ot *= 2;
        if (ot < (int)d->c_n) ot = (int)d->c_n;
        return find_sched(0, rows >= 4 ? 4 : 2, ot);
    }
    if (rows >= 16) return 15;   // LDS 16 x 16 block tile
    if (rows >= 8) return 18;    // LDS 8 x 32
    if (rows >= 4) return 20;    // LDS 4 x 64
    return 19;                   // LDS 2 x 64
}

static bool sched_valid(const hyena_conv_desc *d, const MacSched &t) {
    if (t.syn) return !d->depthwise && taps_per_word(d) <= (uint32_t)t.syn;
    if (!d->depthwise) return true;
    return t.lds == 0 && (d->ci % (uint32_t)t.ot == 0 || t.ot == 1) && (uint32_t)t.ot >= 1;
}

static hipError_t dispatch_mac(const MacArgs &a, const MacSched &t, hipStream_t s) {
    if (t.syn) {
#define HY_S(M, O, R, W, S, T) \
    if (t.mt == M && t.ot == O && t.wr == R && t.wo == W && t.ns == S && t.syn == T) \
        return launch_mac_lds<M, O, R, W, S, T>(a, s);
        HY_S(8, 8, 2, 2, 4, 9) HY_S(8, 8, 4, 1, 4, 9) HY_S(8, 8, 2, 2, 4, 18) HY_S(8, 8, 4, 1, 4, 18)
#undef HY_S
        return hipErrorInvalidValue;
    }
    if (t.lds) {
#define HY_L(M, O, R, W, S) \
    if (t.mt == M && t.ot == O && t.wr == R && t.wo == W && t.ns == S) return launch_mac_lds<M, O, R, W, S>(a, s);
        HY_L(8, 8, 2, 2, 4) HY_L(8, 8, 2, 2, 3) HY_L(4, 8, 2, 2, 4) HY_L(8, 8, 1, 4, 4)
        HY_L(2, 16, 1, 4, 4) HY_L(4, 16, 1, 4, 3) HY_L(8, 4, 4, 1, 4) HY_L(4, 8, 1, 4, 4)
        HY_L(8, 8, 2, 2, 5) HY_L(8, 8, 2, 2, 6)
#undef HY_L
        return hipErrorInvalidValue;
    }
#define HY_CASE(M, O) \
    if (t.mt == M && t.ot == O) return launch_mac<M, O>(a, s);
    HY_CASE(2, 1) HY_CASE(2, 2) HY_CASE(2, 4) HY_CASE(2, 8) HY_CASE(2, 16)
    HY_CASE(4, 1) HY_CASE(4, 2) HY_CASE(4, 4) HY_CASE(4, 8) HY_CASE(4, 16)
    HY_CASE(8, 1) HY_CASE(8, 2) HY_CASE(8, 4) HY_CASE(8, 8)
    HY_CASE(16, 4)
#undef HY_CASE
    return hipErrorInvalidValue;
}

MacArgs conv_make_args(const hyena_ctx *c, const hyena_conv_desc *d, const uint32_t *ct, const uint32_t *w,
                       const int32_t *taps, uint32_t *out, int sched, bool per_channel, bool *needs_wht) {
    const MacSched &t = kScheds[sched];
    const uint32_t cn = d->c_n ? d->c_n : 1;
    MacArgs a{};
    a.ct = ct;
    a.w = w;
    a.out = out;
    if (t.syn) {
        a.taps = taps;
        a.fw = c->d_fw;
        a.T = taps_per_word(d);
        a.T4 = (a.T + 3) & ~3u;
        const uint32_t kk = d->k * d->k;
        for (uint32_t i = 0; i < a.T && i < (uint32_t)kSynthTapsMax; i++) {
            const uint32_t cp = i / kk, di = (i % kk) / d->k, dj = i % d->k;
            a.texp[i] = d->O - cp * d->Bt - di * d->Wp - dj;
        }
        // c_n^{-1} 2^64 mod q_i: Montgomery form of the output scale c_n^{-1} 2^32
        for (uint32_t i = 0; i < c->L; i++)
            a.wscale[i] = to_montgomery(to_montgomery(h_powmod(cn, c->q[i] - 2, c->q[i]), c->q[i]), c->q[i]);
    }
    a.N = c->N;
    a.L = c->L;
    a.logN = c->logN;
    a.Co = d->Co;
    a.n_groups = d->n_groups;
    a.w_groups = d->w_groups;
    a.rows = 2 * (d->batch ? d->batch : 1) * d->tiles;
    a.ci = d->ci;
    a.c_n = cn;
    a.depthwise = d->depthwise;
    a.lt = c->lt;
    const bool fuse_in_mac = cn > 1 && (uint32_t)t.ot >= cn && (uint32_t)t.ot % cn == 0;
    a.fuse = (per_channel && fuse_in_mac) ? 1 : 0;
    if (t.lds) {
        a.n_ot = (a.Co + t.wo * t.ot - 1) / (t.wo * t.ot);
        a.n_mt = (a.rows + t.wr * t.mt - 1) / (t.wr * t.mt);
        a.kchunks = a.N / 64;
    } else {
        a.n_ot = (a.Co + t.ot - 1) / t.ot;
        a.n_mt = (a.rows + t.mt - 1) / t.mt;
        a.kchunks = a.N / 256;
    }
    if (needs_wht) *needs_wht = cn > 1 && per_channel && !fuse_in_mac;
    return a;
}

int conv_num_scheds() { return kNumScheds; }
int conv_sched_syn(int sched) { return sched >= 0 && sched < kNumScheds ? kScheds[sched].syn : 0; }
int conv_default_synth_sched(const hyena_conv_desc *d) { return default_synth_sched(d); }
bool conv_sched_valid(const hyena_conv_desc *d, int sched) {
    return sched >= 0 && sched < kNumScheds && sched_valid(d, kScheds[sched]);
}
int conv_default_sched(const hyena_conv_desc *d) { return default_sched(d); }
int conv_sched_info(int sched, int *info) {
    const MacSched &t = kScheds[sched];
    info[0] = t.lds; info[1] = t.mt; info[2] = t.ot; info[3] = t.wr; info[4] = t.wo; info[5] = t.ns;
    return HYENA_OK;
}
hipError_t conv_launch_wht(const hyena_ctx *c, uint32_t cn, const uint32_t *in, uint32_t *out, size_t G,
                           hipStream_t s) {
    return launch_wht(c, cn, in, out, G, s);
}

int conv_launch(const hyena_ctx *c, const hyena_conv_desc *d, const uint32_t *ct, const uint32_t *w,
                const int32_t *taps, uint32_t *out, int sched, bool per_channel, hipStream_t s) {
    if (!c || !d || !ct || !out) return set_error(HYENA_EINVAL, "hyena_conv: NULL argument");
    if (!d->Bt || !d->n_groups) return set_error(HYENA_EINVAL, "hyena_conv: descriptor not planned");
    if (sched < 0) sched = w ? default_sched(d) : default_synth_sched(d);
    if (sched < 0 || sched >= kNumScheds) return set_error(HYENA_EINVAL, "hyena_conv: unknown schedule");
    const MacSched &t = kScheds[sched];
    if (t.syn ? !taps : !w)
        return set_error(HYENA_EINVAL, t.syn ? "hyena_conv: a synthesizing schedule needs the integer taps"
                                             : "hyena_conv: NULL weights");
    if (((uintptr_t)ct | (uintptr_t)(t.syn ? nullptr : w) | (uintptr_t)out) & 15u)
        return set_error(HYENA_EINVAL, "hyena_conv: device arrays must be 16-byte aligned");
    if ((uintptr_t)taps & 3u) return set_error(HYENA_EINVAL, "hyena_conv: taps must be 4-byte aligned");
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_conv: context was created host-only");
    if (c->N % 256) return set_error(HYENA_EUNSUPPORTED, "hyena_conv: N must be a multiple of 256");
    if (!sched_valid(d, t)) return set_error(HYENA_EINVAL, "hyena_conv: schedule not valid for this layer");
    bool wht = false;
    const MacArgs a = conv_make_args(c, d, ct, w, taps, out, sched, per_channel, &wht);
    hipError_t e = dispatch_mac(a, t, s);
    if (e == hipErrorInvalidValue) return set_error(HYENA_EINVAL, "hyena_conv: unsupported MAC schedule");
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_conv: ") + hipGetErrorString(e));
    if (wht) {
        const size_t G = (size_t)a.rows / 2 * d->Co / a.c_n;
        e = launch_wht(c, a.c_n, out, out, G, s);
        if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_conv: ") + hipGetErrorString(e));
    }
    return HYENA_OK;
}

extern "C" int hyena_conv_schedules(int *count) {
    if (count) *count = kNumScheds;
    return HYENA_OK;
}

extern "C" int hyena_conv_schedule_info(int sched, int *info /* [6] */) {
    if (sched < 0 || sched >= kNumScheds || !info) return set_error(HYENA_EINVAL, "hyena_conv_schedule_info: bad schedule");
    const MacSched &t = kScheds[sched];
    info[0] = t.lds; info[1] = t.mt; info[2] = t.ot; info[3] = t.wr; info[4] = t.wo; info[5] = t.ns;
    return HYENA_OK;
}

extern "C" int hyena_conv_default_schedule(const hyena_conv_desc *d) {
    if (!d) return set_error(HYENA_EINVAL, "hyena_conv_default_schedule: NULL descriptor");
    return default_sched(d);
}

extern "C" int hyena_conv(const hyena_ctx *c, const hyena_conv_desc *d, const uint32_t *d_ct_ntt,
                          const uint32_t *d_wntt, uint32_t *d_out_ntt, hyena_stream_t s) {
    if (!d) return set_error(HYENA_EINVAL, "hyena_conv: NULL descriptor");
    if (!d_wntt) return set_error(HYENA_EINVAL, "hyena_conv: NULL argument");
    // without HYENA_FUSE_WHT the output holds the Walsh components
    const bool per_channel = (d->flags & HYENA_FUSE_WHT) || d->c_n <= 1;
    return conv_launch(c, d, d_ct_ntt, d_wntt, nullptr, d_out_ntt, -1, per_channel, (hipStream_t)s);
}

extern "C" int hyena_conv_synth(const hyena_ctx *c, const hyena_conv_desc *d, const uint32_t *d_ct_ntt,
                                const int32_t *d_taps, uint32_t *d_out_ntt, hyena_stream_t s) {
    if (!d) return set_error(HYENA_EINVAL, "hyena_conv_synth: NULL descriptor");
    if (!d_taps) return set_error(HYENA_EINVAL, "hyena_conv_synth: NULL argument");
    if (!d->Bt) return set_error(HYENA_EINVAL, "hyena_conv_synth: descriptor not planned");
    if (d->depthwise) return set_error(HYENA_EUNSUPPORTED, "hyena_conv_synth: depthwise layers stream their weights");
    if (taps_per_word(d) > (uint32_t)kSynthTapsMax)
        return set_error(HYENA_EUNSUPPORTED, "hyena_conv_synth: more than 18 taps per weight word");
    const bool per_channel = (d->flags & HYENA_FUSE_WHT) || d->c_n <= 1;
    return conv_launch(c, d, d_ct_ntt, nullptr, d_taps, d_out_ntt, default_synth_sched(d), per_channel,
                       (hipStream_t)s);
}

extern "C" int hyena_conv_tiled(const hyena_ctx *c, const hyena_conv_desc *d, const uint32_t *d_ct_ntt,
                                const uint32_t *d_wntt, uint32_t *d_out_ntt, int sched, hyena_stream_t s) {
    if (!d) return set_error(HYENA_EINVAL, "hyena_conv_tiled: NULL descriptor");
    const bool per_channel = (d->flags & HYENA_FUSE_WHT) || d->c_n <= 1;
    // a synthesizing schedule takes the integer taps in place of d_wntt
    const bool syn = sched >= 0 && sched < kNumScheds && kScheds[sched].syn;
    return conv_launch(c, d, d_ct_ntt, syn ? nullptr : d_wntt, syn ? (const int32_t *)d_wntt : nullptr,
                       d_out_ntt, sched, per_channel, (hipStream_t)s);
}

extern "C" int hyena_conv_schedule_taps(int sched) {
    if (sched < 0 || sched >= kNumScheds) return set_error(HYENA_EINVAL, "hyena_conv_schedule_taps: bad schedule");
    return kScheds[sched].syn;
}

extern "C" int hyena_synth_taps(const hyena_ctx *c, const hyena_conv_desc *d, const int8_t *d_w, int32_t *d_taps,
                                hyena_stream_t s) {
    if (!c || !d || !d_w || !d_taps) return set_error(HYENA_EINVAL, "hyena_synth_taps: NULL argument");
    if (!d->Bt) return set_error(HYENA_EINVAL, "hyena_synth_taps: descriptor not planned");
    if (d->c_n & (d->c_n - 1)) return set_error(HYENA_EINVAL, "hyena_synth_taps: c_n must be a power of two");
    if (d->depthwise) return set_error(HYENA_EUNSUPPORTED, "hyena_synth_taps: depthwise layers stream their weights");
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_synth_taps: context was created host-only");
    if ((uintptr_t)d_taps & 3u) return set_error(HYENA_EINVAL, "hyena_synth_taps: d_taps must be 4-byte aligned");
    TapArgs a{};
    a.w = d_w;
    a.taps = d_taps;
    a.Co = d->Co;
    a.Ci = d->Ci;
    a.k = d->k;
    a.ci = d->ci;
    a.w_groups = d->w_groups;
    a.c_n = d->c_n ? d->c_n : 1;
    a.T = taps_per_word(d);
    a.T4 = (a.T + 3) & ~3u;
    const size_t n = (size_t)a.Co * a.w_groups * a.T4;
    if (n == 0) return HYENA_OK;
    if ((n + 255) / 256 > 0x7fffffff) return set_error(HYENA_EINVAL, "hyena_synth_taps: layer too large");
    hipLaunchKernelGGL(synth_taps_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_synth_taps: ") + hipGetErrorString(e));
    return HYENA_OK;
}

extern "C" int hyena_wht_pack(const hyena_ctx *c, uint32_t cn, const uint32_t *in, uint32_t *out, size_t G,
                              hyena_stream_t s) {
    if (!c || (G && (!in || !out))) return set_error(HYENA_EINVAL, "hyena_wht_pack: NULL argument");
    if (((uintptr_t)in | (uintptr_t)out) & 15u)
        return set_error(HYENA_EINVAL, "hyena_wht_pack: device arrays must be 16-byte aligned");
    if (cn == 0 || (cn & (cn - 1)) || cn > 64) return set_error(HYENA_EINVAL, "hyena_wht_pack: c_n must be 1..64, a power of two");
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_wht_pack: context was created host-only");
    if (G == 0) return HYENA_OK;
    if (cn == 1) {
        if (in != out) HIP_TRY(hipMemcpyAsync(out, in, G * 2 * (size_t)c->L * c->N * 4, hipMemcpyDeviceToDevice, (hipStream_t)s));
        return HYENA_OK;
    }
    hipError_t e = launch_wht(c, cn, in, out, G, (hipStream_t)s);
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_wht_pack: ") + hipGetErrorString(e));
    return HYENA_OK;
}

extern "C" int hyena_encode_weights(const hyena_ctx *c, const hyena_conv_desc *d, const int8_t *d_w,
                                    uint32_t *d_wntt, hyena_stream_t s) {
    if (!c || !d || !d_w || !d_wntt) return set_error(HYENA_EINVAL, "hyena_encode_weights: NULL argument");
    if ((uintptr_t)d_wntt & 15u) return set_error(HYENA_EINVAL, "hyena_encode_weights: d_wntt must be 16-byte aligned");
    if (!d->Bt) return set_error(HYENA_EINVAL, "hyena_encode_weights: descriptor not planned");
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_encode_weights: context was created host-only");
    const hipStream_t st = (hipStream_t)s;
    const size_t polys = (size_t)d->Co * d->w_groups;
    const size_t words = polys * c->L * c->N;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)std::min<size_t>((words + 255) / 256, 65536)), dim3(256), 0,
                       st, d_wntt, words);
    EncArgs a{};
    a.w = d_w;
    a.out = d_wntt;
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
    a.w_groups = d->w_groups;
    a.c_n = d->c_n ? d->c_n : 1;
    a.depthwise = d->depthwise;
    a.lt = c->lt;
    for (uint32_t i = 0; i < c->L; i++) a.wscale[i] = to_montgomery(h_powmod(a.c_n, c->q[i] - 2, c->q[i]), c->q[i]);
    const size_t taps = (size_t)d->Co * (d->depthwise ? a.c_n : d->Ci) * d->k * d->k;
    hipLaunchKernelGGL(encode_scatter_kernel, dim3((unsigned)((taps + 255) / 256)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_encode_weights: ") + hipGetErrorString(e));
    return launch_ntt(c, d_wntt, polys, false, st);
}
