// Convolution planning: geometry of the coefficient-encoded padded tensor
// (the "Prior Art on Homomorphic Convolution" section: padded channels, the C x H x W tensor split over
// ceil(CHW / n) ciphertexts), the noise-budget check of the "Homomorphic Operations in BFV" section
// (||v|| < Delta / 2) and the host packing helpers.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace {
constexpr uint64_t kErrBound = 32;  // fresh error bound B = 10 sigma
constexpr uint64_t kValBound = 8;   // |x|, |f| <= 8 for signed 4-bit values
}  // namespace

extern "C" int hyena_conv_plan(const hyena_ctx *c, hyena_conv_desc *d) {
    if (!c || !d) return set_error(HYENA_EINVAL, "hyena_conv_plan: NULL argument");
    const uint32_t N = c->N;
    if (d->k != 1 && d->k != 3) return set_error(HYENA_EINVAL, "hyena_conv_plan: k must be 1 or 3");
    if (!d->H || !d->W || !d->Ci || !d->Co) return set_error(HYENA_EINVAL, "hyena_conv_plan: empty layer");
    if (d->stride != 0 && d->stride != 1 && d->stride != 2)
        return set_error(HYENA_EINVAL, "hyena_conv_plan: stride must be 1 or 2");
    if (d->depthwise && d->Ci != d->Co) return set_error(HYENA_EINVAL, "hyena_conv_plan: depthwise needs Ci == Co");
    const uint32_t cn = d->c_n ? d->c_n : 1;
    if (cn & (cn - 1)) return set_error(HYENA_EINVAL, "hyena_conv_plan: c_n must be a power of two");
    if (d->Co % cn) return set_error(HYENA_EINVAL, "hyena_conv_plan: c_n must divide Co");
    if (cn > 64) return set_error(HYENA_EINVAL, "hyena_conv_plan: c_n above 64 is not supported");
    d->c_n = cn;
    if (d->batch == 0) d->batch = 1;
    const uint32_t p = (d->k - 1) / 2;
    d->pad = p;
    d->Wp = d->W + 2 * p;
    const uint64_t full = (uint64_t)(d->H + 2 * p) * d->Wp;
    if (full <= N) {
        d->R = d->H;
        d->tiles = 1;
        d->Bt = (uint32_t)full;
        const uint32_t cmax = std::min<uint32_t>(d->Ci, N / d->Bt);
        const uint32_t ci = d->ci_req ? d->ci_req : cmax;
        if (ci < 1 || ci > cmax) return set_error(HYENA_EINVAL, "hyena_conv_plan: ci_req out of range");
        d->ci = ci;
    } else {
        if (N / d->Wp <= 2 * p) return set_error(HYENA_EINVAL, "hyena_conv_plan: padded row does not fit N");
        if (d->ci_req > 1) return set_error(HYENA_EINVAL, "hyena_conv_plan: row-tiled layers use ci = 1");
        d->R = N / d->Wp - 2 * p;
        d->tiles = (d->H + d->R - 1) / d->R;
        d->Bt = (d->R + 2 * p) * d->Wp;
        d->ci = 1;
    }
    d->n_groups = (d->Ci + d->ci - 1) / d->ci;
    d->O = (d->ci - 1) * d->Bt + (d->k - 1) * d->Wp + (d->k - 1);
    d->n_in = d->tiles * d->n_groups;
    d->n_out = d->tiles * d->Co;
    if (d->depthwise) {
        // every output of a Walsh group must read the same input ciphertext
        if (cn > 1 && d->ci % cn) return set_error(HYENA_EINVAL, "hyena_conv_plan: depthwise c_n must divide ci");
        d->w_groups = 1;
    } else {
        d->w_groups = d->n_groups;
    }

    // Noise budget (the "Homomorphic Operations in BFV" section): the product's noise E = sum_g e_g K_{o,g}
    // with |e| <= B, plus the lift term r |Y| (r = q mod t), must stay below
    // q / (2t) scaled: 2 (t B ||K||_1 + r |Y|) < q, and |Y| < t / 2.
    const uint64_t taps = (uint64_t)d->k * d->k * (d->depthwise ? 1 : d->Ci);
    const uint64_t l1 = taps * kValBound;
    const uint64_t ymax = l1 * kValBound;
    const uint64_t t = 1ull << c->log2_t;
    if (2 * ymax >= t)
        return set_error(HYENA_ENOISE, "hyena_conv_plan: worst-case output " + std::to_string(ymax) +
                                           " does not fit t/2");
    double logq = 0;
    for (uint32_t q : c->q) logq += std::log2((double)q);
    if (logq < 120) {  // exact check when q fits 128 bits
        unsigned __int128 q = 1;
        for (uint32_t qi : c->q) q *= qi;
        const unsigned __int128 r = q % t;
        const unsigned __int128 need = 2 * ((unsigned __int128)t * kErrBound * l1 + r * ymax);
        if (need >= q)
            return set_error(HYENA_ENOISE, "hyena_conv_plan: worst-case noise exceeds Delta/2 "
                                           "(more RNS limbs are needed)");
    }
    return HYENA_OK;
}

extern "C" int hyena_pack_input(const hyena_conv_desc *d, uint32_t N, const int8_t *x, int32_t *msg) {
    if (!d || !x || !msg) return set_error(HYENA_EINVAL, "hyena_pack_input: NULL argument");
    if (!d->Bt) return set_error(HYENA_EINVAL, "hyena_pack_input: descriptor not planned");
    const uint32_t p = d->pad, Hp = d->H + 2 * p;
    std::memset(msg, 0, sizeof(int32_t) * (size_t)d->tiles * d->n_groups * N);
    for (uint32_t tau = 0; tau < d->tiles; tau++)
        for (uint32_t g = 0; g < d->n_groups; g++) {
            int32_t *m = msg + ((size_t)tau * d->n_groups + g) * N;
            for (uint32_t c = 0; c < d->ci; c++) {
                const uint32_t ch = g * d->ci + c;
                if (ch >= d->Ci) break;
                for (uint32_t r = 0; r < d->R + 2 * p; r++) {
                    const uint32_t prow = tau * d->R + r;  // row of the padded image
                    if (prow >= Hp) break;
                    if (prow < p || prow >= p + d->H) continue;  // zero padding rows
                    const int8_t *src = x + ((size_t)ch * d->H + (prow - p)) * d->W;
                    int32_t *dst = m + (size_t)c * d->Bt + (size_t)r * d->Wp + p;
                    for (uint32_t col = 0; col < d->W; col++) dst[col] = src[col];
                }
            }
        }
    return HYENA_OK;
}

extern "C" int hyena_unpack_output(const hyena_conv_desc *d, uint32_t N, const int32_t *msg, int32_t *y) {
    if (!d || !msg || !y) return set_error(HYENA_EINVAL, "hyena_unpack_output: NULL argument");
    if (!d->Bt) return set_error(HYENA_EINVAL, "hyena_unpack_output: descriptor not planned");
    // a stride-s layer keeps rows and columns 0, s, 2s, ... of the stride-1
    // output that the server computes
    const uint32_t s = d->stride > 1 ? d->stride : 1;
    const uint32_t Ho = (d->H + s - 1) / s, Wo = (d->W + s - 1) / s;
    for (uint32_t tau = 0; tau < d->tiles; tau++)
        for (uint32_t o = 0; o < d->Co; o++) {
            const int32_t *m = msg + ((size_t)tau * d->Co + o) * N;
            for (uint32_t r = 0; r < d->R; r++) {
                const uint32_t row = tau * d->R + r;
                if (row >= d->H) break;
                if (row % s) continue;
                const int32_t *src = m + d->O + (size_t)r * d->Wp;
                int32_t *dst = y + ((size_t)o * Ho + row / s) * Wo;
                if (s == 1) {
                    std::memcpy(dst, src, sizeof(int32_t) * d->W);
                } else {
                    for (uint32_t j = 0; j < Wo; j++) dst[j] = src[(size_t)j * s];
                }
            }
        }
    return HYENA_OK;
}
