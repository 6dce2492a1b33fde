// Test-setup BFV operations on the host (the client side of the "Homomorphic Operations in BFV" section):
// ternary key generation, symmetric encryption and RNS decryption.
#include <cmath>
#include <cstring>
#include <thread>

#include "bfv.h"

namespace {

inline uint64_t sm64(uint64_t key, uint64_t ctr) { return hy_sm64(key, ctr); }

constexpr int kB = kErrBound;    // error bound B = 10 sigma
constexpr double kSigma = 3.2;  // error standard deviation

// Thresholds of the rounded Gaussian on [-B, B]: cumulative weights
// exp(-x^2 / (2 sigma^2)) from x = -B upward, scaled to 2^63.
struct Cdt {
    uint64_t t[2 * kB + 1];
    Cdt() {
        double cum[2 * kB + 1];
        double run = 0.0;
        for (int x = -kB; x <= kB; x++) {
            run += std::exp(-(double)(x * x) / (2.0 * kSigma * kSigma));
            cum[x + kB] = run;
        }
        for (int k = 0; k <= 2 * kB; k++)
            t[k] = (uint64_t)(cum[k] / run * 9223372036854775808.0);
    }
    int sample(uint64_t r) const {
        uint64_t u = r >> 1;
        int cnt = 0;
        for (int k = 0; k < 2 * kB; k++) cnt += (u >= t[k]);
        return cnt - kB;
    }
};

const Cdt &cdt() {
    static const Cdt table;
    return table;
}

inline uint32_t uniform_mod(uint64_t r, uint32_t q) {
    return (uint32_t)(((unsigned __int128)r * q) >> 64);
}

inline uint32_t lift(int64_t x, uint32_t q) {
    int64_t r = x % (int64_t)q;
    return (uint32_t)(r < 0 ? r + q : r);
}

// floor(q / 2^log2_t) mod q_i, with q = prod q_j held as 32-bit words.
std::vector<uint32_t> delta_residues(const hyena_ctx *c) {
    std::vector<uint32_t> w(1, 1);  // little-endian words of q
    for (uint32_t q : c->q) {
        uint64_t carry = 0;
        for (auto &x : w) {
            uint64_t v = (uint64_t)x * q + carry;
            x = (uint32_t)v;
            carry = v >> 32;
        }
        if (carry) w.push_back((uint32_t)carry);
    }
    // shift right by log2_t
    const uint32_t s = c->log2_t;
    std::vector<uint32_t> d(w.size(), 0);
    for (size_t i = 0; i < w.size(); i++) {
        uint64_t lo = w[i] >> s;
        uint64_t hi = (i + 1 < w.size()) ? ((uint64_t)w[i + 1] << (32 - s)) : 0;
        d[i] = (uint32_t)(lo | hi);
    }
    std::vector<uint32_t> out;
    for (uint32_t q : c->q) {
        uint64_t r = 0;
        for (size_t i = d.size(); i-- > 0;) r = ((r << 32) | d[i]) % q;
        out.push_back((uint32_t)r);
    }
    return out;
}

template <class F>
void parallel_for(size_t n, F f) {
    unsigned hw = std::thread::hardware_concurrency();
    unsigned nt = (unsigned)std::min<size_t>(n, hw ? std::min(hw, 16u) : 4u);
    if (nt <= 1) {
        for (size_t i = 0; i < n; i++) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; t++)
        th.emplace_back([&, t] {
            for (size_t i = t; i < n; i += nt) f(i);
        });
    for (auto &x : th) x.join();
}

// NTT of the secret key per limb.
std::vector<uint32_t> secret_ntt(const hyena_ctx *c, const int8_t *sk) {
    std::vector<uint32_t> s((size_t)c->L * c->N);
    for (uint32_t i = 0; i < c->L; i++) {
        for (uint32_t j = 0; j < c->N; j++) s[(size_t)i * c->N + j] = lift(sk[j], c->q[i]);
        host_ntt(c, i, &s[(size_t)i * c->N]);
    }
    return s;
}

}  // namespace

// Shared with the batch versions on the device (client.hip), so that both
// compute with the same constants.
std::vector<uint32_t> bfv_delta_residues(const hyena_ctx *c) { return delta_residues(c); }
void bfv_error_thresholds(uint64_t *t64) {
    for (int k = 0; k < 2 * kB; k++) t64[k] = cdt().t[k];
}
void bfv_hps_constants(const hyena_ctx *c, uint64_t *A, uint64_t *F) {
    const uint64_t t = 1ull << c->log2_t;
    for (uint32_t i = 0; i < c->L; i++) {
        const uint32_t q = c->q[i];
        uint64_t Mi = 1;  // (q / q_i) mod q_i
        for (uint32_t j = 0; j < c->L; j++)
            if (j != i) Mi = Mi * (c->q[j] % q) % q;
        const uint64_t yi = h_powmod((uint32_t)Mi, q - 2, q);
        const uint64_t ty = (t % q) * yi;  // t * y_i (< 2^51), exact
        A[i] = ty / q;
        F[i] = (uint64_t)(((unsigned __int128)(ty % q) << 64) / q);   // (t y_i mod q_i) / q_i in 0.64
    }
}

extern "C" int hyena_keygen(const hyena_ctx *c, uint64_t seed, int8_t *sk) {
    if (!c || !sk) return set_error(HYENA_EINVAL, "hyena_keygen: NULL argument");
    for (uint32_t j = 0; j < c->N; j++) {
        uint64_t hi = sm64(seed, j) >> 32;
        sk[j] = (int8_t)((int)((hi * 3) >> 32) - 1);
    }
    return HYENA_OK;
}

extern "C" int hyena_encrypt(const hyena_ctx *c, const int8_t *sk, const int32_t *msg, size_t n,
                             uint64_t seed, uint32_t *ct) {
    if (!c || !sk || (n && (!msg || !ct))) return set_error(HYENA_EINVAL, "hyena_encrypt: NULL argument");
    const uint32_t N = c->N, L = c->L;
    const int64_t t = 1ll << c->log2_t;
    for (size_t k = 0; k < n * N; k++)
        if (msg[k] <= -t / 2 || msg[k] > t / 2)
            return set_error(HYENA_EINVAL, "hyena_encrypt: message outside (-t/2, t/2]");
    const auto s_hat = secret_ntt(c, sk);
    const auto delta = delta_residues(c);
    const Cdt &g = cdt();
    parallel_for(n, [&](size_t m) {
        std::vector<int> e(N);
        for (uint32_t j = 0; j < N; j++) e[j] = g.sample(sm64(seed, 2 * ((uint64_t)m * N + j) + 1));
        std::vector<uint32_t> a(N), as(N);
        for (uint32_t i = 0; i < L; i++) {
            const uint32_t q = c->q[i];
            for (uint32_t j = 0; j < N; j++)
                a[j] = uniform_mod(sm64(seed, 2 * (((uint64_t)m * L + i) * N + j)), q);
            as = a;
            host_ntt(c, i, as.data());
            for (uint32_t j = 0; j < N; j++) as[j] = h_mulmod(as[j], s_hat[(size_t)i * N + j], q);
            host_intt(c, i, as.data());
            uint32_t *c0 = ct + (((size_t)m * 2 + 0) * L + i) * N;
            uint32_t *c1 = ct + (((size_t)m * 2 + 1) * L + i) * N;
            for (uint32_t j = 0; j < N; j++) {
                uint64_t v = (uint64_t)h_mulmod(delta[i], lift(msg[(size_t)m * N + j], q), q) + as[j] +
                             lift(e[j], q);
                c0[j] = (uint32_t)(v % q);
                c1[j] = a[j] ? q - a[j] : 0;
            }
        }
    });
    return HYENA_OK;
}

// RNS decryption (Halevi, Polyakov & Shoup, CT-RSA 2019): with v the CRT
// value of the residues v_i and y_i = (q/q_i)^{-1} mod q_i,
//   t v / q = sum_i v_i t y_i / q_i  (mod t).
// Each term splits into an integer part v_i A_i and a fraction v_i B_i / q_i
// (A_i, B_i the quotient and remainder of t y_i by q_i); with
// F_i = floor(2^64 B_i / q_i) the fraction is taken as v_i F_i / 2^64, a 96-bit
// product, short of it by less than v_i 2^-64 < 2^-33, and the terms are
// summed in 32.64 fixed point (the sum short by less than L 2^-33).
extern "C" int hyena_decrypt(const hyena_ctx *c, const int8_t *sk, const uint32_t *ct, size_t n,
                             int32_t *msg) {
    if (!c || !sk || (n && (!msg || !ct))) return set_error(HYENA_EINVAL, "hyena_decrypt: NULL argument");
    const uint32_t N = c->N, L = c->L;
    const uint64_t t = 1ull << c->log2_t;
    const auto s_hat = secret_ntt(c, sk);
    std::vector<uint64_t> A(L), F(L);
    bfv_hps_constants(c, A.data(), F.data());
    for (size_t k = 0; k < n * L; k++) {
        const uint32_t q = c->q[k % L];
        for (uint32_t j = 0; j < N; j++)
            if (ct[(k / L * 2) * L * N + (k % L) * N + j] >= q || ct[(k / L * 2 + 1) * L * N + (k % L) * N + j] >= q)
                return set_error(HYENA_EINVAL, "hyena_decrypt: residue not below its prime");
    }
    parallel_for(n, [&](size_t m) {
        std::vector<uint32_t> v((size_t)L * N);
        for (uint32_t i = 0; i < L; i++) {
            const uint32_t q = c->q[i];
            const uint32_t *c0 = ct + (((size_t)m * 2 + 0) * L + i) * N;
            const uint32_t *c1 = ct + (((size_t)m * 2 + 1) * L + i) * N;
            uint32_t *vi = &v[(size_t)i * N];
            std::memcpy(vi, c1, sizeof(uint32_t) * N);
            host_ntt(c, i, vi);
            for (uint32_t j = 0; j < N; j++) vi[j] = h_mulmod(vi[j], s_hat[(size_t)i * N + j], q);
            host_intt(c, i, vi);
            for (uint32_t j = 0; j < N; j++) {
                uint32_t s = vi[j] + c0[j];
                vi[j] = s >= q || s < c0[j] ? s - q : s;
            }
        }
        for (uint32_t j = 0; j < N; j++) {
            uint64_t ipart = 0, frac = 0;   // integer part (mod 2^64) and 0.64 fraction
            for (uint32_t i = 0; i < L; i++) {
                const uint64_t vi = v[(size_t)i * N + j];
                ipart += vi * A[i];
                const unsigned __int128 p = (unsigned __int128)vi * F[i];   // < 2^95
                const uint64_t lo = (uint64_t)p;
                ipart += (uint64_t)(p >> 64);
                frac += lo;
                ipart += frac < lo;                      // carry of the fraction sum
            }
            uint64_t r = (ipart + (frac >> 63)) & (t - 1);   // round half up
            int64_t sr = (int64_t)r;
            if (r > t / 2) sr -= (int64_t)t;
            msg[(size_t)m * N + j] = (int32_t)sr;
        }
    });
    return HYENA_OK;
}

// Key-switching key for s(X^g) -> s with digits in base 2^log2_base (RNS-BV):
// key (i, j) = (a s + e + [k == i] s(X^g) 2^(j log2_base), -a) on every limb k,
// a and e drawn as for the encryption of message number i D + j.
extern "C" int hyena_galois_keygen(const hyena_ctx *c, const int8_t *sk, uint32_t g, uint32_t log2_base,
                                   uint64_t seed, uint32_t *ksk) {
    if (!c || !sk || !ksk) return set_error(HYENA_EINVAL, "hyena_galois_keygen: NULL argument");
    if (!(g & 1)) return set_error(HYENA_EINVAL, "hyena_galois_keygen: g must be odd");
    if (log2_base < 1 || log2_base > 29) return set_error(HYENA_EINVAL, "hyena_galois_keygen: log2_base must be in [1, 29]");
    const uint32_t N = c->N, L = c->L, D = (31 + log2_base - 1) / log2_base;
    // s(X^g): coefficient j moves to j g mod 2N, negated past N
    std::vector<int> sg(N, 0);
    for (uint32_t j = 0; j < N; j++) {
        const uint64_t e = (uint64_t)j * g % (2 * N);
        if (e < N) sg[e] += sk[j];
        else sg[e - N] -= sk[j];
    }
    const auto s_hat = secret_ntt(c, sk);
    const Cdt &gs = cdt();
    parallel_for((size_t)L * D, [&](size_t key) {
        const uint32_t i = (uint32_t)(key / D), j = (uint32_t)(key % D);
        std::vector<int> e(N);
        for (uint32_t x = 0; x < N; x++) e[x] = gs.sample(sm64(seed, 2 * ((uint64_t)key * N + x) + 1));
        std::vector<uint32_t> a(N), as(N);
        for (uint32_t k = 0; k < L; k++) {
            const uint32_t q = c->q[k];
            for (uint32_t x = 0; x < N; x++) a[x] = uniform_mod(sm64(seed, 2 * (((uint64_t)key * L + k) * N + x)), q);
            as = a;
            host_ntt(c, k, as.data());
            for (uint32_t x = 0; x < N; x++) as[x] = h_mulmod(as[x], s_hat[(size_t)k * N + x], q);
            host_intt(c, k, as.data());
            const uint32_t pw = (uint32_t)((((unsigned __int128)1) << (log2_base * j)) % q);
            uint32_t *b0 = ksk + ((key * 2 + 0) * L + k) * (size_t)N;
            uint32_t *b1 = ksk + ((key * 2 + 1) * L + k) * (size_t)N;
            for (uint32_t x = 0; x < N; x++) {
                uint64_t v = (uint64_t)as[x] + lift(e[x], q);
                if (k == i) v += h_mulmod(lift(sg[x], q), pw, q);
                b0[x] = (uint32_t)(v % q);
                b1[x] = a[x] ? q - a[x] : 0;
            }
        }
    });
    return HYENA_OK;
}
