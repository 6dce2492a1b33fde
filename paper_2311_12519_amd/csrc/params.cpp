// Context creation: RNS primes, roots, twiddle tables and per-limb constants.
//
// Ring R_q = Z_q[X]/(X^N+1) with q = prod q_i (the "Homomorphic Operations in BFV" section). The negacyclic NTT
// needs q_i = 1 mod 2N (the "Optimal Parameter Selection" section, parameter-selection step 1); psi_i is the
// smallest integer >= 2 with psi_i^N = -1 mod q_i.
#include <cstring>
#include <cmath>
#include <mutex>

#include "internal.h"

static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

extern "C" const char *hyena_last_error(void) { return g_last_error.c_str(); }

uint32_t h_powmod(uint32_t b, uint64_t e, uint32_t q) {
    uint64_t r = 1 % q, x = b % q;
    while (e) {
        if (e & 1) r = r * x % q;
        x = x * x % q;
        e >>= 1;
    }
    return (uint32_t)r;
}

uint32_t bit_reverse(uint32_t x, uint32_t logn) {
    uint32_t r = 0;
    for (uint32_t i = 0; i < logn; i++) r = (r << 1) | ((x >> i) & 1u);
    return r;
}

// Deterministic Miller-Rabin for n < 2^32 (bases 2, 7, 61).
static bool is_prime_u32(uint32_t n) {
    if (n < 2) return false;
    for (uint32_t p : {2u, 3u, 5u, 7u, 11u, 13u}) {
        if (n % p == 0) return n == p;
    }
    uint32_t d = n - 1, s = 0;
    while (!(d & 1)) { d >>= 1; s++; }
    for (uint32_t a : {2u, 7u, 61u}) {
        if (a % n == 0) continue;
        uint64_t x = h_powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (uint32_t r = 1; r < s; r++) {
            x = x * x % n;
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

static const struct { uint32_t N, logq; } kSecurity128[] = {
    {1024, 27}, {2048, 54}, {4096, 109}, {8192, 218}, {16384, 438}};

static uint32_t security_ceiling(uint32_t N) {
    for (auto &e : kSecurity128)
        if (e.N == N) return e.logq;
    return 0;
}

static void build_tables(hyena_ctx *c) {
    const uint32_t N = c->N;
    c->h_fw.assign((size_t)c->L * N, 0);
    c->h_iw.assign((size_t)c->L * N, 0);
    for (uint32_t i = 0; i < c->L; i++) {
        const uint32_t q = c->q[i], psi = c->psi[i];
        const uint32_t psi_inv = h_powmod(psi, q - 2, q);
        // powers psi^k and psi^-k in natural order, then bit-reversed placement
        std::vector<uint32_t> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (uint32_t k = 1; k < N; k++) {
            pw[k] = h_mulmod(pw[k - 1], psi, q);
            ipw[k] = h_mulmod(ipw[k - 1], psi_inv, q);
        }
        for (uint32_t k = 0; k < N; k++) {
            uint32_t r = bit_reverse(k, c->logN);
            c->h_fw[(size_t)i * N + k] = pw[r];
            c->h_iw[(size_t)i * N + k] = ipw[r];
        }
        LimbConst &lc = c->lt.c[i];
        lc.q = q;
        lc.r32 = (uint32_t)((1ull << 32) % q);
        uint32_t inv = 1;  // Newton iteration for q^{-1} mod 2^32
        for (int it = 0; it < 5; it++) inv *= 2u - q * inv;
        lc.qinv_neg = 0u - inv;
        lc.ninv = h_powmod(N, q - 2, q);
        lc.ninv_m = to_montgomery(lc.ninv, q);
        lc.w1n_m = to_montgomery(h_mulmod(c->h_iw[(size_t)i * N + 1], lc.ninv, q), q);
        // After a fold the accumulator is < 2^32 (r32 + 1); each product is
        // <= (q-1)^2. Products that fit before the next fold:
        unsigned __int128 room = (((unsigned __int128)1) << 64) - 1 -
                                 (((unsigned __int128)(lc.r32 + 1ull)) << 32);
        unsigned __int128 f = room / ((unsigned __int128)(q - 1) * (q - 1));
        lc.fold = (uint32_t)(f > 15 ? 15 : (f < 1 ? 1 : f));
        // Unfolded products after the last fold that the final Montgomery
        // reduction still takes without a fold of its own: its input must stay
        // below q 2^32 (at most fold - 1 are ever left over)
        unsigned __int128 redc_room = (((unsigned __int128)q) << 32) - 1 -
                                      (((unsigned __int128)(lc.r32 + 1ull)) << 32);
        unsigned __int128 nf = redc_room / ((unsigned __int128)(q - 1) * (q - 1));
        lc.nofold = (uint32_t)(nf > lc.fold - 1 ? lc.fold - 1 : nf);
        lc.r64 = (uint32_t)((((unsigned __int128)1) << 64) % q);
    }
    c->lazy_ntt = true;
    for (uint32_t i = 0; i < c->L; i++)
        if (c->q[i] >= (1u << 30)) c->lazy_ntt = false;
    c->fold_min = 15;
    for (uint32_t i = 0; i < c->L; i++)
        if (c->lt.c[i].fold < c->fold_min) c->fold_min = c->lt.c[i].fold;
}

extern "C" int hyena_create(uint32_t N, uint32_t L, const uint32_t *primes, uint32_t log2_t,
                            uint32_t flags, hyena_ctx **out) {
    if (!out) return set_error(HYENA_EINVAL, "hyena_create: out is NULL");
    *out = nullptr;
    if (N < 1024 || N > 16384 || (N & (N - 1)))
        return set_error(HYENA_EUNSUPPORTED, "hyena_create: N must be a power of two in [1024, 16384]");
    if (L < 1 || L > HYENA_MAX_LIMBS)
        return set_error(HYENA_EUNSUPPORTED, "hyena_create: L must be in [1, 16]");
    if (log2_t < 1 || log2_t > 30)
        return set_error(HYENA_EUNSUPPORTED, "hyena_create: log2_t must be in [1, 30]");
    auto *c = new (std::nothrow) hyena_ctx();
    if (!c) return set_error(HYENA_ENOMEM, "hyena_create: out of host memory");
    c->N = N;
    c->L = L;
    c->log2_t = log2_t;
    c->flags = flags;
    while ((1u << c->logN) < N) c->logN++;
    if (primes) {
        for (uint32_t i = 0; i < L; i++) {
            uint32_t q = primes[i];
            const uint32_t lo = (flags & HYENA_PLAINTEXT_PRIME) ? 2u : (1u << 29);
            if (q <= lo || q >= (1u << 31) || q % (2 * N) != 1 || !is_prime_u32(q)) {
                delete c;
                return set_error(HYENA_EUNSUPPORTED,
                                 "hyena_create: prime " + std::to_string(q) +
                                     " is not a prime in (" + (lo == 2 ? "2" : "2^29") +
                                     ", 2^31) with q = 1 mod 2N");
            }
            for (uint32_t j = 0; j < i; j++)
                if (primes[j] == q) {
                    delete c;
                    return set_error(HYENA_EINVAL, "hyena_create: primes must be distinct");
                }
            c->q.push_back(q);
        }
    } else if (flags & HYENA_PLAINTEXT_PRIME) {
        delete c;
        return set_error(HYENA_EINVAL, "hyena_create: HYENA_PLAINTEXT_PRIME needs the prime");
    } else {
        const uint32_t bits = (flags & HYENA_PRIMES_30BIT) ? 30 : 31;
        uint64_t q = ((1ull << bits) - 1) / (2 * N) * (2 * N) + 1;
        while (c->q.size() < L) {
            if (q < (1ull << bits) && is_prime_u32((uint32_t)q)) c->q.push_back((uint32_t)q);
            q -= 2 * N;
            if (q <= (1u << 29)) {
                delete c;
                return set_error(HYENA_EUNSUPPORTED, "hyena_create: ran out of primes");
            }
        }
    }
    if (!(flags & (HYENA_ALLOW_INSECURE | HYENA_PLAINTEXT_PRIME))) {
        double logq = 0;
        for (uint32_t q : c->q) logq += std::log2((double)q);
        uint32_t ceil = security_ceiling(N);
        if (logq > (double)ceil) {
            delete c;
            return set_error(HYENA_EUNSUPPORTED,
                             "hyena_create: log2 q = " + std::to_string(logq) +
                                 " exceeds the 128-bit ceiling " + std::to_string(ceil) +
                                 " for N = " + std::to_string(N));
        }
    }
    for (uint32_t q : c->q) {
        uint32_t x = 2;
        while (h_powmod(x, N, q) != q - 1) x++;
        c->psi.push_back(x);
    }
    build_tables(c);

    if (flags & HYENA_HOST_ONLY) {
        *out = c;
        return HYENA_OK;
    }
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) {
        if (int rc = client_scratch_setup(c->device)) {
            hyena_destroy(c);
            return rc;
        }
    }
    const size_t bytes = sizeof(uint32_t) * (size_t)L * N;
    if (e == hipSuccess) e = hipMalloc((void **)&c->d_fw, bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&c->d_iw, bytes);
    if (e == hipSuccess) {
        std::vector<uint32_t> fw((size_t)L * N), iw((size_t)L * N);
        for (uint32_t i = 0; i < L; i++)
            for (size_t k = 0; k < N; k++) {
                fw[(size_t)i * N + k] = to_montgomery(c->h_fw[(size_t)i * N + k], c->q[i]);
                iw[(size_t)i * N + k] = to_montgomery(c->h_iw[(size_t)i * N + k], c->q[i]);
            }
        e = hipMemcpy(c->d_fw, fw.data(), bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->d_iw, iw.data(), bytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        std::string msg = std::string("hyena_create: ") + hipGetErrorString(e);
        hyena_destroy(c);
        return set_error(e == hipErrorOutOfMemory ? HYENA_ENOMEM : HYENA_EHIP, msg);
    }
    *out = c;
    return HYENA_OK;
}

extern "C" void hyena_destroy(hyena_ctx *c) {
    if (!c) return;
    if (c->d_fw) (void)hipFree(c->d_fw);
    if (c->d_iw) (void)hipFree(c->d_iw);
    delete c;
}

extern "C" int hyena_get_params(const hyena_ctx *c, uint32_t *N, uint32_t *L, uint32_t *primes,
                                uint32_t *psi) {
    if (!c) return set_error(HYENA_EINVAL, "hyena_get_params: ctx is NULL");
    if (N) *N = c->N;
    if (L) *L = c->L;
    for (uint32_t i = 0; i < c->L; i++) {
        if (primes) primes[i] = c->q[i];
        if (psi) psi[i] = c->psi[i];
    }
    return HYENA_OK;
}

// Host negacyclic NTT: Cooley-Tukey butterflies with psi powers in
// bit-reversed order (output in bit-reversed order); the inverse uses
// Gentleman-Sande butterflies and the factor N^{-1}.
void host_ntt(const hyena_ctx *c, uint32_t limb, uint32_t *a) {
    const uint32_t N = c->N, q = c->q[limb];
    const uint32_t *tw = &c->h_fw[(size_t)limb * N];
    uint32_t t = N;
    for (uint32_t m = 1; m < N; m <<= 1) {
        t >>= 1;
        for (uint32_t i = 0; i < m; i++) {
            const uint32_t w = tw[m + i];
            uint32_t *x = a + 2 * i * t;
            for (uint32_t j = 0; j < t; j++) {
                uint32_t u = x[j], v = h_mulmod(x[j + t], w, q);
                uint32_t s = u + v;
                x[j] = s >= q ? s - q : s;
                x[j + t] = u >= v ? u - v : u + q - v;
            }
        }
    }
}

void host_intt(const hyena_ctx *c, uint32_t limb, uint32_t *a) {
    const uint32_t N = c->N, q = c->q[limb];
    const uint32_t *tw = &c->h_iw[(size_t)limb * N];
    uint32_t t = 1;
    for (uint32_t m = N; m > 1; m >>= 1) {
        const uint32_t h = m >> 1;
        for (uint32_t i = 0; i < h; i++) {
            const uint32_t w = tw[h + i];
            uint32_t *x = a + 2 * i * t;
            for (uint32_t j = 0; j < t; j++) {
                uint32_t u = x[j], v = x[j + t];
                uint32_t s = u + v;
                x[j] = s >= q ? s - q : s;
                x[j + t] = h_mulmod(u >= v ? u - v : u + q - v, w, q);
            }
        }
        t <<= 1;
    }
    const uint32_t ninv = c->lt.c[limb].ninv;
    for (uint32_t j = 0; j < N; j++) a[j] = h_mulmod(a[j], ninv, q);
}
