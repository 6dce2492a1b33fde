// Internal declarations of the gfx950 Hyena library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "hyena.h"

#define HYENA_MAX_LIMBS 16
#define HYENA_MAX_SEGS 48

// Per-limb constants, passed to kernels by value.
struct LimbConst {
    uint32_t q;        // prime modulus, 2^29 < q < 2^31
    uint32_t r32;      // 2^32 mod q
    uint32_t qinv_neg; // -q^{-1} mod 2^32 (Montgomery)
    uint32_t ninv;     // N^{-1} mod q
    uint32_t ninv_m;   // N^{-1} 2^32 mod q (Montgomery form)
    uint32_t fold;     // products that fit between two folds of a lazy accumulator
    uint32_t nofold;   // products after the last fold the final reduction takes unfolded
    uint32_t r64;      // 2^64 mod q: a Montgomery product by it multiplies by 2^32
    uint32_t w1n_m;    // last inverse-NTT twiddle psi^-brv(1) times N^{-1}, Montgomery form
};

struct LimbTable {
    LimbConst c[HYENA_MAX_LIMBS];
};

struct hyena_ctx {
    uint32_t N = 0, L = 0, logN = 0, log2_t = 0, flags = 0;
    int device = 0;
    std::vector<uint32_t> q, psi;
    LimbTable lt{};
    uint32_t fold_min = 1;   // minimum of lt.c[i].fold
    bool lazy_ntt = false;   // every q_i < 2^30: NTT butterflies may run lazily
    // host twiddles (for the host-side NTT used by test-setup encryption)
    std::vector<uint32_t> h_fw, h_iw;  // [L][N]
    // device twiddles in Montgomery form (w 2^32 mod q): forward psi powers
    // in bit-reversed order, inverse psi^-1 powers likewise.  [L][N]
    uint32_t *d_fw = nullptr;
    uint32_t *d_iw = nullptr;
};

// error reporting
int set_error(int code, const std::string &msg);
// Record this device's address of the no-allocation workspace (client.hip);
// hyena_create calls it with the context's device current.
int client_scratch_setup(int device);
#define HIP_TRY(expr)                                                          \
    do {                                                                       \
        hipError_t _e = (expr);                                                \
        if (_e != hipSuccess)                                                  \
            return set_error(HYENA_EHIP, std::string(#expr) + ": " +          \
                                             hipGetErrorString(_e));           \
    } while (0)

// modular helpers (host)
static inline uint32_t h_mulmod(uint32_t a, uint32_t b, uint32_t q) {
    return (uint32_t)((uint64_t)a * b % q);
}
// x 2^32 mod q: the Montgomery form the device NTT multiplies by
static inline uint32_t to_montgomery(uint32_t x, uint32_t q) {
    return (uint32_t)(((uint64_t)x << 32) % q);
}
uint32_t h_powmod(uint32_t b, uint64_t e, uint32_t q);
uint32_t bit_reverse(uint32_t x, uint32_t logn);

// host NTT (same transform as the device one), used by test-setup crypto
void host_ntt(const hyena_ctx *ctx, uint32_t limb, uint32_t *a);
void host_intt(const hyena_ctx *ctx, uint32_t limb, uint32_t *a);

// launchers shared by translation units
int launch_ntt(const hyena_ctx *ctx, uint32_t *d_poly, size_t P, bool inverse, hipStream_t s);
int launch_ntt_sched(const hyena_ctx *c, uint32_t *d, size_t P, bool inv, int sched, hipStream_t s);
int launch_ntt_segs(const hyena_ctx *c, uint32_t *const *ptrs, const size_t *P, uint32_t nseg, bool inv,
                    int sched, hipStream_t s);
int ntt_default_schedule(uint32_t logN);
