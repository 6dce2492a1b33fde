// Batched BFV encryption and decryption on gfx950 (the client side of the
// "Homomorphic Operations in BFV" section): the same ciphertexts and messages
// as the host hyena_encrypt / hyena_decrypt, for many messages per call, with
// every step in device kernels and the library's NTT.
//
// Encryption of message m (limb i, coefficient j), NTT(s) prepared once:
//   a  = floor(q_i sm64(seed, 2((m L + i) N + j)) / 2^64)
//   c1 = [-a]_{q_i},  c0 = [Delta_i lift(msg) + INTT(NTT(a) . NTT(s)) + lift(e)]_{q_i}
// with e the rounded Gaussian drawn from sm64(seed, 2(m N + j) + 1).
// Decryption: v = [c0 + INTT(NTT(c1) . NTT(s))]_{q_i}, then the RNS rounding of
// t v / q of Halevi, Polyakov and Shoup, in the same integer steps as the host
// (fractions in 0.64 fixed point).
#include <mutex>

#include "bfv.h"

namespace {

constexpr uint32_t CTH = 256;   // threads per block; one block covers 256 coefficients

static_assert((kErrBound & (kErrBound - 1)) == 0 && 2 * kErrBound <= CTH, "sampler search over 2B thresholds");

struct Thresholds {
    uint64_t t[2 * kErrBound];
};

struct ClientConst {
    uint32_t dm[HYENA_MAX_LIMBS];   // Delta_i 2^32 mod q_i (Montgomery form)
    uint64_t A[HYENA_MAX_LIMBS];    // floor(t y_i / q_i)
    uint64_t F[HYENA_MAX_LIMBS];    // floor(2^64 (t y_i mod q_i) / q_i)
};

__device__ __forceinline__ uint32_t ccsub(uint32_t x, uint32_t q) { return min(x, x - q); }

// a b 2^-32 mod q in [0, q) for a, b < q
__device__ __forceinline__ uint32_t cmont(uint32_t a, uint32_t b, const LimbConst &lc) {
    const uint64_t t = (uint64_t)a * b;
    const uint32_t m = (uint32_t)t * lc.qinv_neg;
    return ccsub((uint32_t)(((uint64_t)m * lc.q + t) >> 32), lc.q);
}

__device__ __forceinline__ uint32_t caddmod(uint32_t a, uint32_t b, uint32_t q) { return ccsub(a + b, q); }

// x mod q for any int32 x (the host's lift); no division when |x| < q
__device__ __forceinline__ uint32_t clift(int32_t x, uint32_t q) {
    const uint32_t a = x >= 0 ? (uint32_t)x : (uint32_t)(-(int64_t)x);
    const uint32_t r = a < q ? a : a % q;
    return x >= 0 || r == 0 ? r : q - r;
}


// Blocks walk chunks of 256 coefficients; chunk c of a [P][L][N] array is
// coefficients (c mod N/256) 256 ... + 255 of limb-polynomial c / (N/256).

__global__ void __launch_bounds__(CTH) lift_secret_kernel(const int8_t *sk, uint32_t *s, uint32_t logN, uint32_t L,
                                                          LimbTable lt) {
    const uint32_t N = 1u << logN;
    for (uint32_t c = blockIdx.x; c < (L << (logN - 8)); c += gridDim.x) {
        const uint32_t i = c >> (logN - 8), j = ((c << 8) & (N - 1)) + threadIdx.x;
        const int32_t v = sk[j];
        const uint32_t q = lt.c[i].q;
        s[(size_t)i * N + j] = v >= 0 ? (uint32_t)v : q - (uint32_t)(-v);
    }
}

// s <- s 2^32 mod q (a Montgomery product by 2^64 mod q)
__global__ void __launch_bounds__(CTH) to_montgomery_kernel(uint32_t *s, uint32_t logN, uint32_t L, LimbTable lt) {
    for (uint32_t c = blockIdx.x; c < (L << (logN - 8)); c += gridDim.x) {
        const uint32_t i = c >> (logN - 8);
        const LimbConst lc = lt.c[i];
        uint32_t *p = s + ((size_t)c << 8) + threadIdx.x;
        *p = cmont(*p, lc.r64, lc);
    }
}

// c0 <- [Delta_i lift(msg) + work + lift(e)]_{q_i} (work = a s); e drawn once per (m, j) for all limbs
__global__ void __launch_bounds__(CTH) encrypt_finish_kernel(uint32_t *ct, const uint32_t *work, const int32_t *msg,
                                                             size_t n, uint32_t logN, uint32_t L, uint64_t seed,
                                                             LimbTable lt, ClientConst cc, Thresholds th) {
    __shared__ uint64_t thr[2 * kErrBound];
    if (threadIdx.x < 2 * kErrBound) thr[threadIdx.x] = th.t[threadIdx.x];
    __syncthreads();
    const uint32_t cpl = 1u << (logN - 8);
    const size_t LN = (size_t)L << logN, chunks = n * cpl;
    for (size_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const size_t m = c >> (logN - 8);
        const size_t mj = (c << 8) + threadIdx.x;      // m N + j
        const uint32_t j = (uint32_t)(mj & ((1u << logN) - 1));
        const uint64_t u = hy_sm64(seed, 2 * (uint64_t)mj + 1) >> 1;
        // #{k < 2B : u >= T[k]}: the thresholds are nondecreasing, so the count
        // is the length of the prefix below u, found by binary search
        uint32_t cnt = 0;
#pragma unroll
        for (uint32_t step = kErrBound; step >= 1; step >>= 1)
            if (u >= thr[cnt + step - 1]) cnt += step;
        if (cnt == 2 * kErrBound - 1 && u >= thr[2 * kErrBound - 1]) cnt++;
        const int32_t e = (int32_t)cnt - kErrBound;
        const int32_t x = msg[mj];
        uint32_t ws[HYENA_MAX_LIMBS];   // loaded together, as in decrypt_finish_kernel
#pragma unroll
        for (uint32_t i = 0; i < HYENA_MAX_LIMBS; i++)
            if (i < L) ws[i] = work[m * LN + ((size_t)i << logN) + j];
#pragma unroll
        for (uint32_t i = 0; i < HYENA_MAX_LIMBS; i++) {
            if (i >= L) break;
            const LimbConst lc = lt.c[i];
            const uint32_t q = lc.q;
            const size_t r = ((size_t)i << logN) + j;
            const uint32_t dm = cmont(cc.dm[i], clift(x, q), lc);
            const uint32_t le = e >= 0 ? (uint32_t)e : q - (uint32_t)(-e);
            ct[m * 2 * LN + r] = caddmod(caddmod(dm, ws[i], q), le, q);
        }
    }
}

// msg <- round(t v / q) mod t, centered, v = work = [c0 + c1 s]_q; the host decryption's integer steps
__global__ void __launch_bounds__(CTH) decrypt_finish_kernel(const uint32_t *work, int32_t *msg,
                                                             size_t n, uint32_t logN, uint32_t L, uint32_t log2_t,
                                                             ClientConst cc) {
    const uint32_t cpl = 1u << (logN - 8);
    const size_t LN = (size_t)L << logN, chunks = n * cpl;
    const uint32_t t = 1u << log2_t;
    for (size_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const size_t m = c >> (logN - 8);
        const size_t mj = (c << 8) + threadIdx.x;
        const uint32_t j = (uint32_t)(mj & ((1u << logN) - 1));
        // integer part mod 2^32 (t divides it) and the 0.64 fraction, as the
        // host sums them: per limb v A_i + v F_i / 2^64, v F_i a 96-bit product
        // the limbs' words are loaded before any of them is used, so that
        // their loads are in flight together
        uint32_t vs[HYENA_MAX_LIMBS];
#pragma unroll
        for (uint32_t i = 0; i < HYENA_MAX_LIMBS; i++)
            if (i < L) vs[i] = work[m * LN + ((size_t)i << logN) + j];   // c0 + c1 s mod q_i
        uint32_t ipart = 0;
        uint64_t frac = 0;
#pragma unroll
        for (uint32_t i = 0; i < HYENA_MAX_LIMBS; i++) {
            if (i >= L) break;
            const uint32_t v = vs[i];
            const uint64_t a = (uint64_t)v * (uint32_t)cc.F[i];          // v F_lo
            const uint64_t b = (uint64_t)v * (uint32_t)(cc.F[i] >> 32);  // v F_hi
            const uint64_t lo = a + (b << 32);                           // low 64 bits of v F
            ipart += v * (uint32_t)cc.A[i] + (uint32_t)(b >> 32) + (lo < a);
            frac += lo;
            ipart += frac < lo;
        }
        const uint32_t rr = (ipart + (uint32_t)(frac >> 63)) & (t - 1);
        msg[mj] = rr > t / 2 ? (int32_t)rr - (int32_t)t : (int32_t)rr;
    }
}

unsigned grid_for(size_t chunks) { return (unsigned)std::min<size_t>(chunks, 8192); }

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return na && nb && a0 < b0 + nb && b0 < a0 + na;
}

int check_ctx(const hyena_ctx *c, const char *who) {
    if (!c->d_fw) return set_error(HYENA_EINVAL, std::string(who) + ": context was created host-only");
    if (c->logN < 8) return set_error(HYENA_EUNSUPPORTED, std::string(who) + ": N below 256");
    return HYENA_OK;
}

int launched(const char *who) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string(who) + ": " + hipGetErrorString(e));
    return HYENA_OK;
}

ClientConst client_constants(const hyena_ctx *c) {
    ClientConst cc{};
    const auto delta = bfv_delta_residues(c);
    bfv_hps_constants(c, cc.A, cc.F);
    for (uint32_t i = 0; i < c->L; i++) cc.dm[i] = to_montgomery(delta[i], c->q[i]);
    return cc;
}

// Workspace of hyena_decrypt_device_noalloc: a file-scope device array that
// every GPU the library runs on holds for the life of the process (its own
// copy, at its own address). Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): it uses the
// device address that hipGetSymbolAddress returned for the device, recorded
// once per device when a context is created on it.
__device__ __align__(256) uint32_t scratch[HYENA_NOALLOC_SCRATCH_WORDS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch[kMaxDevices] = {};

uint32_t *scratch_for(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[device];
}

}  // namespace

// Called by hyena_create with the context's device current.
int client_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices)
        return set_error(HYENA_EUNSUPPORTED, "hyena_create: device index above the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return HYENA_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(HYENA_EHIP, std::string("hyena_create: scratch address: ") + hipGetErrorString(e));
    g_scratch[device] = (uint32_t *)p;
    return HYENA_OK;
}

extern "C" int hyena_secret_prepare(const hyena_ctx *c, const int8_t *d_sk, uint32_t *d_s_hat, hyena_stream_t stream) {
    static const char *who = "hyena_secret_prepare";
    if (!c || !d_sk || !d_s_hat) return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = check_ctx(c, who)) return rc;
    if (overlaps(d_sk, c->N, d_s_hat, (size_t)c->L * c->N * 4))
        return set_error(HYENA_EINVAL, std::string(who) + ": d_s_hat overlaps d_sk");
    const hipStream_t s = (hipStream_t)stream;
    const size_t chunks = (size_t)c->L << (c->logN - 8);
    hipLaunchKernelGGL(lift_secret_kernel, dim3(grid_for(chunks)), dim3(CTH), 0, s, d_sk, d_s_hat, c->logN, c->L, c->lt);
    if (int rc = launched(who)) return rc;
    if (int rc = launch_ntt(c, d_s_hat, 1, false, s)) return rc;
    hipLaunchKernelGGL(to_montgomery_kernel, dim3(grid_for(chunks)), dim3(CTH), 0, s, d_s_hat, c->logN, c->L, c->lt);
    return launched(who);
}

extern "C" int hyena_encrypt_device(const hyena_ctx *c, const uint32_t *d_s_hat, const int32_t *d_msg, size_t n,
                                    uint64_t seed, uint32_t *d_work, uint32_t *d_ct, hyena_stream_t stream) {
    static const char *who = "hyena_encrypt_device";
    if (!c || !d_s_hat || (n && (!d_msg || !d_work || !d_ct)))
        return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = check_ctx(c, who)) return rc;
    if (n == 0) return HYENA_OK;
    const uint32_t N = c->N, L = c->L;
    const size_t LN = (size_t)L * N;
    if (n > (((size_t)1 << 31) - 1) / L) return set_error(HYENA_EINVAL, std::string(who) + ": too many messages");
    if ((uintptr_t)d_work & 15u) return set_error(HYENA_EINVAL, std::string(who) + ": d_work is not 16-byte aligned");
    const size_t ct_bytes = n * 2 * LN * 4, work_bytes = n * LN * 4, msg_bytes = n * N * 4;
    if (overlaps(d_ct, ct_bytes, d_msg, msg_bytes) || overlaps(d_ct, ct_bytes, d_s_hat, LN * 4) ||
        overlaps(d_work, work_bytes, d_ct, ct_bytes) || overlaps(d_work, work_bytes, d_msg, msg_bytes) ||
        overlaps(d_work, work_bytes, d_s_hat, LN * 4))
        return set_error(HYENA_EINVAL, std::string(who) + ": d_work or d_ct overlaps another array");
    const hipStream_t s = (hipStream_t)stream;
    const ClientConst cc = client_constants(c);
    Thresholds th;
    bfv_error_thresholds(th.t);
    for (int k = 0; k + 1 < 2 * kErrBound; k++)   // the kernel's binary search relies on it
        if (th.t[k] > th.t[k + 1]) return set_error(HYENA_EINVAL, std::string(who) + ": sampler table not monotone");
    // a drawn inside the transform, which writes c1 = -a and a s into the workspace
    if (int rc = launch_ntt_sample_as(c, d_ct, n, d_work, d_s_hat, seed, s)) return rc;
    const size_t fchunks = n << (c->logN - 8);
    hipLaunchKernelGGL(encrypt_finish_kernel, dim3(grid_for(fchunks)), dim3(CTH), 0, s, d_ct, d_work, d_msg, n,
                       c->logN, L, seed, c->lt, cc, th);
    return launched(who);
}

extern "C" int hyena_decrypt_device(const hyena_ctx *c, const uint32_t *d_s_hat, const uint32_t *d_ct, size_t n,
                                    uint32_t *d_work, int32_t *d_msg, hyena_stream_t stream) {
    static const char *who = "hyena_decrypt_device";
    if (!c || !d_s_hat || (n && (!d_ct || !d_work || !d_msg)))
        return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = check_ctx(c, who)) return rc;
    if (n == 0) return HYENA_OK;
    const uint32_t N = c->N, L = c->L;
    const size_t LN = (size_t)L * N;
    if (n > (((size_t)1 << 31) - 1) / L) return set_error(HYENA_EINVAL, std::string(who) + ": too many ciphertexts");
    if ((uintptr_t)d_work & 15u) return set_error(HYENA_EINVAL, std::string(who) + ": d_work is not 16-byte aligned");
    const size_t work_bytes = n * LN * 4, msg_bytes = n * N * 4;
    if (overlaps(d_work, work_bytes, d_ct, n * 2 * LN * 4) || overlaps(d_work, work_bytes, d_s_hat, LN * 4) ||
        overlaps(d_work, work_bytes, d_msg, msg_bytes) || overlaps(d_msg, msg_bytes, d_ct, n * 2 * LN * 4) ||
        overlaps(d_msg, msg_bytes, d_s_hat, LN * 4))
        return set_error(HYENA_EINVAL, std::string(who) + ": d_work or d_msg overlaps another array");
    const hipStream_t s = (hipStream_t)stream;
    const ClientConst cc = client_constants(c);
    // v = c0 + INTT(NTT(c1) . NTT(s)) into the workspace, one kernel per limb-polynomial
    if (int rc = launch_ntt_c1s_add(c, d_ct, n, d_work, d_s_hat, s)) return rc;
    const size_t fchunks = n << (c->logN - 8);
    hipLaunchKernelGGL(decrypt_finish_kernel, dim3(grid_for(fchunks)), dim3(CTH), 0, s, d_work, d_msg, n, c->logN,
                       L, c->log2_t, cc);
    return launched(who);
}

extern "C" int hyena_decrypt_device_noalloc(const hyena_ctx *c, const uint32_t *d_s_hat, const uint32_t *d_ct,
                                            size_t n, int32_t *d_msg, hyena_stream_t stream) {
    static const char *who = "hyena_decrypt_device_noalloc";
    if (!c) return set_error(HYENA_EINVAL, std::string(who) + ": NULL argument");
    if (int rc = check_ctx(c, who)) return rc;
    if ((size_t)c->L * c->N > HYENA_NOALLOC_SCRATCH_WORDS ||
        n > HYENA_NOALLOC_SCRATCH_WORDS / ((size_t)c->L * c->N))
        return set_error(HYENA_EINVAL, std::string(who) + ": n * L * N above the scratch size of " +
                                           std::to_string(HYENA_NOALLOC_SCRATCH_WORDS) + " words");
    uint32_t *work = scratch_for(c->device);
    if (!work) return set_error(HYENA_EINVAL, std::string(who) + ": no scratch address for the context's device");
    // the same kernels as hyena_decrypt_device, with this device's scratch as
    // the workspace (it is written whole before it is read: nothing to clear)
    return hyena_decrypt_device(c, d_s_hat, d_ct, n, work, d_msg, stream);
}
