/*
 * hyena.h -- C ABI of the MI355X (gfx950) homomorphic-convolution library.
 *
 * Method: Roh & Choi, "Hyena: Optimizing Homomorphically Encrypted
 * Convolution for Private CNN Inference", ICCAD 2024.
 *
 * The library computes the cloud side of a homomorphically encrypted
 * convolution layer: BFV ciphertexts of coefficient-encoded, zero-padded
 * activation tensors are multiplied by kernel polynomials built from integer
 * weights and summed over input ciphertexts, in Z_q[X]/(X^N+1) with q a
 * product of RNS primes q_i < 2^31, q_i = 1 mod 2N.
 *
 *  - the "Homomorphic Operations in BFV" section: ciphertexts, HAdd, PMult,
 *    CMult; symmetric encryption and decryption (test setup only).
 *  - the "Prior Art on Homomorphic Convolution" section: padded convolution,
 *    weights kept as integers and applied as CMult scalars; the C x H x W
 *    tensor split over ceil(CHW/n) ciphertexts.
 *  - the "Enabling Output Channel Packing" section, Eq. (hadamard2) and its
 *    c_n = 2^k generalisation: output channels handled in groups of c_n
 *    through Walsh-Hadamard weights.
 *  - the "Lazy Reduction" section: products accumulated unreduced in a wide
 *    integer, one reduction per output coefficient.
 *
 * Conventions shared by every call:
 *  - Return 0 (HYENA_OK) on success or a negative HYENA_E* code; the text of
 *    the last error of the calling thread is returned by hyena_last_error().
 *  - Residues are uint32, canonical in [0, q_i). Polynomial arrays are limb
 *    major: [..][L][N], N consecutive coefficients per limb.
 *  - "Host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory on the device that was current at hyena_create. Device calls are
 *    asynchronous on the given stream (0 = the null stream); the caller keeps
 *    every buffer alive until the stream has passed the call.
 *  - The caller allocates and owns every buffer it passes. The library keeps
 *    no caller pointer after a call returns. A context owns its twiddle and
 *    constant tables (device memory) until hyena_destroy; after creation it is
 *    read-only and may be shared by threads and streams.
 *  - No call allocates device memory except hyena_create, hyena_batch_create
 *    and the explicit workspace queries' callers.
 *  - hyena_decrypt_device_noalloc uses a fixed device array of the library
 *    instead of a caller workspace (see its comment).
 */
#ifndef HYENA_H
#define HYENA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *hyena_stream_t; /* identical to hipStream_t */

enum {
    HYENA_OK = 0,
    HYENA_EINVAL = -1,       /* null pointer, bad shape, c_n not a power of two ... */
    HYENA_EUNSUPPORTED = -2, /* N, primes or security level not supported */
    HYENA_ENOISE = -3,       /* worst-case noise or output would break decryption */
    HYENA_EHIP = -4,         /* HIP runtime error */
    HYENA_ENOMEM = -5        /* allocation failure */
};

/* hyena_create flags */
#define HYENA_ALLOW_INSECURE 0x1u /* skip the 128-bit security ceiling on log2 q */
#define HYENA_HOST_ONLY 0x2u      /* no device tables: only the host calls may be used */
#define HYENA_PLAINTEXT_PRIME 0x4u /* primes may be any prime below 2^31 with q = 1 mod 2N:
                                      a context over the SIMD plaintext modulus p (L = 1)
                                      for hyena_simd_encode/decode and the NTT; no
                                      security ceiling applies (it is not a ciphertext
                                      modulus) */

typedef struct hyena_ctx hyena_ctx;

/*
 * Create a context for ring degree N in {4096, 8192, 16384} (any power of two
 * from 1024 to 16384 is accepted) with L RNS limbs and plaintext modulus
 * t = 2^log2_t (1 <= log2_t <= 30).
 *
 * primes: L distinct primes, each 2^29 < q_i < 2^31 and q_i = 1 mod 2N (the
 * NTT condition of the "Optimal Parameter Selection" section, step 1), or NULL for the defaults: the L
 * largest such primes below 2^31 (below 2^30 if flags has bit 0x100,
 * HYENA_PRIMES_30BIT). psi_i is the smallest integer >= 2 with
 * psi_i^N = -1 mod q_i.
 *
 * Unless HYENA_ALLOW_INSECURE is set, sum log2 q_i must not exceed the
 * 128-bit ceiling of the HE security standard for a ternary secret
 * (N = 4096: 109 bits, 8192: 218, 16384: 438); the paper runs its parameters
 * at 128-bit security (the "Evaluation Setup" section).
 *
 * Allocates the device tables on the current HIP device, unless flags has
 * HYENA_HOST_ONLY (then device calls return EINVAL). Errors: EINVAL,
 * EUNSUPPORTED, EHIP, ENOMEM.
 */
#define HYENA_PRIMES_30BIT 0x100u
int hyena_create(uint32_t N, uint32_t L, const uint32_t *primes, uint32_t log2_t,
                 uint32_t flags, hyena_ctx **out);
void hyena_destroy(hyena_ctx *ctx);
const char *hyena_last_error(void);

/* Read back parameters: primes[L] and psi[L] (host arrays, either may be NULL). */
int hyena_get_params(const hyena_ctx *ctx, uint32_t *N, uint32_t *L,
                     uint32_t *primes, uint32_t *psi);

/* ------------------------------------------------------------------------
 * Test setup (host, deterministic by seed); "Homomorphic Operations in BFV".
 * Random numbers: output number c of SplitMix64 seeded with key is
 * mix(key + (c+1) * 0x9E3779B97F4A7C15) (Steele, Lea & Flood 2014).
 * ---------------------------------------------------------------------- */

/* Ternary secret: sk[j] = floor(3 * hi32(sm64(seed, j)) / 2^32) - 1. */
int hyena_keygen(const hyena_ctx *ctx, uint64_t seed, int8_t *sk /* host [N] */);

/*
 * Symmetric BFV encryption of n messages (the "Homomorphic Operations in BFV" section):
 *   c0 = [Delta*m + a*s + e]_q,  c1 = [-a]_q,  Delta = floor(q / t).
 * msg: host int32 [n][N], centered in (-t/2, t/2]. ct: host uint32
 * [n][2][L][N], coefficient domain. a_{m,i,j} = floor(q_i * sm64(seed,
 * 2*((m*L+i)*N+j)) / 2^64); e_{m,j} is the rounded Gaussian, sigma = 3.2,
 * bounded by B = 10 sigma (32), drawn from sm64(seed, 2*(m*N+j)+1) by an
 * integer threshold table. Errors: EINVAL.
 */
int hyena_encrypt(const hyena_ctx *ctx, const int8_t *sk, const int32_t *msg,
                  size_t n, uint64_t seed, uint32_t *ct);

/*
 * Decryption m = [round(t * [c0 + c1 s]_q / q)]_t, centered in (-t/2, t/2].
 * ct: host uint32 [n][2][L][N] coefficient domain; msg: host int32 [n][N].
 * Computed in RNS form (Halevi, Polyakov & Shoup 2019) with the fractions of
 * the L terms taken in 0.64 fixed point (each short by less than 2^-33) and
 * summed with the integer parts: the result is the exact rounding except
 * where the fractional part of t v / q (v = [c0 + c1 s]_q) lies in
 * [1/2, 1/2 + L 2^-33), where it may be one less. So it is exact whenever the
 * noise is below Delta/2 by a margin of L * 2^-33 q/t.
 * hyena_decrypt_device computes the same values. Errors: EINVAL (NULL, a
 * residue not below its prime).
 */
int hyena_decrypt(const hyena_ctx *ctx, const int8_t *sk, const uint32_t *ct,
                  size_t n, int32_t *msg);

/*
 * Batched client operations on the device (the same "Homomorphic Operations in
 * BFV" section): bit for bit the ciphertexts of hyena_encrypt and the messages
 * of hyena_decrypt, for n messages per call, every step in device kernels and
 * the library's NTT. They allocate nothing and are asynchronous on `stream`.
 *
 * hyena_secret_prepare: d_sk device int8 [N] (the secret's coefficients, as
 * from hyena_keygen); d_s_hat device uint32 [L][N], 16-byte aligned, receives
 * 2^32 NTT_i(s) mod q_i, the form the two calls below take. Must not overlap
 * d_sk.
 *
 * hyena_encrypt_device: d_msg device int32 [n][N]; d_work device uint32
 * [n][L][N], 16-byte aligned, overwritten (with a s); d_ct device uint32
 * [n][2][L][N], written whole. d_work and d_ct must not overlap each other,
 * d_msg or d_s_hat. a and e are drawn exactly as in hyena_encrypt from
 * `seed`. Messages are taken as residues mod q_i (hyena_encrypt's range
 * (-t/2, t/2] is not checked here).
 *
 * hyena_decrypt_device: d_ct device uint32 [n][2][L][N] with every residue
 * below its prime (not checked: others give unspecified messages); d_work
 * device uint32 [n][L][N], 16-byte aligned, overwritten (with c0 + c1 s mod
 * q_i); d_msg device int32 [n][N]. d_work and d_msg must not overlap each
 * other, d_ct or d_s_hat.
 *
 * Errors: EINVAL (NULL argument, host-only context, alignment, overlap,
 * n L >= 2^31), EHIP. n = 0 does nothing.
 */
int hyena_secret_prepare(const hyena_ctx *ctx, const int8_t *d_sk, uint32_t *d_s_hat,
                         hyena_stream_t stream);
int hyena_encrypt_device(const hyena_ctx *ctx, const uint32_t *d_s_hat, const int32_t *d_msg,
                         size_t n, uint64_t seed, uint32_t *d_work, uint32_t *d_ct,
                         hyena_stream_t stream);
int hyena_decrypt_device(const hyena_ctx *ctx, const uint32_t *d_s_hat, const uint32_t *d_ct,
                         size_t n, uint32_t *d_work, int32_t *d_msg, hyena_stream_t stream);

/*
 * hyena_decrypt_device without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same messages, bit for bit, from the
 * same kernels. The n*L*N-word workspace is a fixed array of
 * HYENA_NOALLOC_SCRATCH_WORDS uint32 words (16 MiB) in the library's device
 * data, which every GPU the library runs on holds until the process ends; its
 * address on a device is recorded when the first context is created there.
 * The call allocates nothing and is asynchronous on `stream`. All calls on one
 * GPU share that array: calls that overlap in time on one GPU (other streams,
 * other threads) race and give unspecified messages; serialise them.
 * Arguments as for hyena_decrypt_device (d_msg must not overlap d_ct or
 * d_s_hat). Errors: EINVAL (NULL argument, host-only context, n*L*N above
 * HYENA_NOALLOC_SCRATCH_WORDS, e.g. n > 170 at N = 8192, L = 3), EHIP.
 * n = 0 does nothing.
 */
#define HYENA_NOALLOC_SCRATCH_WORDS ((size_t)4 << 20)
int hyena_decrypt_device_noalloc(const hyena_ctx *ctx, const uint32_t *d_s_hat, const uint32_t *d_ct,
                                 size_t n, int32_t *d_msg, hyena_stream_t stream);

/* ------------------------------------------------------------------------
 * Planning and layout (host).
 * ---------------------------------------------------------------------- */

/*
 * Convolution layer descriptor. Fields marked "in" are set by the caller,
 * "out" by hyena_conv_plan.
 *
 * Geometry (coefficient encoding of the zero-padded tensor, the "Prior Art on Homomorphic Convolution" section):
 * p = (k-1)/2, Wp = W + 2p. If (H+2p)*Wp <= N the whole padded channel fits:
 * R = H, tiles = 1, Bt = (H+2p)*Wp and ci = min(Ci, N/Bt) channels share a
 * ciphertext (a caller may lower it through ci_req). Otherwise one channel is
 * split into row tiles: ci = 1, R = N/Wp - 2p, tiles = ceil(H/R),
 * Bt = (R+2p)*Wp. Input channel c' of group g sits at coefficients
 * c'*Bt + r*Wp + col. The kernel polynomial of output o and group g is
 * K_{o,g}(X) = sum f[o][g*ci+c'][di][dj] X^(O - c'*Bt - di*Wp - dj), with
 * O = (ci-1)*Bt + (k-1)*Wp + (k-1); output row r, column col of tile tau is
 * the coefficient O + r*Wp + col of output ciphertext (tau, o).
 */
typedef struct {
    /* in */
    uint32_t H, W, Ci, Co, k;   /* square or rectangular input, k in {1, 3} */
    uint32_t stride;            /* 1 or 2: the server always computes stride 1 */
    uint32_t depthwise;         /* 1: Co == Ci, one k x k filter per channel */
    uint32_t c_n;               /* Walsh group size: power of two dividing Co */
    uint32_t flags;             /* HYENA_FUSE_WHT ... */
    uint32_t ci_req;            /* 0 = as many channels per ciphertext as fit */
    uint32_t batch;             /* images sharing the weights (>= 1; 0 means 1) */
    /* out */
    uint32_t pad, Wp, R, tiles, ci, Bt, O, n_groups;
    uint32_t n_in;              /* input ciphertexts per image = tiles * n_groups */
    uint32_t n_out;             /* output ciphertexts per image = tiles * Co */
    uint32_t w_groups;          /* g extent of the weight array: n_groups, or 1 if depthwise */
} hyena_conv_desc;

#define HYENA_FUSE_WHT 0x1u  /* Walsh butterflies fused into the MAC epilogue */

/*
 * Fill the "out" fields. Errors: EINVAL (shape), ENOISE (worst-case noise
 * sum_g ||e_g K_{o,g}||_inf with |e| <= 32, or worst-case |y| over signed
 * 4-bit activations and the 4-bit weight bound |f| <= 8, breaks the
 * decryption condition ||v|| < Delta/2 of the "Homomorphic Operations in BFV" section or |y| < t/2).
 */
int hyena_conv_plan(const hyena_ctx *ctx, hyena_conv_desc *desc);

/* x: host int8 [Ci][H][W] -> msg: host int32 [tiles][n_groups][N] (zero
 * padding included; unused coefficients are 0). */
int hyena_pack_input(const hyena_conv_desc *desc, uint32_t N, const int8_t *x, int32_t *msg);

/* msg: host int32 [tiles][Co][N], decrypted outputs in hyena_conv order ->
 * y: host int32 [Co][Ho][Wo], the layer's output. The server always computes
 * the stride-1 convolution; for stride 1, Ho = H and Wo = W; for stride 2
 * (MobileNetV1's downsampling layers, the "End-to-end Evaluation" section)
 * Ho = ceil(H/2), Wo = ceil(W/2) and y[o][i][j] is the stride-1 output at row
 * 2i, column 2j, which equals the stride-2 convolution with padding (k-1)/2.
 * Errors: EINVAL (NULL, unplanned descriptor). */
int hyena_unpack_output(const hyena_conv_desc *desc, uint32_t N, const int32_t *msg, int32_t *y);

/* ------------------------------------------------------------------------
 * Device hot path (device pointers, asynchronous on stream).
 * ---------------------------------------------------------------------- */

/*
 * Offline weight preparation (the cloud stores kernel elements as integers,
 * the "Enabling Output Channel Packing" section; the polynomial form is derived from them once per layer).
 * For each Walsh group G, Walsh index j and input group g:
 *   gw[G*c_n+j] = sum_b H[j][b] f[G*c_n+b]     (Sylvester H_{c_n})
 *   Kw_{G,j,g} = c_n^{-1} (mod q_i) * (kernel polynomial of gw, as K above)
 *   d_wntt[G][j][g][i] = 2^32 NTT_i(Kw_{G,j,g}) mod q_i
 * (same transform as hyena_ntt; the factor 2^32 is the Montgomery form that
 * lets hyena_conv finish each output with a single Montgomery reduction, so
 * weights given to hyena_conv from elsewhere must carry it too).
 * d_w: device int8 [Co][Ci][k][k] ([Co][1][k][k] if depthwise).
 * d_wntt: device uint32 [Co/c_n][c_n][w_groups][L][N], 16-byte aligned. For
 * c_n = 1 this is 2^32 times the NTT of K_{o,g}. Errors: EINVAL, EHIP.
 */
int hyena_encode_weights(const hyena_ctx *ctx, const hyena_conv_desc *desc,
                         const int8_t *d_w, uint32_t *d_wntt, hyena_stream_t stream);

/*
 * The same d_wntt as hyena_encode_weights, bit for bit, synthesised directly
 * from the integer taps (the paper stores kernels as small integers and
 * derives their polynomial form on demand, "Enabling Output Channel Packing";
 * the evaluation points are those of the negacyclic NTT that the "Homomorphic
 * Operations in BFV" section multiplies with): word k of limb i is
 *   c_n^{-1} 2^32 * sum_taps gw * psi_i^((2 brv(k) + 1) e_tap)  mod q_i
 * over the ci*k*k taps of the input group, with no coefficient array and no
 * transform. Each word costs ci*k*k multiply-adds, so it is the cheaper form
 * for layers with few taps per input group (up to about 18: ci <= 2 at k = 3).
 * Every word of d_wntt is written (no prior zeroing needed); 4-byte
 * alignment suffices.
 * Errors: EINVAL (NULL, unplanned descriptor, host-only context),
 * EUNSUPPORTED (depthwise layers, N not a multiple of 256), EHIP.
 */
int hyena_synth_weights(const hyena_ctx *ctx, const hyena_conv_desc *desc,
                        const int8_t *d_w, uint32_t *d_wntt, hyena_stream_t stream);

/*
 * In-place forward negacyclic NTT of P polynomials ("Homomorphic Operations
 * in BFV": PMult multiplies in Z_q[X]/(X^N+1), which this transform turns
 * into pointwise products; "Optimal Parameter Selection", step 1: q = 1 mod
 * 2N is what makes it exist), d_poly: device uint32 [P][L][N] (limb i uses
 * q_i):
 *   A[k] = sum_j a[j] psi_i^((2 brv(k) + 1) j) mod q_i
 * (evaluation at the odd powers of psi_i, bit-reversed order; the transform
 * that turns the negacyclic product into a pointwise one, q = 1 mod 2N).
 * Inputs must be residues in [0, q_i). d_poly must be 16-byte aligned
 * (EINVAL otherwise). Errors: EINVAL, EHIP.
 */
int hyena_ntt(const hyena_ctx *ctx, uint32_t *d_poly, size_t P, hyena_stream_t stream);

/*
 * In-place inverse of hyena_ntt, including the factor N^{-1}: the outputs of
 * the NTT-domain products go back to the coefficient domain, where the
 * client decrypts them ("Homomorphic Operations in BFV": the negacyclic ring
 * Z_q[X]/(X^N+1) in which PMult and CMult multiply). d_poly: device uint32
 * [P][L][N], residues in [0, q_i), 16-byte aligned. Errors: EINVAL, EHIP.
 */
int hyena_intt(const hyena_ctx *ctx, uint32_t *d_poly, size_t P, hyena_stream_t stream);

/*
 * NTT schedules (threads per polynomial and butterfly stages per register
 * pass). Every schedule gives the same result as hyena_ntt / hyena_intt; they
 * differ in speed and are searched by the autotuner. hyena_ntt_schedules
 * reports the ids [first, first + count) that exist for ring degree N;
 * hyena_ntt_sched runs the forward (inverse = 0) or inverse transform with
 * schedule `sched` (-1 = default). Errors: EINVAL for a schedule of another N.
 */
int hyena_ntt_schedules(uint32_t N, int *first, int *count);
int hyena_ntt_sched(const hyena_ctx *ctx, uint32_t *d_poly, size_t P, int inverse, int sched,
                    hyena_stream_t stream);

/*
 * The homomorphic convolution in the NTT domain (the "Prior Art on Homomorphic
 * Convolution" and "Enabling Output Channel Packing" sections, with the
 * "Lazy Reduction" of the "Latency Optimization" section):
 *   A[b][tau][G][j][p][i][k] = sum_g ct[b][tau][g][p][i][k] * W[G][j][g][i][k]  mod q_i
 * accumulated lazily in 64 bits with one reduction per output coefficient.
 * With HYENA_FUSE_WHT (or c_n = 1) the output is already per output channel:
 *   Y[.][G*c_n+b] = sum_j H[b][j] A[.][G][j]  mod q_i,
 * otherwise it holds the Walsh components A and hyena_wht_pack finishes.
 * d_ct_ntt: device uint32 [batch][tiles][n_groups][2][L][N], NTT domain.
 * d_wntt:   device uint32 [Co/c_n][c_n][w_groups][L][N] (hyena_encode_weights:
 *           W times 2^32 mod q_i).
 * d_out_ntt: device uint32 [batch][tiles][Co][2][L][N]; must not alias inputs.
 * The three device arrays must be 16-byte aligned (copied in 16-byte pieces).
 * Errors: EINVAL, EHIP.
 */
int hyena_conv(const hyena_ctx *ctx, const hyena_conv_desc *desc,
               const uint32_t *d_ct_ntt, const uint32_t *d_wntt,
               uint32_t *d_out_ntt, hyena_stream_t stream);

/*
 * The same convolution computed in the coefficient domain, straight from the
 * integer taps (the products of ciphertext coefficients by small plaintext
 * integers without reduction and one reduction per output coefficient of the
 * "Lazy Reduction" passage, "Latency Optimization" section):
 *   Y[b][tau][o][p][i] = sum_g ct[b][tau][g][p][i] * K_{o,g}  mod (X^N + 1, q_i)
 * with K_{o,g} the kernel polynomial of hyena_encode_weights' c_n = 1 form,
 * each of its taps f X^e applied as a negacyclic shift. No NTT is involved:
 * the result equals hyena_intt(hyena_conv(hyena_ntt(ct))) with
 * HYENA_FUSE_WHT (or c_n = 1), whatever desc->c_n is. It does less work than
 * that path when an output has few taps (depthwise layers; c_i = 1 layers with
 * few input ciphertexts).
 * d_ct:  device uint32 [batch][tiles][n_groups][2][L][N], coefficient domain.
 * d_w:   device int8 [Co][Ci][k][k] ([Co][1][k][k] if depthwise).
 * d_out: device uint32 [batch][tiles][Co][2][L][N], coefficient domain; must
 *        not overlap d_ct (EINVAL).
 * N must be a multiple of 1024 (EUNSUPPORTED); at most 2^20 taps per output,
 * L * Co and batch * tiles at most 65535 (EINVAL). Errors: EINVAL,
 * EUNSUPPORTED, EHIP.
 */
int hyena_conv_direct(const hyena_ctx *ctx, const hyena_conv_desc *desc, const uint32_t *d_ct,
                      const int8_t *d_w, uint32_t *d_out, hyena_stream_t stream);

/*
 * Schedules of the multiply-accumulate. Every schedule computes the same
 * result as hyena_conv (bit for bit); they differ in speed only, and are what
 * the autotuner searches. hyena_conv_schedules reports how many exist;
 * hyena_conv_schedule_info fills info[6] = {uses_lds, mt, ot, wr, wo, stages}:
 * each thread accumulates mt rows (image, tile, ciphertext part) by ot
 * outputs of one NTT slot; LDS schedules run 4 waves in a wr x wo grid with a
 * `stages`-deep global->LDS copy pipeline. hyena_conv_default_schedule gives
 * the schedule hyena_conv uses for a planned descriptor. hyena_conv_tiled is
 * hyena_conv with an explicit schedule (EINVAL if it does not exist or does
 * not fit the layer: depthwise layers need a register-only schedule whose ot
 * divides ci). hyena_conv_schedule_taps returns 0 for a schedule that reads
 * NTT-domain weights and, for one that synthesizes them (hyena_conv_synth),
 * the most taps per weight word it takes; hyena_conv_tiled then reads d_wntt
 * as the int32 taps of hyena_synth_taps.
 */
int hyena_conv_schedules(int *count);
int hyena_conv_schedule_info(int sched, int *info);
int hyena_conv_schedule_taps(int sched);
int hyena_conv_default_schedule(const hyena_conv_desc *desc);
int hyena_conv_tiled(const hyena_ctx *ctx, const hyena_conv_desc *desc,
                     const uint32_t *d_ct_ntt, const uint32_t *d_wntt,
                     uint32_t *d_out_ntt, int sched, hyena_stream_t stream);

/*
 * Weights kept as integers, their NTT-domain words synthesized inside the
 * multiply-accumulate (the paper stores the kernels as small integers rather
 * than as plaintext polynomials, "Enabling Output Channel Packing"; the words
 * are the evaluations at the NTT points that hyena_synth_weights writes out).
 *
 * hyena_synth_taps: the Walsh-combined integer taps of a standard layer,
 *   d_taps[o][g][t] = sum_b H[j][b] f[G c_n + b][g ci + c'][di][dj]
 * for o = G c_n + j, input group g < w_groups, tap t = c' k^2 + di k + dj <
 * T = ci k^2 (0 past the last input channel and for T <= t < T4, T4 = T
 * rounded up to a multiple of 4). d_w: device int8 [Co][Ci][k][k]; d_taps:
 * device int32 [Co][w_groups][T4], 4-byte aligned (VGG-16's conv2_2: 786 KB
 * against 1.5 GiB of NTT-domain words). Errors: EINVAL (NULL, unplanned,
 * c_n not a power of two, host-only context), EUNSUPPORTED (depthwise), EHIP.
 *
 * hyena_conv_synth: hyena_conv (same d_ct_ntt, d_out_ntt, flags and result,
 * bit for bit) with the weight word of (o, g) at NTT slot s computed in the
 * block that uses it as sum_t taps[o][g][t] c_n^{-1} 2^32 r_s^e_t mod q_i
 * (r_s = psi_i^(2 brv(s) + 1), e_t the exponent of tap t in the kernel
 * polynomial) instead of read from an encoded-weight array: T multiply-adds
 * and one reduction per word and block, in place of streaming 4 bytes per
 * word. Layers with at most 18 taps per weight word (ci <= 2 at k = 3,
 * ci <= 18 at k = 1). Errors: EINVAL, EUNSUPPORTED (depthwise, more than 18
 * taps per word), EHIP.
 */
int hyena_synth_taps(const hyena_ctx *ctx, const hyena_conv_desc *desc, const int8_t *d_w,
                     int32_t *d_taps, hyena_stream_t stream);
int hyena_conv_synth(const hyena_ctx *ctx, const hyena_conv_desc *desc, const uint32_t *d_ct_ntt,
                     const int32_t *d_taps, uint32_t *d_out_ntt, hyena_stream_t stream);

/* ------------------------------------------------------------------------
 * The paper's own SIMD setting (batch encoding with a prime plaintext modulus
 * p = 1 mod 2n): the parameter selection of the "Optimal Parameter Selection"
 * section and the building blocks of its convolution ("Homomorphic
 * Operations in BFV": PMult, the automorphisms behind HRot). Slot s < n/2
 * holds the value at zeta^(3^s mod 2n), slot n/2 + s the value at
 * zeta^(-3^s mod 2n), zeta the least primitive 2n-th root of unity mod p.
 * ---------------------------------------------------------------------- */

/*
 * Host. h_{p,n}: the two equal nonzero coefficients (at X^(n/4), X^(3n/4)) of
 * the plaintext packing [1, -1] (1 in the first n/2 slots, -1 in the rest);
 * k in [1, kmax] minimising k h mod p (the least such k) and kh = k h mod p,
 * the coefficients of the plaintext packing [k, -k]. n a power of two >= 8,
 * p prime < 2^31, p = 1 mod 2n. Outputs may be NULL. Errors: EINVAL.
 */
int hyena_simd_params(uint32_t n, uint32_t p, uint32_t kmax, uint32_t *h, uint32_t *k,
                      uint32_t *kh);

/*
 * Batch encoding on the device, for a context created with
 * HYENA_PLAINTEXT_PRIME and L = 1 (its prime is p, its N is n):
 * hyena_simd_encode: d_slots device uint32 [P][N] slot values (reduced mod p
 * if not below it) -> d_coef device uint32 [P][N], 16-byte aligned, the
 * plaintext polynomials m with m(zeta^e_s) = v_s. hyena_simd_decode: the
 * inverse; d_coef (16-byte aligned) is overwritten with its NTT. The two
 * arrays must not overlap. Errors: EINVAL (also for L != 1), EHIP.
 */
int hyena_simd_encode(const hyena_ctx *ctx, const uint32_t *d_slots, size_t P, uint32_t *d_coef,
                      hyena_stream_t stream);
int hyena_simd_decode(const hyena_ctx *ctx, uint32_t *d_coef, size_t P, uint32_t *d_slots,
                      hyena_stream_t stream);

/*
 * Galois automorphism a(X) -> a(X^g) mod (X^N + 1, q_i) of P polynomials
 * [P][L][N] (coefficient domain), g odd (EINVAL otherwise). On slots,
 * g = 3^r rotates both rows by r, g = 2N - 1 swaps them. d_in, d_out device
 * uint32 [P][L][N], not overlapping. Errors: EINVAL, EHIP.
 */
int hyena_automorphism(const hyena_ctx *ctx, const uint32_t *d_in, size_t P, uint32_t g,
                       uint32_t *d_out, hyena_stream_t stream);

/*
 * PMult by a sparse plaintext w = sum_t coefs[t] X^exps[t] (at most 16
 * monomials; exps[t] < 2N, coefs[t] the plaintext integers, e.g. in [0, p)):
 *   d_out = w * d_in  mod (X^N + 1, q_i), for P polynomials [P][L][N].
 * With the two monomials kh X^(N/4) + kh X^(3N/4) this is PMult by the
 * [k, -k] plaintext. exps, coefs: host arrays. d_in, d_out device, not
 * overlapping. Errors: EINVAL, EHIP.
 */
int hyena_pmult_sparse(const hyena_ctx *ctx, const uint32_t *d_in, size_t P, uint32_t n_terms,
                       const uint32_t *exps, const uint32_t *coefs, uint32_t *d_out,
                       hyena_stream_t stream);

/*
 * HRot (Galois automorphism + key switching, "Homomorphic Operations in BFV",
 * with the decomposition base that trades noise against computation and
 * hoisting: decompose once, rotate many times). Digits are base 2^log2_base
 * (1 <= log2_base <= 29) of each limb's residues, D = ceil(31 / log2_base)
 * per limb (RNS-BV: the CRT basis element of limb i is 1 mod q_i, 0 mod the
 * others).
 *
 * hyena_galois_keygen (host, test setup like hyena_encrypt): key-switching key
 * for s(X^g) -> s, ksk host uint32 [L*D][2][L][N], coefficient domain: key
 * (i, j) = (a s + e + [k == i] s(X^g) 2^(j log2_base), -a) on limb k, a and e
 * drawn as for the encryption of message number i*D + j with `seed`.
 *
 * hyena_ksk_prepare: in place on device keys [n_polys][L][N] (n_polys = 2*L*D
 * per key), 16-byte aligned: 2^32 NTT(key) mod q_i, the form
 * hyena_hrot_hoisted takes.
 *
 * hyena_hrot_hoisted: n_ct ciphertexts d_ct [n_ct][2][L][N] (coefficient
 * domain) rotated by the n_rot <= 64 odd exponents gs (host array):
 *   d_out[m][r] = (c0(X^g) + sum_ij d_ij(X^g) b0_ij, sum_ij d_ij(X^g) b1_ij),
 * d_ij the digits of c1 (one decomposition and one forward NTT per ciphertext
 * serve every rotation). d_ksk: device, prepared keys [n_rot][L*D][2][L][N];
 * d_work: device uint32 [n_ct][L*D + 1][L][N], 16-byte aligned, overwritten;
 * d_out: device uint32 [n_ct][n_rot][2][L][N], 16-byte aligned. d_work and
 * d_out must not overlap each other or the inputs. Errors: EINVAL, EHIP.
 */
int hyena_galois_keygen(const hyena_ctx *ctx, const int8_t *sk, uint32_t g, uint32_t log2_base,
                        uint64_t seed, uint32_t *ksk);
int hyena_ksk_prepare(const hyena_ctx *ctx, uint32_t *d_ksk, size_t n_polys, hyena_stream_t stream);
int hyena_hrot_hoisted(const hyena_ctx *ctx, const uint32_t *d_ct, size_t n_ct, uint32_t n_rot,
                       const uint32_t *gs, uint32_t log2_base, const uint32_t *d_ksk,
                       uint32_t *d_work, uint32_t *d_out, hyena_stream_t stream);

/*
 * CMult and HAdd by integer scalars without intermediate reduction ("Lazy
 * Reduction"): d_out[o] = sum_r W[o][r] d_in[r] mod q_i for ciphertexts
 * d_in [R][2][L][N] (either domain), d_w device int32 [O][R] with
 * |W| <= 2^16 (not checked; larger weights give wrong sums), R <= 4096,
 * d_out [O][2][L][N] not overlapping the inputs. With R = 0 the outputs are
 * zero ciphertexts. Errors: EINVAL, EHIP.
 */
int hyena_cmult_accumulate(const hyena_ctx *ctx, const uint32_t *d_in, uint32_t R,
                           const int32_t *d_w, uint32_t O, uint32_t *d_out, hyena_stream_t stream);

/*
 * The paper's convolution with c_n = 2 in the SIMD setting (3x3 kernel):
 * input ciphertext g of n_in holds input channel 2g in its first slot row and
 * 2g + 1 in its second, each as a zero-bordered frame of width frame_w (so a
 * kernel offset (di, dj) is a rotation by (di - 1) frame_w + (dj - 1) slots).
 *   1. hoisted HRot of every input by the nine offsets;
 *   2. CMult + HAdd: A_o = sum wa[o][g*9 + r] rot_{g,r}, B_o likewise with wb;
 *   3. Z_o = A_o + PMult(B_o, kh (X^(N/4) + X^(3N/4))), the [k, -k] plaintext;
 *   4. out_o = Z_o + HRot(Z_o, X -> X^(2N-1)), the row swap.
 * With wa = k (f0 + f1) and wb = f0 - f1 (hyena_simd_conv_weights), both
 * rows of out_o hold 2k conv(x)_o mod p ("Enabling Output Channel Packing",
 * Eq. (hadamard2), with the [k, -k] plaintext of "Optimal Parameter
 * Selection"; the 1/2 of the equation is left out, every output carrying 2).
 *
 * hyena_simd_conv_weights (host): f int8 [Co][Ci][3][3], Ci even, k <= 255;
 * wa, wb host int32 [Co][Ci/2 * 9]. hyena_simd_conv_workspace: uint32 words
 * of d_work hyena_simd_conv_cn2 needs (0 for a bad log2_base).
 * hyena_simd_conv_cn2: d_ct device [n_in][2][L][N] (n_in <= 455), d_wa/d_wb
 * device int32 [Co][n_in*9], d_rot_ksk prepared keys [9][L*D][2][L][N] for the
 * nine offsets in (di, dj) order, d_swap_ksk prepared key for 2N - 1, d_work
 * 16-byte aligned, d_out device [Co][2][L][N] not overlapping the rest.
 * Errors: EINVAL, EHIP.
 */
int hyena_simd_conv_weights(uint32_t Ci, uint32_t Co, const int8_t *f, uint32_t k, int32_t *wa,
                            int32_t *wb);
size_t hyena_simd_conv_workspace(const hyena_ctx *ctx, uint32_t n_in, uint32_t Co, uint32_t log2_base);
int hyena_simd_conv_cn2(const hyena_ctx *ctx, const uint32_t *d_ct, uint32_t n_in, uint32_t frame_w,
                        const int32_t *d_wa, const int32_t *d_wb, uint32_t Co, uint32_t kh,
                        uint32_t log2_base, const uint32_t *d_rot_ksk, const uint32_t *d_swap_ksk,
                        uint32_t *d_work, size_t work_words, uint32_t *d_out, hyena_stream_t stream);

/*
 * The same convolution with output channel packing ("Enabling Output Channel
 * Packing": two output channels per output ciphertext, the communication of
 * conventional packed convolution). Every PMult by a two-valued plaintext
 * [a | b] is taken in its Walsh form, k (a + b) CMult + PMult((a - b) CMult,
 * [k, -k]):
 *   1. HRot of every input by X^(2N-1) (row swap);
 *   2. hoisted HRot of the inputs and their swaps by the nine offsets;
 *   3. A = sum wa rot, B = sum wb rot, out = A + PMult(B, [k, -k]).
 * With hyena_simd_conv_weights_packed (a the first row's weights, b the
 * second's: a = f[o][2g], b = f[o+1][2g+1] on input g, a = f[o][2g+1],
 * b = f[o+1][2g] on its swap), output ciphertext o2 holds 2k conv(x)_{2 o2}
 * in its first slot row and 2k conv(x)_{2 o2 + 1} in its second.
 * wa, wb: int32 [Co/2][2 n_in * 9] (index (h n_in + g) 9 + r, h = 1 for the
 * swapped input); Co even; n_in <= 227; d_out [Co/2][2][L][N]. Workspace from
 * hyena_simd_conv_packed_workspace; d_ct, d_work and d_out must not overlap.
 * Errors: EINVAL, EHIP.
 */
int hyena_simd_conv_weights_packed(uint32_t Ci, uint32_t Co, const int8_t *f, uint32_t k,
                                   int32_t *wa, int32_t *wb);
size_t hyena_simd_conv_packed_workspace(const hyena_ctx *ctx, uint32_t n_in, uint32_t Co,
                                        uint32_t log2_base);
int hyena_simd_conv_packed(const hyena_ctx *ctx, const uint32_t *d_ct, uint32_t n_in, uint32_t frame_w,
                           const int32_t *d_wa, const int32_t *d_wb, uint32_t Co, uint32_t kh,
                           uint32_t log2_base, const uint32_t *d_rot_ksk, const uint32_t *d_swap_ksk,
                           uint32_t *d_work, size_t work_words, uint32_t *d_out, hyena_stream_t stream);

/*
 * Decomposition base from the noise budget ("Optimal Parameter Selection":
 * the noise the [k, -k] plaintext saves allows a larger base for HRot, hence
 * fewer digits and less computation). Returns in *log2_base the largest
 * b <= 29 whose worst-case output noise of hyena_simd_conv_cn2 (packed = 0) or
 * hyena_simd_conv_packed (packed = 1) with weights wa, wb (host int32 [O][R],
 * as passed to those calls) and PMult coefficient kh stays below
 * q / (2p) - p, and in *margin_bits (may be NULL) log2 of that limit over the
 * bound. The bound: fresh and key errors at most 32; L D N (2^b - 1) 32 per
 * key switching; q mod p per automorphism, per unit of sum |w| of a CMult and
 * HAdd, per HAdd and 2 kh per PMult; noise times sum |w| and times 2 kh.
 * Errors: EINVAL, ENOISE (no base fits).
 */
int hyena_simd_conv_choose_base(const hyena_ctx *ctx, uint32_t p, uint32_t kh, const int32_t *wa,
                                const int32_t *wb, uint32_t O, uint32_t R, int packed,
                                uint32_t *log2_base, double *margin_bits);

/*
 * Walsh-Hadamard recombination across groups of c_n polynomials (the "Enabling Output Channel Packing" section):
 *   out[G][b] = sum_j H[b][j] in[G][j]  mod q_i, b, j < c_n,
 * H the Sylvester-ordered Walsh-Hadamard matrix (H_1 = [1],
 * H_2m = [[H_m, H_m], [H_m, -H_m]]), each in[G][j] one ciphertext of 2*L*N
 * uint32 residues in [2][L][N] order (the limb of a residue, and so its
 * prime, follows from its position). Applied to the Walsh components of
 * hyena_conv (computed with weights scaled by c_n^{-1}) it gives the
 * per-output-channel products exactly.
 * d_in, d_out: device uint32 [G][c_n][2][L][N], 16-byte aligned; d_out may
 * alias d_in. c_n: a power of two, 1 to 64. G = 0 does nothing.
 * Errors: EINVAL (NULL, alignment, c_n, host-only context), EHIP.
 */
int hyena_wht_pack(const hyena_ctx *ctx, uint32_t c_n, const uint32_t *d_in,
                   uint32_t *d_out, size_t G, hyena_stream_t stream);

/* ------------------------------------------------------------------------
 * Batched path: many layers (and images) per step.
 *
 * A step runs, for every layer: the forward NTT of its input ciphertexts (in
 * place), the multiply-accumulate with the Walsh-Hadamard recombination, and
 * the inverse NTT of its outputs, leaving d_out in the coefficient domain
 * exactly as the per-layer calls (hyena_ntt, hyena_conv with HYENA_FUSE_WHT,
 * hyena_intt) would. Layers are independent (the nonlinear layers between
 * convolutions are evaluated by the other party, outside this computation).
 * A second run transforms d_ct again: refill it before a run whose result
 * matters.
 * ---------------------------------------------------------------------- */
typedef struct {
    const hyena_conv_desc *desc;  /* planned; desc->batch images share the weights */
    uint32_t *d_ct;               /* device [batch][tiles][n_groups][2][L][N], coefficient domain */
    const uint32_t *d_wntt;       /* device, from hyena_encode_weights, or NULL when d_taps is given */
    uint32_t *d_out;              /* device [batch][tiles][Co][2][L][N]; must not alias d_ct */
    const int32_t *d_taps;        /* device, from hyena_synth_taps, or NULL: with it the autotuner
                                     also times the schedules that synthesize the weight words in
                                     the multiply-accumulate (hyena_conv_synth) */
} hyena_layer_io;                 /* d_ct, d_wntt, d_out 16-byte aligned; d_taps 4-byte */

typedef struct hyena_batch hyena_batch;

#define HYENA_BATCH_PERSISTENT 0x1u /* layers sharing an LDS schedule run in one persistent launch */
#define HYENA_BATCH_GRAPH 0x2u      /* the step is captured once into a hipGraph and replayed */
#define HYENA_BATCH_TUNE 0x4u       /* MAC schedule per layer and NTT schedule per direction chosen
                                       by timing (the forward on the inputs, the inverse on the
                                       outputs; inverse schedules within 5% of each other are
                                       timed again right after a multiply-accumulate phase, as
                                       they run in a step), and with HYENA_BATCH_PERSISTENT
                                       whether the persistent launch or one launch per layer runs
                                       the multiply-accumulate phase; choices cached in the file
                                       named by the environment variable HYENA_TUNE_CACHE when set */
#define HYENA_BATCH_TIMING 0x8u     /* record HIP events between the phases of every run for
                                       hyena_batch_phase_ms (with HYENA_BATCH_GRAPH: one graph
                                       per phase, events between their launches) */

/*
 * Build a batched step over n_layers layers. Copies the descriptors and keeps
 * the buffer pointers (the caller keeps the buffers alive until
 * hyena_batch_destroy). With HYENA_BATCH_TUNE the schedules are timed on the
 * given buffers: the input ciphertexts and the weights are left unchanged, the
 * output arrays are overwritten (as by every step). Allocates small device
 * tables. Errors: EINVAL, EHIP, ENOMEM.
 */
int hyena_batch_create(const hyena_ctx *ctx, const hyena_layer_io *layers, uint32_t n_layers,
                       uint32_t flags, hyena_batch **out);
/* Enqueue one step on stream (with HYENA_BATCH_GRAPH: replay the graph,
 * capturing it on the first call). Calls on one batch must not overlap. */
int hyena_batch_run(hyena_batch *b, hyena_stream_t stream);
/* info[] = {ntt forward schedule, ntt inverse schedule, kernel launches per
 * step, n_layers, persistent launches (0 when the autotuner chose one launch
 * per layer), MAC schedule of layer 0, 1, ...};
 * entries beyond the end are -1. */
int hyena_batch_info(const hyena_batch *b, int *info, size_t n_info);
/* Durations of the last run's phases in ms: ms[0] forward NTTs, ms[1]
 * multiply-accumulate (incl. counter reset and unfused Walsh kernels), ms[2]
 * inverse NTTs. Waits for the run. Needs HYENA_BATCH_TIMING. */
int hyena_batch_phase_ms(const hyena_batch *b, float *ms);
void hyena_batch_destroy(hyena_batch *b);

/* ------------------------------------------------------------------------
 * Learned cost model: an FP32 MLP 8 -> 64 -> 64 -> 1 with ReLU that predicts
 * the log time of a layer configuration (ring degree, RNS limbs, channel
 * partition, Walsh group, layer shape) and replaces an exhaustive timed search
 * over the parameters the paper selects by hand (the "Optimal Parameter
 * Selection" and "Evaluation Setup" sections choose n and q per layer).
 * Parameters: one device fp32 array theta of hyena_mlp_params() words laid out
 * as W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3. Features: device fp32
 * [B][8]; targets and predictions: device fp32 [B].
 * ---------------------------------------------------------------------- */
uint32_t hyena_mlp_params(void);
/* floats of the workspace hyena_mlp_loss_grad needs for batch size B */
size_t hyena_mlp_workspace_floats(uint32_t B);
/* y = MLP(x) */
int hyena_mlp_forward(const float *d_theta, const float *d_x, uint32_t B, float *d_y,
                      hyena_stream_t stream);
/* loss = mean (MLP(x) - t)^2 (d_loss may be NULL) and its gradient d_grad
 * [params]; deterministic (fixed summation order). */
int hyena_mlp_loss_grad(const float *d_theta, const float *d_x, const float *d_t, uint32_t B,
                        float *d_grad, float *d_loss, float *d_work, hyena_stream_t stream);
/* One Adam step (Kingma & Ba 2015) with bias correction for step >= 1. */
int hyena_mlp_adam(float *d_theta, const float *d_grad, float *d_m, float *d_v, uint32_t step,
                   float lr, float beta1, float beta2, float eps, hyena_stream_t stream);

/* ------------------------------------------------------------------------
 * Measurement helper: the integer instruction rates of the device, which the
 * multiply-accumulate's and the NTT's ALU roofline fractions are quoted
 * against. Runs `blocks` x 256 threads, each with eight independent chains of
 * iters x 4 operations op (0: v_mad_u64_u32, 32 x 32 -> 64-bit product plus a
 * 64-bit addend; 1: v_mul_lo_u32; 2: v_mul_hi_u32; 3: v_add_u32) on the null
 * stream, after two untimed launches; returns the timed launch's duration in
 * ms and its lane operations (rate = lane_ops / ms). d_out: device uint32
 * [blocks * 256], overwritten. Synchronous. Errors: EINVAL, EHIP.
 * ---------------------------------------------------------------------- */
int hyena_valu_rate(int op, uint32_t blocks, uint32_t iters, uint32_t *d_out, float *ms, double *lane_ops);

#ifdef __cplusplus
}
#endif
#endif /* HYENA_H */
