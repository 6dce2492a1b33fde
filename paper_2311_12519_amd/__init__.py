"""Python binding of libhyena.so, the gfx950 Hyena homomorphic-convolution library.

Argument marshalling only: every step of the convolution runs in the HIP
kernels of the library. Host calls take numpy arrays; device calls take
torch tensors that live on the GPU (torch is used for device memory and
streams only) and the stream to run on (default: torch's current stream).

The function names are those of the C ABI in ``include/hyena.h``. Importing
this package never falls back to anything: if ``libhyena.so`` is missing or
cannot be loaded, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# HYENA_LIB names another build of the same library (the sanitizer build of
# the host code loads this way); by default the in-tree libhyena.so
LIB_PATH = os.environ.get("HYENA_LIB") or os.path.join(_HERE, "libhyena.so")

HYENA_OK = 0
HYENA_EINVAL = -1
HYENA_EUNSUPPORTED = -2
HYENA_ENOISE = -3
HYENA_EHIP = -4
HYENA_ENOMEM = -5

HYENA_ALLOW_INSECURE = 0x1
HYENA_HOST_ONLY = 0x2
HYENA_PLAINTEXT_PRIME = 0x4
HYENA_PRIMES_30BIT = 0x100
HYENA_FUSE_WHT = 0x1
HYENA_BATCH_PERSISTENT = 0x1
HYENA_BATCH_GRAPH = 0x2
HYENA_BATCH_TUNE = 0x4
HYENA_BATCH_TIMING = 0x8

_ERRNAMES = {-1: "EINVAL", -2: "EUNSUPPORTED", -3: "ENOISE", -4: "EHIP", -5: "ENOMEM"}


class HyenaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"HYENA_{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class ConvDesc(ctypes.Structure):
    """Mirror of hyena_conv_desc."""
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "H", "W", "Ci", "Co", "k", "stride", "depthwise", "c_n", "flags", "ci_req", "batch",
        "pad", "Wp", "R", "tiles", "ci", "Bt", "O", "n_groups", "n_in", "n_out", "w_groups")]


class LayerIO(ctypes.Structure):
    """Mirror of hyena_layer_io."""
    _fields_ = [("desc", ctypes.c_void_p), ("d_ct", ctypes.c_void_p), ("d_wntt", ctypes.c_void_p),
                ("d_out", ctypes.c_void_p), ("d_taps", ctypes.c_void_p)]


_lib = None
_P = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_sz = ctypes.c_size_t

_SIGS = {
    "hyena_create": [_u32, _u32, _P, _u32, _u32, _P],
    "hyena_destroy": [_P],
    "hyena_get_params": [_P, _P, _P, _P, _P],
    "hyena_keygen": [_P, _u64, _P],
    "hyena_encrypt": [_P, _P, _P, _sz, _u64, _P],
    "hyena_decrypt": [_P, _P, _P, _sz, _P],
    "hyena_conv_plan": [_P, _P],
    "hyena_pack_input": [_P, _u32, _P, _P],
    "hyena_unpack_output": [_P, _u32, _P, _P],
    "hyena_encode_weights": [_P, _P, _P, _P, _P],
    "hyena_synth_weights": [_P, _P, _P, _P, _P],
    "hyena_ntt": [_P, _P, _sz, _P],
    "hyena_intt": [_P, _P, _sz, _P],
    "hyena_conv": [_P, _P, _P, _P, _P, _P],
    "hyena_conv_direct": [_P, _P, _P, _P, _P, _P],
    "hyena_secret_prepare": [_P, _P, _P, _P],
    "hyena_encrypt_device": [_P, _P, _P, _sz, _u64, _P, _P, _P],
    "hyena_decrypt_device": [_P, _P, _P, _sz, _P, _P, _P],
    "hyena_decrypt_device_noalloc": [_P, _P, _P, _sz, _P, _P],
    "hyena_simd_params": [_u32, _u32, _u32, _P, _P, _P],
    "hyena_simd_encode": [_P, _P, _sz, _P, _P],
    "hyena_simd_decode": [_P, _P, _sz, _P, _P],
    "hyena_automorphism": [_P, _P, _sz, _u32, _P, _P],
    "hyena_pmult_sparse": [_P, _P, _sz, _u32, _P, _P, _P, _P],
    "hyena_galois_keygen": [_P, _P, _u32, _u32, _u64, _P],
    "hyena_ksk_prepare": [_P, _P, _sz, _P],
    "hyena_hrot_hoisted": [_P, _P, _sz, _u32, _P, _u32, _P, _P, _P, _P],
    "hyena_cmult_accumulate": [_P, _P, _u32, _P, _u32, _P, _P],
    "hyena_simd_conv_weights": [_u32, _u32, _P, _u32, _P, _P],
    "hyena_simd_conv_cn2": [_P, _P, _u32, _u32, _P, _P, _u32, _u32, _u32, _P, _P, _P, _sz, _P, _P],
    "hyena_simd_conv_weights_packed": [_u32, _u32, _P, _u32, _P, _P],
    "hyena_simd_conv_packed": [_P, _P, _u32, _u32, _P, _P, _u32, _u32, _u32, _P, _P, _P, _sz, _P, _P],
    "hyena_simd_conv_choose_base": [_P, _u32, _u32, _P, _P, _u32, _u32, ctypes.c_int, _P, _P],
    "hyena_wht_pack": [_P, _u32, _P, _P, _sz, _P],
    "hyena_conv_tiled": [_P, _P, _P, _P, _P, ctypes.c_int, _P],
    "hyena_conv_schedules": [_P],
    "hyena_conv_schedule_info": [ctypes.c_int, _P],
    "hyena_conv_schedule_taps": [ctypes.c_int],
    "hyena_conv_default_schedule": [_P],
    "hyena_synth_taps": [_P, _P, _P, _P, _P],
    "hyena_conv_synth": [_P, _P, _P, _P, _P, _P],
    "hyena_ntt_schedules": [_u32, _P, _P],
    "hyena_valu_rate": [ctypes.c_int, _u32, _u32, _P, _P, _P],
    "hyena_ntt_sched": [_P, _P, _sz, ctypes.c_int, ctypes.c_int, _P],
}


def lib() -> ctypes.CDLL:
    """Load libhyena.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_2311_12519_amd/build.py` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None if name == "hyena_destroy" else ctypes.c_int
        L.hyena_last_error.restype = ctypes.c_char_p
        L.hyena_last_error.argtypes = []
        for name in ("hyena_simd_conv_workspace", "hyena_simd_conv_packed_workspace"):   # size_t results
            f = getattr(L, name)
            f.argtypes = [_P, _u32, _u32, _u32]
            f.restype = _sz
        _register_extra(L)
        _lib = L
    return _lib


def _register_extra(L):
    """Signatures of the batched-path and cost-model entry points, if present."""
    extra = {
        "hyena_batch_create": [_P, _P, _u32, _u32, _P],
        "hyena_batch_destroy": [_P],
        "hyena_batch_run": [_P, _P],
        "hyena_batch_info": [_P, _P, _sz],
        "hyena_batch_phase_ms": [_P, _P],
        "hyena_conv_tiled": [_P, _P, _P, _P, _P, ctypes.c_int, _P],
        "hyena_conv_schedules": [_P],
        "hyena_conv_schedule_info": [ctypes.c_int, _P],
        "hyena_conv_default_schedule": [_P],
        "hyena_mlp_forward": [_P, _P, _u32, _P, _P],
        "hyena_mlp_loss_grad": [_P, _P, _P, _u32, _P, _P, _P, _P],
        "hyena_mlp_adam": [_P, _P, _P, _P, _u32, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, ctypes.c_float, _P],
    }
    for name, args in extra.items():
        if hasattr(L, name):
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None if name == "hyena_batch_destroy" else ctypes.c_int
    if hasattr(L, "hyena_mlp_params"):
        L.hyena_mlp_params.argtypes = []
        L.hyena_mlp_params.restype = ctypes.c_uint32
        L.hyena_mlp_workspace_floats.argtypes = [_u32]
        L.hyena_mlp_workspace_floats.restype = ctypes.c_size_t


def _check(code: int) -> None:
    if code != HYENA_OK:
        raise HyenaError(code, lib().hyena_last_error().decode())


def _np_ptr(a: np.ndarray, dtype) -> ctypes.c_void_p:
    if a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
        raise TypeError(f"expected a C-contiguous {np.dtype(dtype).name} array")
    return ctypes.c_void_p(a.ctypes.data)


def _dev_ptr(t, dtype_name: str) -> ctypes.c_void_p:
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch." + dtype_name:
        raise TypeError(f"expected a contiguous device tensor of torch.{dtype_name}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ---------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------

class Ctx:
    """Owns a hyena_ctx handle; destroyed with the object."""

    def __init__(self, handle: ctypes.c_void_p, N: int, L: int, log2_t: int):
        self.handle = handle
        self.N, self.L, self.log2_t = N, L, log2_t
        p = np.zeros(L, dtype=np.uint32)
        s = np.zeros(L, dtype=np.uint32)
        _check(lib().hyena_get_params(handle, None, None, _np_ptr(p, np.uint32), _np_ptr(s, np.uint32)))
        self.primes = [int(x) for x in p]
        self.psi = [int(x) for x in s]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.hyena_destroy(h)
            self.handle = None

    @property
    def _as_parameter_(self):
        return self.handle


def hyena_create(N: int, L: int, primes=None, log2_t: int = 20, flags: int = 0) -> Ctx:
    out = ctypes.c_void_p()
    pr = None
    if primes is not None:
        arr = np.ascontiguousarray(primes, dtype=np.uint32)
        pr = _np_ptr(arr, np.uint32)
    _check(lib().hyena_create(N, L, pr, log2_t, flags, ctypes.byref(out)))
    return Ctx(out, N, L, log2_t)


def hyena_destroy(ctx: Ctx) -> None:
    if ctx.handle:
        lib().hyena_destroy(ctx.handle)
        ctx.handle = None


def hyena_keygen(ctx: Ctx, seed: int) -> np.ndarray:
    sk = np.zeros(ctx.N, dtype=np.int8)
    _check(lib().hyena_keygen(ctx.handle, seed, _np_ptr(sk, np.int8)))
    return sk


def hyena_encrypt(ctx: Ctx, sk: np.ndarray, msg: np.ndarray, seed: int) -> np.ndarray:
    msg = np.ascontiguousarray(msg, dtype=np.int32).reshape(-1, ctx.N)
    ct = np.zeros((msg.shape[0], 2, ctx.L, ctx.N), dtype=np.uint32)
    _check(lib().hyena_encrypt(ctx.handle, _np_ptr(np.ascontiguousarray(sk, dtype=np.int8), np.int8),
                               _np_ptr(msg, np.int32), msg.shape[0], seed, _np_ptr(ct, np.uint32)))
    return ct


def hyena_decrypt(ctx: Ctx, sk: np.ndarray, ct: np.ndarray) -> np.ndarray:
    ct = np.ascontiguousarray(ct, dtype=np.uint32).reshape(-1, 2, ctx.L, ctx.N)
    msg = np.zeros((ct.shape[0], ctx.N), dtype=np.int32)
    _check(lib().hyena_decrypt(ctx.handle, _np_ptr(np.ascontiguousarray(sk, dtype=np.int8), np.int8),
                               _np_ptr(ct, np.uint32), ct.shape[0], _np_ptr(msg, np.int32)))
    return msg


def hyena_conv_plan(ctx: Ctx, H: int, W: int, Ci: int, Co: int, k: int = 3, *, stride: int = 1,
                    depthwise: bool = False, c_n: int = 1, flags: int = 0, ci_req: int = 0,
                    batch: int = 1) -> ConvDesc:
    d = ConvDesc(H=H, W=W, Ci=Ci, Co=Co, k=k, stride=stride, depthwise=int(depthwise), c_n=c_n,
                 flags=flags, ci_req=ci_req, batch=batch)
    _check(lib().hyena_conv_plan(ctx.handle, ctypes.byref(d)))
    return d


def hyena_pack_input(desc: ConvDesc, N: int, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.int8)
    msg = np.zeros((desc.tiles, desc.n_groups, N), dtype=np.int32)
    _check(lib().hyena_pack_input(ctypes.byref(desc), N, _np_ptr(x, np.int8), _np_ptr(msg, np.int32)))
    return msg


def hyena_unpack_output(desc: ConvDesc, N: int, msg: np.ndarray) -> np.ndarray:
    msg = np.ascontiguousarray(msg, dtype=np.int32)
    s = max(1, desc.stride)
    y = np.zeros((desc.Co, -(-desc.H // s), -(-desc.W // s)), dtype=np.int32)
    _check(lib().hyena_unpack_output(ctypes.byref(desc), N, _np_ptr(msg, np.int32), _np_ptr(y, np.int32)))
    return y


# ---------------------------------------------------------------------------
# device hot path
# ---------------------------------------------------------------------------

def hyena_encode_weights(ctx: Ctx, desc: ConvDesc, d_w, d_wntt, stream=None) -> None:
    _check(lib().hyena_encode_weights(ctx.handle, ctypes.byref(desc), _dev_ptr(d_w, "int8"),
                                      _dev_ptr(d_wntt, "int32"), _stream(stream)))


def hyena_synth_weights(ctx: Ctx, desc: ConvDesc, d_w, d_wntt, stream=None) -> None:
    _check(lib().hyena_synth_weights(ctx.handle, ctypes.byref(desc), _dev_ptr(d_w, "int8"),
                                     _dev_ptr(d_wntt, "int32"), _stream(stream)))


def hyena_ntt(ctx: Ctx, d_poly, stream=None) -> None:
    P = d_poly.numel() // (ctx.L * ctx.N)
    if P * ctx.L * ctx.N != d_poly.numel():
        raise ValueError("tensor size is not a multiple of L*N")
    _check(lib().hyena_ntt(ctx.handle, _dev_ptr(d_poly, "int32"), P, _stream(stream)))


def hyena_intt(ctx: Ctx, d_poly, stream=None) -> None:
    P = d_poly.numel() // (ctx.L * ctx.N)
    if P * ctx.L * ctx.N != d_poly.numel():
        raise ValueError("tensor size is not a multiple of L*N")
    _check(lib().hyena_intt(ctx.handle, _dev_ptr(d_poly, "int32"), P, _stream(stream)))


def hyena_ntt_schedules(N: int) -> list:
    first, count = ctypes.c_int(), ctypes.c_int()
    _check(lib().hyena_ntt_schedules(N, ctypes.byref(first), ctypes.byref(count)))
    return list(range(first.value, first.value + count.value))


def hyena_ntt_sched(ctx: Ctx, d_poly, inverse: bool, sched: int, stream=None) -> None:
    P = d_poly.numel() // (ctx.L * ctx.N)
    if P * ctx.L * ctx.N != d_poly.numel():
        raise ValueError("tensor size is not a multiple of L*N")
    _check(lib().hyena_ntt_sched(ctx.handle, _dev_ptr(d_poly, "int32"), P, int(inverse), sched, _stream(stream)))


def hyena_conv(ctx: Ctx, desc: ConvDesc, d_ct_ntt, d_wntt, d_out_ntt, stream=None) -> None:
    _check(lib().hyena_conv(ctx.handle, ctypes.byref(desc), _dev_ptr(d_ct_ntt, "int32"),
                            _dev_ptr(d_wntt, "int32"), _dev_ptr(d_out_ntt, "int32"), _stream(stream)))


def hyena_conv_direct(ctx: Ctx, desc: ConvDesc, d_ct, d_w, d_out, stream=None) -> None:
    """Coefficient-domain convolution from the int8 taps (no NTT); the result
    equals hyena_intt(hyena_conv(hyena_ntt(d_ct))) with per-channel outputs."""
    _check(lib().hyena_conv_direct(ctx.handle, ctypes.byref(desc), _dev_ptr(d_ct, "int32"),
                                   _dev_ptr(d_w, "int8"), _dev_ptr(d_out, "int32"), _stream(stream)))


def _need(t, numel: int, what: str) -> None:
    if t.numel() != numel:
        raise ValueError(f"{what} has {t.numel()} elements, expected {numel}")


def hyena_secret_prepare(ctx: Ctx, d_sk, d_s_hat, stream=None) -> None:
    """d_s_hat <- 2^32 NTT(s) mod q_i from the device int8 secret d_sk [N]."""
    _need(d_sk, ctx.N, "d_sk")
    _need(d_s_hat, ctx.L * ctx.N, "d_s_hat")
    _check(lib().hyena_secret_prepare(ctx.handle, _dev_ptr(d_sk, "int8"), _dev_ptr(d_s_hat, "int32"),
                                      _stream(stream)))


def hyena_encrypt_device(ctx: Ctx, d_s_hat, d_msg, seed: int, d_work, d_ct, stream=None) -> None:
    """Encrypt the n messages d_msg [n][N] into d_ct [n][2][L][N]; the same
    ciphertexts as hyena_encrypt with the same secret and seed. d_work is an
    int32 workspace of n*L*N elements (overwritten)."""
    n = d_msg.numel() // ctx.N
    _need(d_msg, n * ctx.N, "d_msg")
    _need(d_ct, n * 2 * ctx.L * ctx.N, "d_ct")
    _need(d_s_hat, ctx.L * ctx.N, "d_s_hat")
    if d_work.numel() < n * ctx.L * ctx.N:
        raise ValueError(f"d_work has {d_work.numel()} elements, needs {n * ctx.L * ctx.N}")
    _check(lib().hyena_encrypt_device(ctx.handle, _dev_ptr(d_s_hat, "int32"), _dev_ptr(d_msg, "int32"), n, seed,
                                      _dev_ptr(d_work, "int32"), _dev_ptr(d_ct, "int32"), _stream(stream)))


def hyena_decrypt_device(ctx: Ctx, d_s_hat, d_ct, d_work, d_msg, stream=None) -> None:
    """Decrypt the n ciphertexts d_ct [n][2][L][N] into d_msg [n][N]; d_work
    is an int32 workspace of n*L*N elements (overwritten)."""
    n = d_ct.numel() // (2 * ctx.L * ctx.N)
    _need(d_ct, n * 2 * ctx.L * ctx.N, "d_ct")
    _need(d_msg, n * ctx.N, "d_msg")
    _need(d_s_hat, ctx.L * ctx.N, "d_s_hat")
    if d_work.numel() < n * ctx.L * ctx.N:
        raise ValueError(f"d_work has {d_work.numel()} elements, needs {n * ctx.L * ctx.N}")
    _check(lib().hyena_decrypt_device(ctx.handle, _dev_ptr(d_s_hat, "int32"), _dev_ptr(d_ct, "int32"), n,
                                      _dev_ptr(d_work, "int32"), _dev_ptr(d_msg, "int32"), _stream(stream)))


HYENA_NOALLOC_SCRATCH_WORDS = 4 << 20


def hyena_decrypt_device_noalloc(ctx: Ctx, d_s_hat, d_ct, d_msg, stream=None) -> None:
    """hyena_decrypt_device with the library's fixed device workspace
    (n*L*N <= HYENA_NOALLOC_SCRATCH_WORDS; the library refuses larger n)."""
    n = d_ct.numel() // (2 * ctx.L * ctx.N)
    _need(d_ct, n * 2 * ctx.L * ctx.N, "d_ct")
    _need(d_msg, n * ctx.N, "d_msg")
    _need(d_s_hat, ctx.L * ctx.N, "d_s_hat")
    _check(lib().hyena_decrypt_device_noalloc(ctx.handle, _dev_ptr(d_s_hat, "int32"), _dev_ptr(d_ct, "int32"), n,
                                              _dev_ptr(d_msg, "int32"), _stream(stream)))


def hyena_simd_params(n: int, p: int, kmax: int):
    """(h_{p,n}, k, k h mod p): the [1, -1] plaintext's coefficient and the
    k in [1, kmax] minimising k h mod p."""
    h, k, kh = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().hyena_simd_params(n, p, kmax, ctypes.byref(h), ctypes.byref(k), ctypes.byref(kh)))
    return h.value, k.value, kh.value


def _polys(ctx: Ctx, t, limbs: int) -> int:
    P = t.numel() // (limbs * ctx.N)
    if P * limbs * ctx.N != t.numel():
        raise ValueError("tensor size is not a multiple of the polynomial size")
    return P


def hyena_simd_encode(ctx: Ctx, d_slots, d_coef, stream=None) -> None:
    """Slots [P][N] (mod p) -> plaintext polynomials [P][N] (plaintext-prime context)."""
    P = _polys(ctx, d_slots, 1)
    _need(d_coef, P * ctx.N, "d_coef")
    _check(lib().hyena_simd_encode(ctx.handle, _dev_ptr(d_slots, "int32"), P, _dev_ptr(d_coef, "int32"),
                                   _stream(stream)))


def hyena_simd_decode(ctx: Ctx, d_coef, d_slots, stream=None) -> None:
    """Plaintext polynomials [P][N] -> slots [P][N]; d_coef is overwritten with its NTT."""
    P = _polys(ctx, d_coef, 1)
    _need(d_slots, P * ctx.N, "d_slots")
    _check(lib().hyena_simd_decode(ctx.handle, _dev_ptr(d_coef, "int32"), P, _dev_ptr(d_slots, "int32"),
                                   _stream(stream)))


def hyena_automorphism(ctx: Ctx, d_in, g: int, d_out, stream=None) -> None:
    """d_out = d_in(X^g) for polynomials [P][L][N]."""
    P = _polys(ctx, d_in, ctx.L)
    _need(d_out, d_in.numel(), "d_out")
    _check(lib().hyena_automorphism(ctx.handle, _dev_ptr(d_in, "int32"), P, g, _dev_ptr(d_out, "int32"),
                                    _stream(stream)))


def hyena_pmult_sparse(ctx: Ctx, d_in, exps, coefs, d_out, stream=None) -> None:
    """d_out = (sum_t coefs[t] X^exps[t]) * d_in for polynomials [P][L][N]."""
    P = _polys(ctx, d_in, ctx.L)
    _need(d_out, d_in.numel(), "d_out")
    e = np.ascontiguousarray(exps, dtype=np.uint32)
    c = np.ascontiguousarray(coefs, dtype=np.uint32)
    if e.shape != c.shape:
        raise ValueError("exps and coefs differ in length")
    _check(lib().hyena_pmult_sparse(ctx.handle, _dev_ptr(d_in, "int32"), P, e.shape[0], _np_ptr(e, np.uint32),
                                    _np_ptr(c, np.uint32), _dev_ptr(d_out, "int32"), _stream(stream)))


def n_digits(log2_base: int) -> int:
    """Digits per residue in base 2^log2_base (residues below 2^31); bases
    outside [1, 29] are refused by the library calls themselves."""
    return -(-31 // max(1, log2_base))


def hyena_galois_keygen(ctx: Ctx, sk: np.ndarray, g: int, log2_base: int, seed: int) -> np.ndarray:
    """Host key-switching key for s(X^g) -> s: uint32 [L*D][2][L][N]."""
    D = n_digits(log2_base)
    ksk = np.zeros((ctx.L * D, 2, ctx.L, ctx.N), dtype=np.uint32)
    _check(lib().hyena_galois_keygen(ctx.handle, _np_ptr(np.ascontiguousarray(sk, dtype=np.int8), np.int8), g,
                                     log2_base, seed, _np_ptr(ksk, np.uint32)))
    return ksk


def hyena_ksk_prepare(ctx: Ctx, d_ksk, stream=None) -> None:
    """In place: keys [..][L][N] -> 2^32 NTT(keys)."""
    P = _polys(ctx, d_ksk, ctx.L)
    _check(lib().hyena_ksk_prepare(ctx.handle, _dev_ptr(d_ksk, "int32"), P, _stream(stream)))


def hyena_hrot_hoisted(ctx: Ctx, d_ct, gs, log2_base: int, d_ksk, d_work, d_out, stream=None) -> None:
    """Rotate every ciphertext of d_ct [n][2][L][N] by every g in gs."""
    D, LN = n_digits(log2_base), ctx.L * ctx.N
    n = _polys(ctx, d_ct, 2 * ctx.L)
    g = np.ascontiguousarray(gs, dtype=np.uint32)
    R = g.shape[0]
    _need(d_ksk, R * ctx.L * D * 2 * LN, "d_ksk")
    _need(d_out, n * R * 2 * LN, "d_out")
    if d_work.numel() < n * (ctx.L * D + 1) * LN:
        raise ValueError(f"d_work has {d_work.numel()} elements, needs {n * (ctx.L * D + 1) * LN}")
    _check(lib().hyena_hrot_hoisted(ctx.handle, _dev_ptr(d_ct, "int32"), n, R, _np_ptr(g, np.uint32), log2_base,
                                    _dev_ptr(d_ksk, "int32"), _dev_ptr(d_work, "int32"), _dev_ptr(d_out, "int32"),
                                    _stream(stream)))


def hyena_cmult_accumulate(ctx: Ctx, d_in, d_w, d_out, stream=None) -> None:
    """d_out[o] = sum_r W[o][r] d_in[r] for ciphertexts [R][2][L][N], W int32 [O][R]."""
    R = _polys(ctx, d_in, 2 * ctx.L)
    if d_w.dim() != 2 or d_w.shape[1] != R:
        raise ValueError("d_w must be [O][R]")
    O = d_w.shape[0]
    _need(d_out, O * 2 * ctx.L * ctx.N, "d_out")
    _check(lib().hyena_cmult_accumulate(ctx.handle, _dev_ptr(d_in, "int32"), R, _dev_ptr(d_w, "int32"), O,
                                        _dev_ptr(d_out, "int32"), _stream(stream)))


def hyena_simd_conv_weights(f: np.ndarray, k: int):
    """Walsh CMult scalars (wa, wb) int32 [Co][Ci/2 * 9] of the c_n = 2 SIMD
    convolution from integer weights f [Co][Ci][3][3]."""
    f = np.ascontiguousarray(f, dtype=np.int8)
    Co, Ci = f.shape[0], f.shape[1]
    wa = np.zeros((Co, Ci // 2 * 9), dtype=np.int32)
    wb = np.zeros_like(wa)
    _check(lib().hyena_simd_conv_weights(Ci, Co, _np_ptr(f, np.int8), k, _np_ptr(wa, np.int32), _np_ptr(wb, np.int32)))
    return wa, wb


def hyena_simd_conv_workspace(ctx: Ctx, n_in: int, Co: int, log2_base: int) -> int:
    """uint32 words of workspace hyena_simd_conv_cn2 needs (0 for a bad base)."""
    return int(lib().hyena_simd_conv_workspace(ctx.handle, n_in, Co, log2_base))


def hyena_simd_conv_cn2(ctx: Ctx, d_ct, frame_w: int, d_wa, d_wb, kh: int, log2_base: int, d_rot_ksk, d_swap_ksk,
                        d_work, d_out, stream=None) -> None:
    """The paper's c_n = 2 SIMD convolution (3x3): d_out[o] holds 2k conv(x)_o in both rows."""
    n_in = _polys(ctx, d_ct, 2 * ctx.L)
    Co = d_wa.shape[0]
    if tuple(d_wa.shape) != (Co, n_in * 9) or tuple(d_wb.shape) != (Co, n_in * 9):
        raise ValueError("d_wa and d_wb must be [Co][n_in * 9]")
    _need(d_out, Co * 2 * ctx.L * ctx.N, "d_out")
    _check(lib().hyena_simd_conv_cn2(ctx.handle, _dev_ptr(d_ct, "int32"), n_in, frame_w, _dev_ptr(d_wa, "int32"),
                                     _dev_ptr(d_wb, "int32"), Co, kh, log2_base, _dev_ptr(d_rot_ksk, "int32"),
                                     _dev_ptr(d_swap_ksk, "int32"), _dev_ptr(d_work, "int32"), d_work.numel(),
                                     _dev_ptr(d_out, "int32"), _stream(stream)))


def hyena_simd_conv_weights_packed(f: np.ndarray, k: int):
    """Walsh CMult scalars (wa, wb) int32 [Co/2][Ci * 9] of the output-packed
    c_n = 2 SIMD convolution from integer weights f [Co][Ci][3][3]."""
    f = np.ascontiguousarray(f, dtype=np.int8)
    Co, Ci = f.shape[0], f.shape[1]
    wa = np.zeros((max(Co // 2, 1), Ci * 9), dtype=np.int32)
    wb = np.zeros_like(wa)
    _check(lib().hyena_simd_conv_weights_packed(Ci, Co, _np_ptr(f, np.int8), k, _np_ptr(wa, np.int32),
                                                _np_ptr(wb, np.int32)))
    return wa, wb


def hyena_simd_conv_packed_workspace(ctx: Ctx, n_in: int, Co: int, log2_base: int) -> int:
    """uint32 words of workspace hyena_simd_conv_packed needs (0 for a bad base)."""
    return int(lib().hyena_simd_conv_packed_workspace(ctx.handle, n_in, Co, log2_base))


def hyena_simd_conv_packed(ctx: Ctx, d_ct, frame_w: int, d_wa, d_wb, kh: int, log2_base: int, d_rot_ksk,
                           d_swap_ksk, d_work, d_out, stream=None) -> None:
    """Output-packed c_n = 2 SIMD convolution: d_out[o2] holds 2k conv(x)_{2 o2}
    and 2k conv(x)_{2 o2 + 1} in its two slot rows."""
    n_in = _polys(ctx, d_ct, 2 * ctx.L)
    P2 = d_wa.shape[0]
    if tuple(d_wa.shape) != (P2, 2 * n_in * 9) or tuple(d_wb.shape) != (P2, 2 * n_in * 9):
        raise ValueError("d_wa and d_wb must be [Co/2][2 n_in * 9]")
    _need(d_out, P2 * 2 * ctx.L * ctx.N, "d_out")
    _check(lib().hyena_simd_conv_packed(ctx.handle, _dev_ptr(d_ct, "int32"), n_in, frame_w, _dev_ptr(d_wa, "int32"),
                                        _dev_ptr(d_wb, "int32"), 2 * P2, kh, log2_base, _dev_ptr(d_rot_ksk, "int32"),
                                        _dev_ptr(d_swap_ksk, "int32"), _dev_ptr(d_work, "int32"), d_work.numel(),
                                        _dev_ptr(d_out, "int32"), _stream(stream)))


def hyena_simd_conv_choose_base(ctx: Ctx, p: int, kh: int, wa: np.ndarray, wb: np.ndarray, packed: bool = False):
    """(log2 of the largest decomposition base the worst-case noise allows, margin in bits)."""
    wa = np.ascontiguousarray(wa, dtype=np.int32)
    wb = np.ascontiguousarray(wb, dtype=np.int32)
    if wa.shape != wb.shape or wa.ndim != 2:
        raise ValueError("wa and wb must be [O][R] of the same shape")
    b, m = ctypes.c_uint32(), ctypes.c_double()
    _check(lib().hyena_simd_conv_choose_base(ctx.handle, p, kh, _np_ptr(wa, np.int32), _np_ptr(wb, np.int32),
                                             wa.shape[0], wa.shape[1], int(packed), ctypes.byref(b), ctypes.byref(m)))
    return b.value, m.value


def hyena_wht_pack(ctx: Ctx, c_n: int, d_in, d_out, G: int, stream=None) -> None:
    _check(lib().hyena_wht_pack(ctx.handle, c_n, _dev_ptr(d_in, "int32"), _dev_ptr(d_out, "int32"),
                                G, _stream(stream)))


def hyena_conv_tiled(ctx: Ctx, desc: ConvDesc, d_ct_ntt, d_wntt, d_out_ntt, sched: int, stream=None) -> None:
    _check(lib().hyena_conv_tiled(ctx.handle, ctypes.byref(desc), _dev_ptr(d_ct_ntt, "int32"),
                                  _dev_ptr(d_wntt, "int32"), _dev_ptr(d_out_ntt, "int32"), sched,
                                  _stream(stream)))


def hyena_conv_schedules() -> list:
    """[(uses_lds, mt, ot, wr, wo, stages)] indexed by schedule id."""
    n = ctypes.c_int()
    _check(lib().hyena_conv_schedules(ctypes.byref(n)))
    out = []
    for i in range(n.value):
        info = (ctypes.c_int * 6)()
        _check(lib().hyena_conv_schedule_info(i, info))
        out.append(tuple(info))
    return out


def hyena_conv_schedule_taps(sched: int) -> int:
    """0 for a schedule that streams NTT-domain weights, else the most taps per
    weight word it synthesizes."""
    r = lib().hyena_conv_schedule_taps(sched)
    if r < 0:
        _check(r)
    return r


def synth_taps_words(desc: ConvDesc) -> int:
    """int32 words of the integer-tap array [Co][w_groups][T4]."""
    T = desc.ci * desc.k * desc.k
    return desc.Co * desc.w_groups * ((T + 3) & ~3)


def hyena_synth_taps(ctx: Ctx, desc: ConvDesc, d_w, d_taps, stream=None) -> None:
    _need(d_taps, synth_taps_words(desc), "d_taps")
    _check(lib().hyena_synth_taps(ctx.handle, ctypes.byref(desc), _dev_ptr(d_w, "int8"), _dev_ptr(d_taps, "int32"),
                                  _stream(stream)))


def hyena_conv_synth(ctx: Ctx, desc: ConvDesc, d_ct_ntt, d_taps, d_out_ntt, stream=None) -> None:
    _check(lib().hyena_conv_synth(ctx.handle, ctypes.byref(desc), _dev_ptr(d_ct_ntt, "int32"),
                                  _dev_ptr(d_taps, "int32"), _dev_ptr(d_out_ntt, "int32"), _stream(stream)))


def hyena_conv_default_schedule(desc: ConvDesc) -> int:
    return lib().hyena_conv_default_schedule(ctypes.byref(desc))


def wntt_words(ctx: Ctx, desc: ConvDesc) -> int:
    """uint32 words of the encoded-weight array [Co][w_groups][L][N]."""
    return desc.Co * desc.w_groups * ctx.L * ctx.N


def u32_view(t):
    """Reinterpret an int32 device tensor's words as unsigned (host numpy side)."""
    return t.cpu().numpy().view(np.uint32)


# ---------------------------------------------------------------------------
# batched path
# ---------------------------------------------------------------------------

class Batch:
    """Owns a hyena_batch handle and keeps the descriptors and buffers alive."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.hyena_batch_destroy(h)
            self.handle = None


def hyena_batch_create(ctx: Ctx, layers, flags: int = 0) -> Batch:
    """layers: list of (ConvDesc, d_ct, d_wntt, d_out) or (ConvDesc, d_ct,
    d_wntt, d_out, d_taps) with int32 device tensors; d_wntt or d_taps may be
    None (not both)."""
    arr = (LayerIO * len(layers))()
    keep = []
    for i, lay in enumerate(layers):
        desc, d_ct, d_wn, d_out = lay[:4]
        d_taps = lay[4] if len(lay) > 4 else None
        arr[i].desc = ctypes.cast(ctypes.pointer(desc), ctypes.c_void_p)
        arr[i].d_ct = _dev_ptr(d_ct, "int32")
        arr[i].d_wntt = _dev_ptr(d_wn, "int32") if d_wn is not None else None
        arr[i].d_out = _dev_ptr(d_out, "int32")
        arr[i].d_taps = _dev_ptr(d_taps, "int32") if d_taps is not None else None
        keep.append((desc, d_ct, d_wn, d_out, d_taps))
    out = ctypes.c_void_p()
    _check(lib().hyena_batch_create(ctx.handle, arr, len(layers), flags, ctypes.byref(out)))
    return Batch(out, (ctx, keep))


def hyena_batch_run(b: Batch, stream=None) -> None:
    _check(lib().hyena_batch_run(b.handle, _stream(stream)))


def hyena_batch_info(b: Batch) -> dict:
    n = 5 + 256
    info = (ctypes.c_int * n)()
    _check(lib().hyena_batch_info(b.handle, info, n))
    nl = info[3]
    return {"ntt_fwd": info[0], "ntt_inv": info[1], "launches": info[2], "layers": nl,
            "persistent_launches": info[4], "mac_sched": [info[5 + i] for i in range(nl)]}


def hyena_batch_phase_ms(b: Batch) -> list:
    ms = (ctypes.c_float * 3)()
    _check(lib().hyena_batch_phase_ms(b.handle, ms))
    return [ms[0], ms[1], ms[2]]


def hyena_batch_destroy(b: Batch) -> None:
    if b.handle:
        lib().hyena_batch_destroy(b.handle)
        b.handle = None


# ---------------------------------------------------------------------------
# cost-model MLP kernels
# ---------------------------------------------------------------------------

def hyena_mlp_params() -> int:
    return int(lib().hyena_mlp_params())


def hyena_mlp_workspace_floats(B: int) -> int:
    return int(lib().hyena_mlp_workspace_floats(B))


def hyena_mlp_forward(d_theta, d_x, d_y, stream=None) -> None:
    B = d_x.shape[0]
    _check(lib().hyena_mlp_forward(_dev_ptr(d_theta, "float32"), _dev_ptr(d_x, "float32"), B,
                                   _dev_ptr(d_y, "float32"), _stream(stream)))


def hyena_mlp_loss_grad(d_theta, d_x, d_t, d_grad, d_loss, d_work, stream=None) -> None:
    B = d_x.shape[0]
    _check(lib().hyena_mlp_loss_grad(_dev_ptr(d_theta, "float32"), _dev_ptr(d_x, "float32"),
                                     _dev_ptr(d_t, "float32"), B, _dev_ptr(d_grad, "float32"),
                                     _dev_ptr(d_loss, "float32") if d_loss is not None else None,
                                     _dev_ptr(d_work, "float32"), _stream(stream)))


def hyena_mlp_adam(d_theta, d_grad, d_m, d_v, step: int, lr: float, beta1: float = 0.9,
                   beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    _check(lib().hyena_mlp_adam(_dev_ptr(d_theta, "float32"), _dev_ptr(d_grad, "float32"),
                                _dev_ptr(d_m, "float32"), _dev_ptr(d_v, "float32"), step, lr, beta1, beta2,
                                eps, _stream(stream)))


VALU_OPS = ("v_mad_u64_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_add_u32")


def hyena_valu_rate(op: int, d_out, blocks: int = 8192, iters: int = 2048) -> float:
    """Measured lane operations per second of VALU_OPS[op] (d_out: int32 device
    tensor of blocks * 256 elements)."""
    _need(d_out, blocks * 256, "d_out")
    ms = ctypes.c_float()
    ops = ctypes.c_double()
    _check(lib().hyena_valu_rate(op, blocks, iters, _dev_ptr(d_out, "int32"), ctypes.byref(ms), ctypes.byref(ops)))
    return ops.value / (ms.value * 1e-3)
