"""Oracle: a plain, slow CPU reference for the Hyena homomorphic convolution.

Roh & Choi, "Hyena: Optimizing Homomorphically Encrypted Convolution for
Private CNN Inference" (ICCAD 2024).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU library (``paper_2311_12519_amd``) and never imports it.

What it computes, in the paper's terms:

* BFV symmetric key generation, encryption and decryption (the "Homomorphic
  Operations in BFV" section: the symmetric-encryption and decryption
  equations), with a ternary secret, a B-bounded rounded Gaussian error
  (B = 10 sigma) and a centered message.
* The coefficient encoding of zero-padded input tensors and the kernel
  polynomials of the padded convolution (the "Prior Art on
  Homomorphic Convolution" section: channels padded with zeros, kernel elements used
  as scalars), in the exact geometry written out in ``plan``.
* The homomorphic convolution as its plain definition: for every output
  channel o and tile, sum over input ciphertexts g of ct_g * K_{o,g} in
  Z_q[X]/(X^N+1), by schoolbook products over the nonzero taps.
* The plaintext convolution it must reproduce (the method does not change
  the inference result: introduction and "Optimal Parameter Selection").
* The Walsh-Hadamard matrix and Walsh weights of the "Enabling Output
  Channel Packing" section (Eq. (hadamard2) and its generalisation to c_n = 2^k).
* The negacyclic NTT by O(N^2) evaluation at the odd powers of psi.

Readings of the paper this oracle adopts where the paper is silent or uses
another setting: coefficient encoding with t = 2^20 instead of SIMD batch
encoding (a power-of-two t admits no batching); a ternary secret instead of
{0, 1}; centered messages in (-t/2, t/2]; the 1/c_n of Eq. (hadamard2) as
the inverse of c_n mod q_i; decryption rounding half up (no tie can occur,
q odd and t a power of two).

Every function that is pinned by a test against something other than itself
is noted as such in tests/test_oracle_pins.py; no function here is "parity
unpinned".
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

T_DEFAULT_LOG2 = 20      # plaintext modulus t = 2^20
SIGMA = 3.2              # error standard deviation
B_ERR = 32               # error bound B = 10 sigma (rounded down to an integer)
GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


# ---------------------------------------------------------------------------
# build / load the C helpers
# ---------------------------------------------------------------------------

def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        import subprocess
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wextra", "-Werror",
                               "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _c():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        u32 = ctypes.c_uint32
        lib.orc_negacyclic_mul.argtypes = [P, P, P, u32, u32]
        lib.orc_conv_products.argtypes = [P, u32, u32, u32, u32, P, P, P, P, u32, P, P, P]
        lib.orc_ntt_eval.argtypes = [P, P, u32, u32, u32, P, u32]
        lib.orc_intt_eval.argtypes = [P, P, u32, u32, u32]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# parameters: primes, roots, security, noise
# ---------------------------------------------------------------------------

def is_prime(n: int) -> bool:
    """Trial division (n < 2^32 here)."""
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    f = 3
    while f * f <= n:
        if n % f == 0:
            return False
        f += 2
    return True


def ntt_primes(N: int, L: int, bits: int = 31) -> list:
    """The L largest primes q < 2^bits with q = 1 mod 2N, in descending order.

    q = 1 mod 2N is what the negacyclic NTT needs (the "Optimal Parameter Selection" section, step 1 of the
    parameter selection: q = 1 mod 2n)."""
    out = []
    q = ((1 << bits) - 1) // (2 * N) * (2 * N) + 1
    while len(out) < L:
        if q >= (1 << bits):
            q -= 2 * N
            continue
        if is_prime(q):
            out.append(q)
        q -= 2 * N
    return out


def find_psi(q: int, N: int) -> int:
    """Smallest integer x >= 2 with x^N = -1 mod q (a primitive 2N-th root)."""
    x = 2
    while pow(x, N, q) != q - 1:
        x += 1
    return x


# 128-bit security ceiling on log2(q) for a ternary secret (the public
# Homomorphic Encryption Security Standard, Albrecht et al. 2018, Table
# "uniform ternary", 128-bit column). The paper itself only states that its
# parameters meet 128-bit security (the "Evaluation Setup" section).
SECURITY_LOGQ_128 = {1024: 27, 2048: 54, 4096: 109, 8192: 218, 16384: 438, 32768: 881}


def bitrev(x: int, logn: int) -> int:
    r = 0
    for i in range(logn):
        r |= ((x >> i) & 1) << (logn - 1 - i)
    return r


# ---------------------------------------------------------------------------
# counter-based random numbers (SplitMix64; Steele, Lea & Flood, OOPSLA 2014)
# ---------------------------------------------------------------------------

def sm64(key: int, ctr) -> np.ndarray:
    """Output number ctr (0-based) of a SplitMix64 generator seeded with key:
    the state after ctr+1 increments by the golden gamma, then the finaliser."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key & MASK64) + (ctr + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _uniform_mod(r: np.ndarray, q: int) -> np.ndarray:
    """floor(r * q / 2^64) for 64-bit r (multiply-shift), exact."""
    r = r.astype(np.uint64)
    hi = r >> np.uint64(32)
    lo = r & np.uint64(0xFFFFFFFF)
    qq = np.uint64(q)
    return ((hi * qq + ((lo * qq) >> np.uint64(32))) >> np.uint64(32)).astype(np.uint64)


def gaussian_cdt() -> list:
    """Integer thresholds of the cumulative distribution of the rounded Gaussian
    restricted to [-B, B]: P(x) proportional to exp(-x^2 / (2 sigma^2)).
    T[k] = floor(2^63 * cum_k / S), accumulated from x = -B upward."""
    cums = []
    cum = 0.0
    for x in range(-B_ERR, B_ERR + 1):
        cum += math.exp(-(x * x) / (2.0 * SIGMA * SIGMA))
        cums.append(cum)
    S = cums[-1]
    return [int(c / S * 9223372036854775808.0) for c in cums]


_CDT = None


def sample_error(key: int, ctr: np.ndarray) -> np.ndarray:
    """e = -B + #{k < 2B : u >= T[k]}, u = the top 63 bits of sm64(key, ctr)."""
    global _CDT
    if _CDT is None:
        _CDT = np.array(gaussian_cdt()[:-1], dtype=np.uint64)
    u = sm64(key, ctr) >> np.uint64(1)
    return (np.searchsorted(_CDT, u, side="right").astype(np.int64) - B_ERR)


# ---------------------------------------------------------------------------
# BFV key generation, encryption, decryption (the "Homomorphic Operations in BFV" section)
# ---------------------------------------------------------------------------

def keygen(N: int, seed: int) -> np.ndarray:
    """Ternary secret s_j = floor(3 * hi32(sm64(seed, j)) / 2^32) - 1."""
    r = sm64(seed, np.arange(N, dtype=np.uint64)) >> np.uint64(32)
    return ((r * np.uint64(3)) >> np.uint64(32)).astype(np.int64).astype(np.int8) - np.int8(1)


def negacyclic_mul(a: np.ndarray, b: np.ndarray, q: int) -> np.ndarray:
    """a*b in Z_q[X]/(X^N+1) by dense schoolbook (C helper)."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    r = np.empty_like(a)
    _c().orc_negacyclic_mul(_ptr(a), _ptr(b), _ptr(r), a.shape[0], q)
    return r


def _lift(x: np.ndarray, q: int) -> np.ndarray:
    """Signed integers to canonical residues mod q."""
    return np.mod(np.asarray(x, dtype=np.int64), q).astype(np.uint32)


def encrypt(primes, log2_t: int, s: np.ndarray, msgs: np.ndarray, seed: int) -> np.ndarray:
    """Symmetric BFV: c0 = [Delta*m + a*s + e]_q, c1 = [-a]_q, Delta = floor(q/t).

    msgs: int [n][N] centered in (-t/2, t/2]. Returns uint32 [n][2][L][N].
    a_{n,i,j} = floor(q_i * sm64(seed, 2*((n*L+i)*N+j)) / 2^64) (uniform per limb,
    so uniform mod q by the CRT); e_{n,j} from sm64(seed, 2*(n*N+j)+1)."""
    msgs = np.asarray(msgs, dtype=np.int64)
    n, N = msgs.shape
    L = len(primes)
    q = math.prod(primes)
    delta = q // (1 << log2_t)
    out = np.empty((n, 2, L, N), dtype=np.uint32)
    j = np.arange(N, dtype=np.uint64)
    for m in range(n):
        e = sample_error(seed, np.uint64(2) * (np.uint64(m * N) + j) + np.uint64(1))
        for i, qi in enumerate(primes):
            a = _uniform_mod(sm64(seed, np.uint64(2) * (np.uint64((m * L + i) * N) + j)), qi)
            a = a.astype(np.uint32)
            as_ = negacyclic_mul(a, _lift(s, qi), qi).astype(np.uint64)
            dm = (np.uint64(delta % qi) * _lift(msgs[m], qi).astype(np.uint64)) % np.uint64(qi)
            c0 = (dm + as_ + _lift(e, qi).astype(np.uint64)) % np.uint64(qi)
            out[m, 0, i] = c0.astype(np.uint32)
            out[m, 1, i] = ((np.uint64(qi) - a.astype(np.uint64)) % np.uint64(qi)).astype(np.uint32)
    return out


def crt(residues, primes) -> list:
    """Exact CRT: residues [L][N] -> list of N Python ints in [0, q)."""
    q = math.prod(primes)
    acc = np.zeros(residues[0].shape[0], dtype=object)
    for r_i, qi in zip(residues, primes):
        Mi = q // qi
        yi = pow(Mi, -1, qi)
        acc = acc + np.asarray(r_i, dtype=np.uint64).astype(object) * (Mi * yi)
    return [int(v) % q for v in acc]


def decrypt_phase(primes, s: np.ndarray, ct: np.ndarray) -> list:
    """v = [c0 + c1*s]_q as exact integers in [0, q), one ciphertext [2][L][N]."""
    res = []
    for i, qi in enumerate(primes):
        c1s = negacyclic_mul(ct[1, i], _lift(s, qi), qi).astype(np.uint64)
        res.append(((ct[0, i].astype(np.uint64) + c1s) % np.uint64(qi)))
    return crt(res, primes)


def decrypt(primes, log2_t: int, s: np.ndarray, ct: np.ndarray) -> np.ndarray:
    """m = [round(t * [c0 + c1 s]_q / q)]_t, centered in (-t/2, t/2].

    ct: uint32 [n][2][L][N] -> int64 [n][N]. Rounding is half up; a tie
    cannot occur because q is odd and t a power of two."""
    ct = np.asarray(ct)
    q = math.prod(primes)
    t = 1 << log2_t
    out = np.empty((ct.shape[0], ct.shape[-1]), dtype=np.int64)
    for m in range(ct.shape[0]):
        v = decrypt_phase(primes, s, ct[m])
        vals = [((t * x + q // 2) // q) % t for x in v]
        out[m] = [x - t if x > t // 2 else x for x in vals]
    return out


def noise_inf(primes, log2_t: int, s: np.ndarray, ct: np.ndarray, msg: np.ndarray) -> int:
    """||v||_inf for one ciphertext: v = [c0 + c1 s - Delta m]_q, centered."""
    q = math.prod(primes)
    delta = q // (1 << log2_t)
    v = decrypt_phase(primes, s, ct)
    worst = 0
    for x, mm in zip(v, np.asarray(msg, dtype=np.int64)):
        d = (x - delta * int(mm)) % q
        if d > q // 2:
            d -= q
        worst = max(worst, abs(d))
    return worst


# ---------------------------------------------------------------------------
# geometry of the coefficient-encoded padded convolution
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Plan:
    N: int
    H: int
    W: int
    Ci: int
    Co: int
    k: int
    depthwise: bool
    pad: int
    Wp: int      # padded width W + 2p
    R: int       # output rows per tile
    tiles: int
    Bt: int      # coefficients per packed channel block, (R + 2p) * Wp
    ci: int      # channels per input ciphertext
    n_groups: int
    O: int       # offset of the first valid output coefficient


def plan(N: int, H: int, W: int, Ci: int, Co: int, k: int, depthwise: bool = False,
         ci: int | None = None) -> Plan:
    """Geometry: channels zero-padded by p = (k-1)/2 and packed back to back.

    If one padded channel fits, c_i padded channels share a ciphertext
    (the "Prior Art on Homomorphic Convolution" section: C x H x W split over ceil(CHW/n) ciphertexts, here with
    padding); otherwise one channel is split into row tiles of R output rows
    with a 2p-row halo. ``ci`` may lower the channels per ciphertext."""
    if k not in (1, 3) or N & (N - 1):
        raise ValueError("k must be 1 or 3 and N a power of two")
    if depthwise and Ci != Co:
        raise ValueError("depthwise needs Ci == Co")
    p = (k - 1) // 2
    Wp = W + 2 * p
    if (H + 2 * p) * Wp <= N:
        R, tiles, Bt = H, 1, (H + 2 * p) * Wp
        cmax = min(Ci, N // Bt)
        c = cmax if ci is None else ci
        if not 1 <= c <= cmax:
            raise ValueError("channel partition out of range")
    else:
        R = N // Wp - 2 * p
        if R < 1:
            raise ValueError("padded row does not fit the ring")
        tiles = -(-H // R)
        Bt = (R + 2 * p) * Wp
        c = 1
        if ci not in (None, 1):
            raise ValueError("row-tiled layers carry one channel per ciphertext")
    n_groups = -(-Ci // c)
    O = (c - 1) * Bt + (k - 1) * Wp + (k - 1)
    return Plan(N, H, W, Ci, Co, k, depthwise, p, Wp, R, tiles, Bt, c, n_groups, O)


def pad_input(x: np.ndarray, p: int) -> np.ndarray:
    C, H, W = x.shape
    xp = np.zeros((C, H + 2 * p, W + 2 * p), dtype=np.int64)
    xp[:, p:p + H, p:p + W] = x
    return xp


def pack_input(pl: Plan, x: np.ndarray) -> np.ndarray:
    """Messages int64 [tiles][n_groups][N]:
    m_{tau,g}[c'*Bt + r*Wp + col] = x_pad[g*ci + c'][tau*R + r][col],
    for r < R + 2p and col < Wp; rows past the padded image are zero."""
    xp = pad_input(np.asarray(x, dtype=np.int64), pl.pad)
    Hp = xp.shape[1]
    out = np.zeros((pl.tiles, pl.n_groups, pl.N), dtype=np.int64)
    for tau in range(pl.tiles):
        for g in range(pl.n_groups):
            for c in range(pl.ci):
                ch = g * pl.ci + c
                if ch >= pl.Ci:
                    break
                for r in range(pl.R + 2 * pl.pad):
                    row = tau * pl.R + r
                    if row >= Hp:
                        break
                    base = c * pl.Bt + r * pl.Wp
                    out[tau, g, base:base + pl.Wp] = xp[ch, row]
    return out


def kernel_taps(pl: Plan, w: np.ndarray):
    """Nonzero taps of every kernel polynomial K_{o,g}:
    K_{o,g}(X) = sum_{c',di,dj} f[o][g*ci+c'][di][dj] * X^(O - c'*Bt - di*Wp - dj).

    Returns CSR arrays (tap_ptr int64 [Co*n_groups+1], tap_exp uint32, tap_w int32).
    Depthwise layers (w: [C][1][k][k]) only have the tap block of c' = o - g*ci."""
    w = np.asarray(w, dtype=np.int64)
    ptr = [0]
    exps, ws = [], []
    for o in range(pl.Co):
        for g in range(pl.n_groups):
            for c in range(pl.ci):
                ch = g * pl.ci + c
                if ch >= pl.Ci:
                    break
                if pl.depthwise and ch != o:
                    continue
                for di in range(pl.k):
                    for dj in range(pl.k):
                        f = int(w[o, 0 if pl.depthwise else ch, di, dj])
                        if f == 0:
                            continue
                        exps.append(pl.O - c * pl.Bt - di * pl.Wp - dj)
                        ws.append(f)
            ptr.append(len(exps))
    return (np.array(ptr, dtype=np.int64), np.array(exps, dtype=np.uint32),
            np.array(ws, dtype=np.int32))


def kernel_poly(pl: Plan, w: np.ndarray, o: int, g: int) -> np.ndarray:
    """K_{o,g} as a dense signed integer polynomial int64 [N]."""
    ptr, exps, ws = kernel_taps(pl, w)
    K = np.zeros(pl.N, dtype=np.int64)
    s, e = ptr[o * pl.n_groups + g], ptr[o * pl.n_groups + g + 1]
    for t in range(s, e):
        K[exps[t]] += ws[t]
    return K


def conv_products(pl: Plan, ct: np.ndarray, w: np.ndarray, primes, outputs=None) -> np.ndarray:
    """Y_{tau,o} = sum_g ct_{tau,g} * K_{o,g} mod (X^N+1, q_i), both parts, all limbs.

    ct: uint32 [tiles][n_groups][2][L][N] (coefficient domain).
    outputs: list of (tau, o) or None for all, in order tau-major then o.
    Returns uint32 [n_sel][2][L][N]."""
    ct = np.ascontiguousarray(ct, dtype=np.uint32)
    L = len(primes)
    assert ct.shape == (pl.tiles, pl.n_groups, 2, L, pl.N)
    if outputs is None:
        outputs = [(tau, o) for tau in range(pl.tiles) for o in range(pl.Co)]
    sel_t = np.array([u[0] for u in outputs], dtype=np.uint32)
    sel_o = np.array([u[1] for u in outputs], dtype=np.uint32)
    ptr, exps, ws = kernel_taps(pl, w)
    if len(exps) == 0:
        exps = np.zeros(1, dtype=np.uint32)
        ws = np.zeros(1, dtype=np.int32)
    pr = np.array(primes, dtype=np.uint32)
    out = np.empty((len(outputs), 2, L, pl.N), dtype=np.uint32)
    _c().orc_conv_products(_ptr(ct), pl.tiles, pl.n_groups, L, pl.N, _ptr(pr),
                           _ptr(ptr), _ptr(exps), _ptr(ws), len(outputs),
                           _ptr(sel_t), _ptr(sel_o), _ptr(out))
    return out


def direct_conv(x: np.ndarray, w: np.ndarray, k: int, depthwise: bool = False) -> np.ndarray:
    """Stride-1 'same' cross-correlation over Z (zero padding p = (k-1)/2):
    y[o][i][j] = sum_{c,di,dj} x_pad[c][i+di][j+dj] * f[o][c][di][dj]."""
    p = (k - 1) // 2
    x = np.asarray(x, dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    C, H, W = x.shape
    xp = pad_input(x, p)
    Co = w.shape[0]
    y = np.zeros((Co, H, W), dtype=np.int64)
    for di in range(k):
        for dj in range(k):
            win = xp[:, di:di + H, dj:dj + W]           # [C][H][W]
            if depthwise:
                y += w[:, 0, di, dj][:, None, None] * win
            else:
                y += np.einsum("oc,chw->ohw", w[:, :, di, dj], win)
    return y


def unpack_output(pl: Plan, msgs: np.ndarray) -> np.ndarray:
    """Decrypted outputs [tiles][Co][N] -> stride-1 y [Co][H][W]:
    y[o][tau*R + r][col] = m_{tau,o}[O + r*Wp + col]."""
    msgs = np.asarray(msgs)
    y = np.zeros((pl.Co, pl.H, pl.W), dtype=np.int64)
    for tau in range(pl.tiles):
        for r in range(pl.R):
            row = tau * pl.R + r
            if row >= pl.H:
                break
            base = pl.O + r * pl.Wp
            y[:, row, :] = msgs[tau, :, base:base + pl.W]
    return y


def subsample(y: np.ndarray, stride: int) -> np.ndarray:
    """Strided layers: the stride-s output is y_s1[:, ::s, ::s]."""
    return y[:, ::stride, ::stride]


def max_abs_output(pl: Plan, w: np.ndarray, xmax: int = 8) -> int:
    """Worst-case |y| over inputs with |x| <= xmax."""
    w = np.abs(np.asarray(w, dtype=np.int64))
    return int(xmax * w.reshape(w.shape[0], -1).sum(axis=1).max())


def noise_ok(pl: Plan, w: np.ndarray, primes, log2_t: int = T_DEFAULT_LOG2) -> bool:
    """Decryption of every output is exact if the worst-case noise of the
    product, E = sum_g e_g K_{o,g} with |e| <= B, and the rounding term of the
    centered lift keep t*|E| + r*|Y| < q/2, r = q mod t (decryption-correctness
    condition ||v|| < Delta/2 of the "Homomorphic Operations in BFV" section), and |y| < t/2."""
    q = math.prod(primes)
    t = 1 << log2_t
    w = np.abs(np.asarray(w, dtype=np.int64))
    l1 = int(w.reshape(w.shape[0], -1).sum(axis=1).max())   # max_o ||K_o||_1 over all g
    ymax = max_abs_output(pl, w)
    return 2 * (t * B_ERR * l1 + (q % t) * ymax) < q and 2 * ymax < t


# ---------------------------------------------------------------------------
# Walsh-Hadamard output-channel packing (the "Enabling Output Channel Packing" section)
# ---------------------------------------------------------------------------

def walsh_matrix(c_n: int) -> np.ndarray:
    """Sylvester construction: H_1 = [1], H_2m = [[H_m, H_m], [H_m, -H_m]]."""
    if c_n < 1 or c_n & (c_n - 1):
        raise ValueError("c_n must be a power of two")
    H = np.array([[1]], dtype=np.int64)
    while H.shape[0] < c_n:
        H = np.block([[H, H], [H, -H]])
    return H


def walsh_weights(w: np.ndarray, c_n: int) -> np.ndarray:
    """g[G*c_n + j] = sum_b H[j][b] * f[G*c_n + b] along the output-channel axis
    (the integers stored instead of plaintexts: Eq. (hadamard2) generalised)."""
    w = np.asarray(w, dtype=np.int64)
    Co = w.shape[0]
    if Co % c_n:
        raise ValueError("c_n must divide Co")
    H = walsh_matrix(c_n)
    blocks = w.reshape(Co // c_n, c_n, -1)
    return np.einsum("jb,Gbx->Gjx", H, blocks).reshape(w.shape)


def walsh_kernel_residues(pl: Plan, w: np.ndarray, c_n: int, primes, G: int, j: int, g: int) -> np.ndarray:
    """Coefficient-domain Walsh kernel c_n^{-1} * Kw_{G,j,g} mod q_i, uint32 [L][N].

    Kw_{G,j,g} = sum_b H[j][b] K_{G*c_n+b, g}: the Walsh components of the c_n
    per-output-channel kernel polynomials (Eq. (hadamard2) applied to the
    polynomials that carry [f0, f1]). For a standard layer this is the kernel
    polynomial of the Walsh weights; for a depthwise layer the c_n terms sit
    at the c_n different channel positions. The factor 1/c_n of Eq.
    (hadamard2) is the inverse of c_n mod q_i."""
    H = walsh_matrix(c_n)
    K = np.zeros(pl.N, dtype=np.int64)
    for b in range(c_n):
        K += int(H[j, b]) * kernel_poly(pl, w, G * c_n + b, g)
    out = np.empty((len(primes), pl.N), dtype=np.uint32)
    for i, qi in enumerate(primes):
        inv = pow(c_n, -1, qi)
        out[i] = ((_lift(K, qi).astype(np.uint64) * np.uint64(inv)) % np.uint64(qi)).astype(np.uint32)
    return out


# ---------------------------------------------------------------------------
# negacyclic NTT by direct evaluation
# ---------------------------------------------------------------------------

def ntt(a: np.ndarray, q: int, psi: int, ks=None) -> np.ndarray:
    """A[k] = sum_j a[j] psi^((2 brv(k) + 1) j) mod q, for all k or the listed ks."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    N = a.shape[0]
    if ks is None:
        out = np.empty(N, dtype=np.uint32)
        _c().orc_ntt_eval(_ptr(a), _ptr(out), N, q, psi, None, 0)
    else:
        ks = np.ascontiguousarray(ks, dtype=np.uint32)
        out = np.empty(ks.shape[0], dtype=np.uint32)
        _c().orc_ntt_eval(_ptr(a), _ptr(out), N, q, psi, _ptr(ks), ks.shape[0])
    return out


def intt(A: np.ndarray, q: int, psi: int) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.uint32)
    out = np.empty_like(A)
    _c().orc_intt_eval(_ptr(A), _ptr(out), A.shape[0], q, psi)
    return out
