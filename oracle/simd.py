"""Oracle for the SIMD (batch-encoded) BFV pieces of the paper's own setting.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
it. It shares no code with the GPU library and never imports it.

What it computes, in the paper's terms:

* SIMD batch encoding with a prime plaintext modulus p = 1 mod 2n (the
  "Homomorphic Operations in BFV" section: slots are the CRT components of
  R_p; step 1 of the "Optimal Parameter Selection" procedure), by its plain
  definition: the plaintext polynomial m with m(zeta^{e_s}) = v_s mod p for
  every slot s, zeta the least primitive 2n-th root of unity mod p.
* The plaintext packing [1, -1] (first half of the slots 1, second half -1)
  and its two equal nonzero coefficients h_{p,n}; the plaintext packing
  [k, -k] and the search for the k that minimises k h_{p,n} mod p (steps 2
  and 3 of the "Optimal Parameter Selection" procedure).
* The worst-case noise factors of PMult quoted in that section: n p / 2 for a
  general plaintext, (f0 + f1 + 2 (f0 - f1) c) / 2 for the Walsh form with the
  [1, -1] (c = h) or [k, -k] (c = k h mod p) plaintext.
* The model storage of the "Enabling Output Channel Packing" section's
  example: one plaintext polynomial plus one word per kernel element, against
  one plaintext polynomial per kernel element.
* Galois automorphisms a(X) -> a(X^g) in R_q (the map behind HRot, "Homomorphic
  Operations in BFV") and PMult by a plaintext in R_q (a negacyclic product).
* HRot with a decomposition base 2^b and hoisting (key generation and key
  switching, RNS-BV digits of each limb's residues).
* BFV with a prime plaintext modulus p, and CMult + HAdd by integer scalars.
* The convolution with c_n = 2 channels per ciphertext ("Enabling Output
  Channel Packing", Eq. (hadamard2), with the [k, -k] plaintext), with and
  without output channel packing, over any number of input ciphertexts.

Readings where the paper is silent: slot s < n/2 holds the value at
zeta^(3^s mod 2n) and slot n/2 + s the value at zeta^(-3^s mod 2n) (the
generator-3 two-row layout of the batch encoder used with the paper's
parameters; with the least primitive root it gives the paper's
h_{2048,307201} = 84248); plaintext coefficients enter PMult as integers in
[0, p), the representation the paper's "minimise k h mod p" criterion
measures; the 1/2 of Eq. (hadamard2) is left out (every output carries the
factor 2, as it carries k); one input channel per slot row, in a
zero-bordered frame of power-of-two width, kernel offsets as row rotations.
"""
from __future__ import annotations

import math

import numpy as np

from . import find_psi, negacyclic_mul


def primitive_root_2n(p: int, n: int) -> int:
    """The least integer zeta >= 2 with zeta^n = -1 mod p."""
    return find_psi(p, n)


def slot_exponents(n: int) -> np.ndarray:
    """e_s for s < n: 3^s mod 2n for the first row, -3^s mod 2n for the second."""
    row = np.empty(n // 2, dtype=np.int64)
    g = 1
    for s in range(n // 2):
        row[s] = g
        g = g * 3 % (2 * n)
    return np.concatenate([row, (2 * n - row) % (2 * n)])


def _power_table(z: int, p: int, n: int) -> np.ndarray:
    """z^e mod p for e < 2n."""
    t = np.empty(2 * n, dtype=np.uint64)
    x = 1
    for e in range(2 * n):
        t[e] = x
        x = x * z % p
    return t


def encode(values, p: int, n: int) -> np.ndarray:
    """The polynomial m (coefficients in [0, p)) with m(zeta^{e_s}) = v_s:
    m_k = n^{-1} sum_s v_s zeta^{-e_s k} mod p (the inverse of the evaluation
    at the n distinct roots of X^n + 1). p < 2^24 keeps every sum in 64 bits."""
    assert p < (1 << 24) and (p - 1) % (2 * n) == 0
    v = np.mod(np.asarray(values, dtype=np.int64), p).astype(np.uint64)
    assert v.shape == (n,)
    z = primitive_root_2n(p, n)
    tinv = _power_table(pow(z, p - 2, p), p, n)
    e = slot_exponents(n).astype(np.uint64)
    ks = np.arange(n, dtype=np.uint64)
    m = np.empty(n, dtype=np.uint64)
    for k in range(n):
        m[k] = int((v * tinv[(e * ks[k]) % np.uint64(2 * n)]).sum() % np.uint64(p))
    return (m * np.uint64(pow(n, p - 2, p)) % np.uint64(p)).astype(np.uint32)


def decode(m, p: int, n: int) -> np.ndarray:
    """v_s = m(zeta^{e_s}) mod p."""
    assert p < (1 << 24) and (p - 1) % (2 * n) == 0
    m = np.asarray(m, dtype=np.uint64) % np.uint64(p)
    z = primitive_root_2n(p, n)
    t = _power_table(z, p, n)
    e = slot_exponents(n).astype(np.uint64)
    ks = np.arange(n, dtype=np.uint64)
    out = np.empty(n, dtype=np.uint64)
    for s in range(n):
        out[s] = int((m * t[(e[s] * ks) % np.uint64(2 * n)]).sum() % np.uint64(p))
    return out.astype(np.uint32)


def pm_plaintext(n: int, p: int, k: int = 1) -> np.ndarray:
    """The plaintext packing [k, -k]: k in the first n/2 slots, -k in the rest."""
    return encode([k] * (n // 2) + [-k] * (n // 2), p, n)


def h_pn(n: int, p: int) -> int:
    """h_{p,n}: the common value of the two nonzero coefficients of the
    plaintext packing [1, -1] (at X^{n/4} and X^{3n/4})."""
    m = pm_plaintext(n, p)
    nz = np.flatnonzero(m)
    assert list(nz) == [n // 4, 3 * n // 4] and m[nz[0]] == m[nz[1]], nz
    return int(m[nz[0]])


def best_k(h: int, p: int, kmax: int):
    """(k, k h mod p) with k in [1, kmax] minimising k h mod p (the least such k)."""
    best = None
    for k in range(1, kmax + 1):
        c = k * h % p
        if best is None or c < best[1]:
            best = (k, c)
    return best


def noise_factor_conventional(n: int, p: int) -> float:
    """Worst-case noise growth of PMult by a general plaintext: n p / 2."""
    return n * p / 2


def noise_factor_walsh(f0: int, f1: int, c: int) -> float:
    """Worst-case noise growth of the Walsh form of PMult by [f0, f1]:
    (f0 + f1 + 2 (f0 - f1) c) / 2, c the coefficient of the [1, -1] (or
    [k, -k]) plaintext; magnitudes, so that signed kernel elements count by
    their size."""
    return (abs(f0 + f1) + 2 * abs(f0 - f1) * c) / 2


def storage_bytes(n: int, elements: int, word_bytes: int = 8):
    """(proposed, conventional) model storage: one plaintext polynomial of n
    words plus one word per kernel element, against one plaintext polynomial
    per kernel element."""
    return n * word_bytes + elements * word_bytes, elements * n * word_bytes


def automorphism(a, g: int, q: int) -> np.ndarray:
    """a(X^g) in Z_q[X]/(X^n + 1) for odd g: coefficient j moves to j g mod 2n,
    negated when that exponent is n or more (X^n = -1)."""
    a = np.asarray(a, dtype=np.int64)
    n = a.shape[0]
    assert g % 2 == 1
    out = np.zeros(n, dtype=np.int64)
    for j in range(n):
        e = j * g % (2 * n)
        if e < n:
            out[e] = (out[e] + a[j]) % q
        else:
            out[e - n] = (out[e - n] - a[j]) % q
    return out.astype(np.uint32)


def pmult(a, plain, q: int) -> np.ndarray:
    """a * plain in Z_q[X]/(X^n + 1), the plaintext's coefficients taken as the
    integers in [0, p) they are stored as."""
    return negacyclic_mul(np.asarray(a, dtype=np.uint32), np.mod(np.asarray(plain, dtype=np.int64), q).astype(np.uint32),
                          q)


# ---------------------------------------------------------------------------
# HRot: Galois automorphism + key switching with a decomposition base
# ("Homomorphic Operations in BFV": HRot and its decomposition base, which
# trades noise against computation; hoisting: decompose once, rotate many)
# ---------------------------------------------------------------------------

def n_digits(log2_base: int, bits: int = 31) -> int:
    """Digits per residue for base 2^log2_base (residues below 2^bits)."""
    return -(-bits // log2_base)


def galois_keygen(primes, s, g: int, log2_base: int, seed: int) -> np.ndarray:
    """Key-switching key for s(X^g) -> s: uint32 [L*D][2][L][N], coefficient
    domain. Key (i, j) (index i*D + j) is an encryption under s, drawn like the
    encryption of message number i*D + j, of s(X^g) 2^{j log2_base} on limb i
    and 0 on the other limbs (the CRT basis element of limb i is 1 mod q_i and
    0 mod the others): b1 = -a, b0 = a s + e + gadget."""
    from . import _lift, _uniform_mod, sample_error, sm64
    s = np.asarray(s, dtype=np.int64)
    N, L = s.shape[0], len(primes)
    D = n_digits(log2_base)
    jn = np.arange(N, dtype=np.uint64)
    out = np.empty((L * D, 2, L, N), dtype=np.uint32)
    for key in range(L * D):
        i, j = divmod(key, D)
        e = sample_error(seed, np.uint64(2) * (np.uint64(key * N) + jn) + np.uint64(1))
        for k, qk in enumerate(primes):
            a = _uniform_mod(sm64(seed, np.uint64(2) * (np.uint64((key * L + k) * N) + jn)), qk).astype(np.uint32)
            as_ = negacyclic_mul(a, _lift(s, qk), qk).astype(np.uint64)
            v = as_ + _lift(e, qk).astype(np.uint64)
            if k == i:
                sg = automorphism(_lift(s, qk), g, qk).astype(np.uint64)
                v = v + sg * np.uint64(pow(2, log2_base * j, qk))
            out[key, 0, k] = (v % np.uint64(qk)).astype(np.uint32)
            out[key, 1, k] = ((np.uint64(qk) - a.astype(np.uint64)) % np.uint64(qk)).astype(np.uint32)
    return out


def hrot(primes, ct, g: int, keys, log2_base: int) -> np.ndarray:
    """Hoisted HRot of one ciphertext [2][L][N] (coefficient domain):
    c0' = c0(X^g) + sum_{i,j} d_ij(X^g) b0_ij,  c1' = sum_{i,j} d_ij(X^g) b1_ij,
    d_ij the base-2^log2_base digits of limb i's residues of c1 (decomposed
    before the automorphism, so that one decomposition serves every g)."""
    ct = np.asarray(ct, dtype=np.uint32)
    L, N = ct.shape[1], ct.shape[2]
    D = n_digits(log2_base)
    mask = (1 << log2_base) - 1
    out = np.empty_like(ct)
    for k, qk in enumerate(primes):
        acc0 = automorphism(ct[0, k], g, qk).astype(np.int64)
        acc1 = np.zeros(N, dtype=np.int64)
        for i in range(L):
            for j in range(D):
                d = (ct[1, i].astype(np.int64) >> (log2_base * j)) & mask
                dg = automorphism(d % qk, g, qk)
                acc0 = (acc0 + negacyclic_mul(dg, keys[i * D + j, 0, k], qk)) % qk
                acc1 = (acc1 + negacyclic_mul(dg, keys[i * D + j, 1, k], qk)) % qk
        out[0, k], out[1, k] = acc0, acc1
    return out


def hrot_noise_bound(N: int, L: int, log2_base: int, B: int) -> int:
    """Added noise of one key switching: sum over the L*D keys of
    d_ij(X^g) e_ij, each coefficient at most N (2^b - 1) B."""
    return L * n_digits(log2_base) * N * ((1 << log2_base) - 1) * B


# ---------------------------------------------------------------------------
# BFV with a prime plaintext modulus p and the pieces of the SIMD convolution
# ---------------------------------------------------------------------------

def encrypt_p(primes, p: int, s, msgs, seed: int) -> np.ndarray:
    """Symmetric BFV with plaintext modulus p ("Homomorphic Operations in BFV":
    c0 = [Delta m + a s + e]_q, c1 = [-a]_q, Delta = floor(q / p)), drawn like
    the power-of-two encryption (same counters); msgs: [n][N] integers (their
    residues mod p are the message; Delta multiplies the integer as given)."""
    from . import _lift, _uniform_mod, sample_error, sm64
    msgs = np.asarray(msgs, dtype=np.int64)
    n, N = msgs.shape
    L = len(primes)
    delta = math.prod(primes) // p
    out = np.empty((n, 2, L, N), dtype=np.uint32)
    j = np.arange(N, dtype=np.uint64)
    for m in range(n):
        e = sample_error(seed, np.uint64(2) * (np.uint64(m * N) + j) + np.uint64(1))
        for i, qi in enumerate(primes):
            a = _uniform_mod(sm64(seed, np.uint64(2) * (np.uint64((m * L + i) * N) + j)), qi).astype(np.uint32)
            as_ = negacyclic_mul(a, _lift(s, qi), qi).astype(object)
            dm = (np.mod(msgs[m], qi).astype(object) * (delta % qi)) % qi
            out[m, 0, i] = ((dm + as_ + _lift(e, qi).astype(object)) % qi).astype(np.uint32)
            out[m, 1, i] = ((np.uint64(qi) - a.astype(np.uint64)) % np.uint64(qi)).astype(np.uint32)
    return out


def decrypt_p(primes, p: int, s, ct) -> np.ndarray:
    """m = [round(p [c0 + c1 s]_q / q)]_p in [0, p) (no tie: q and p odd)."""
    from . import decrypt_phase
    q = math.prod(primes)
    ct = np.asarray(ct)
    out = np.empty((ct.shape[0], ct.shape[-1]), dtype=np.int64)
    for m in range(ct.shape[0]):
        out[m] = [((p * v + q // 2) // q) % p for v in decrypt_phase(primes, s, ct[m])]
    return out


def cmult_accumulate(ins, W, primes) -> np.ndarray:
    """CMult and HAdd of ciphertexts by integer scalars: out[o] = sum_r W[o][r]
    in[r] mod q_i, ins [R][2][L][N], W [O][R] (signed integers)."""
    ins = np.asarray(ins, dtype=np.uint32)
    W = np.asarray(W, dtype=np.int64)
    out = np.empty((W.shape[0],) + ins.shape[1:], dtype=np.uint32)
    for o in range(W.shape[0]):
        for i, q in enumerate(primes):
            acc = np.zeros(ins.shape[1:2] + ins.shape[3:], dtype=object)
            for r in range(ins.shape[0]):
                acc = acc + int(W[o, r]) * ins[r, :, i, :].astype(object)
            out[o, :, i, :] = (acc % q).astype(np.uint32)
    return out


def frame_slots(x, frame_h: int, frame_w: int) -> np.ndarray:
    """Slot rows of a SIMD input ciphertext packing c_n = 2 channels: channel c
    of x [2][H][W] sits in row c at (1 + i) frame_w + (1 + j) of a
    frame_h x frame_w frame (a zero border of at least one, power-of-two
    width, as the paper's packing assumes)."""
    x = np.asarray(x, dtype=np.int64)
    C, H, W = x.shape
    assert C == 2 and H + 2 <= frame_h and W + 2 <= frame_w
    rows = np.zeros((2, frame_h * frame_w), dtype=np.int64)
    for c in range(2):
        f = np.zeros((frame_h, frame_w), dtype=np.int64)
        f[1:1 + H, 1:1 + W] = x[c]
        rows[c] = f.reshape(-1)
    return rows.reshape(-1)


def conv_rotations(n: int, frame_w: int):
    """Galois exponents of the nine 3x3 offsets (di - 1) frame_w + (dj - 1):
    X -> X^(3^r) moves slot s + r to slot s in both rows."""
    return [pow(3, ((di - 1) * frame_w + (dj - 1)) % (n // 2), 2 * n) for di in range(3) for dj in range(3)]


def simd_conv_cn2(primes, ct, w, k: int, kh: int, frame_w: int, rot_keys, swap_keys, log2_base: int) -> np.ndarray:
    """The paper's convolution with c_n = 2 input channels per ciphertext
    ("Enabling Output Channel Packing", Eq. (hadamard2), and the [k, -k]
    plaintext of "Optimal Parameter Selection"), for a 3x3 kernel
    w [Co][2 G][3][3] over G input ciphertexts ct [G][2][L][N] (ciphertext g
    holds channel 2g in its first slot row, 2g + 1 in its second; a single
    ciphertext [2][L][N] is G = 1):
    1. HRot of every input by the nine kernel offsets (hoisted);
    2. CMult + HAdd: A_o = sum_{g,r} k (f0 + f1)_{g,r} rot_{g,r},
       B_o = sum_{g,r} (f0 - f1)_{g,r} rot_{g,r}, f0 = w[o][2g], f1 = w[o][2g+1];
    3. one PMult of B_o by the [k, -k] plaintext kh (X^{n/4} + X^{3n/4}), added to A_o:
       row 0 then holds 2k sum f0 x0, row 1 2k sum f1 x1 (the 1/2 of Eq.
       (hadamard2) is left out: every output carries the same factor 2, like k);
    4. HRot by X^{2n-1} (the row swap) and HAdd, aligning the two rows' partial
       sums: both rows of output o hold 2k conv(x)_o.
    rot_keys: {g: key} for the nine exponents of conv_rotations; swap_keys: the
    key for 2n - 1. Returns [Co][2][L][N]."""
    ct = np.asarray(ct, dtype=np.uint32)
    if ct.ndim == 3:
        ct = ct[None]
    G, n = ct.shape[0], ct.shape[-1]
    gs = conv_rotations(n, frame_w)
    rots = np.stack([hrot(primes, ct[g], r, rot_keys[r], log2_base) for g in range(G) for r in gs])
    w = np.asarray(w, dtype=np.int64)
    Co = w.shape[0]
    out = np.empty((Co,) + ct.shape[1:], dtype=np.uint32)
    wpm = np.zeros(n, dtype=np.int64)
    wpm[n // 4] = wpm[3 * n // 4] = kh
    for o in range(Co):
        f0 = w[o, 0::2].reshape(G * 9)              # index g*9 + r, matching rots
        f1 = w[o, 1::2].reshape(G * 9)
        A, B = cmult_accumulate(rots, np.stack([k * (f0 + f1), f0 - f1]), primes)
        Z = np.empty_like(A)
        for part in range(2):
            for i, q in enumerate(primes):
                Z[part, i] = (A[part, i].astype(np.uint64) + pmult(B[part, i], wpm, q)) % np.uint64(q)
        Zs = hrot(primes, Z, 2 * n - 1, swap_keys, log2_base)
        out[o] = cmult_accumulate(np.stack([Z, Zs]), np.array([[1, 1]]), primes)[0]
    return out


def simd_conv_cn2_packed(primes, ct, w, k: int, kh: int, frame_w: int, rot_keys, swap_keys,
                         log2_base: int) -> np.ndarray:
    """The convolution with c_n = 2 channels per ciphertext on both sides
    (output channel packing, "Enabling Output Channel Packing": each PMult by a
    two-valued plaintext [a | b] in its Walsh form (k (a + b)) CMult +
    PMult((a - b) CMult, [k, -k])), for a 3x3 kernel w [Co][2 G][3][3], Co even:
    1. HRot of every input by X^{2n-1} (the row swap): sct_g holds channel
       2g + 1 in its first row and 2g in its second;
    2. hoisted HRot of every ct_g and sct_g by the nine kernel offsets;
    3. for output pair (o, o + 1), with a the first row's and b the second
       row's weights (ct_g: a = w[o][2g], b = w[o+1][2g+1]; sct_g:
       a = w[o][2g+1], b = w[o+1][2g]):
       A = sum k (a + b) rot, B = sum (a - b) rot, out = A + PMult(B, [k, -k]);
       the first row of out holds 2k conv(x)_o, the second 2k conv(x)_{o+1}.
    Returns [Co/2][2][L][N]."""
    ct = np.asarray(ct, dtype=np.uint32)
    if ct.ndim == 3:
        ct = ct[None]
    G, n = ct.shape[0], ct.shape[-1]
    sct = np.stack([hrot(primes, ct[g], 2 * n - 1, swap_keys, log2_base) for g in range(G)])
    gs = conv_rotations(n, frame_w)
    srcs = np.concatenate([ct, sct])                  # h = 0: ct_g, h = 1: sct_g
    rots = np.stack([hrot(primes, srcs[j], r, rot_keys[r], log2_base) for j in range(2 * G) for r in gs])
    w = np.asarray(w, dtype=np.int64)
    Co = w.shape[0]
    out = np.empty((Co // 2,) + ct.shape[1:], dtype=np.uint32)
    wpm = np.zeros(n, dtype=np.int64)
    wpm[n // 4] = wpm[3 * n // 4] = kh
    for o2 in range(Co // 2):
        o = 2 * o2
        a = np.concatenate([w[o, 0::2].reshape(G * 9), w[o, 1::2].reshape(G * 9)])
        b = np.concatenate([w[o + 1, 1::2].reshape(G * 9), w[o + 1, 0::2].reshape(G * 9)])
        A, B = cmult_accumulate(rots, np.stack([k * (a + b), a - b]), primes)
        for part in range(2):
            for i, q in enumerate(primes):
                out[o2, part, i] = (A[part, i].astype(np.uint64) + pmult(B[part, i], wpm, q)) % np.uint64(q)
    return out
