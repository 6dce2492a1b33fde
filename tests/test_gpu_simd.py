"""GPU parity of the SIMD-setting kernels (batch encoding, Galois
automorphisms, PMult by a sparse plaintext) against oracle/simd.py, bit for
bit, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_12519_amd as hy
from oracle import simd

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def from_dev(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


_CTX = {}


def ptx(n, p):
    key = ("p", n, p)
    if key not in _CTX:
        _CTX[key] = hy.hyena_create(n, 1, primes=[p], flags=hy.HYENA_PLAINTEXT_PRIME)
    return _CTX[key]


def ctx_for(N, L, bits):
    key = (N, L, bits)
    if key not in _CTX:
        flags = (hy.HYENA_PRIMES_30BIT if bits == 30 else 0) | hy.HYENA_ALLOW_INSECURE
        _CTX[key] = hy.hyena_create(N, L, flags=flags)
    return _CTX[key]


# (n, p): the paper's Gazelle parameters, the NewHope prime, a Fermat prime at n = 8192
SIMD_CASES = [(2048, 307201), (1024, 12289), (8192, 65537)]


@pytest.mark.parametrize("n,p", SIMD_CASES)
def test_simd_encode_decode_match_oracle(dev, n, p):
    say(f"simd encode/decode n={n} p={p}")
    ctx = ptx(n, p)
    rng = np.random.default_rng(n)
    P = 3
    v = rng.integers(0, p, size=(P, n)).astype(np.uint32)
    v[0, :3] = [0, p - 1, 1]
    d_v = to_dev(v)
    d_m = to_dev(np.zeros((P, n), dtype=np.uint32))
    hy.hyena_simd_encode(ctx, d_v, d_m)
    m = from_dev(d_m).reshape(P, n)
    for r in range(P):
        assert np.array_equal(m[r], simd.encode(v[r], p, n)), r
    d_s = to_dev(np.zeros((P, n), dtype=np.uint32))
    hy.hyena_simd_decode(ctx, d_m, d_s)
    assert np.array_equal(from_dev(d_s).reshape(P, n), v)


def test_simd_pm_plaintext_and_pmult_semantics_on_gpu(dev):
    """All on the GPU over Z_p: encoding [k, -k] gives kh (X^{n/4} + X^{3n/4})
    with the library's (h, k); PMult of encode(v) by that sparse plaintext
    decodes to (k v | -k v) slot-wise; a rotation by X^3 rotates both rows."""
    n, p = 2048, 307201
    say("simd [k,-k] plaintext semantics")
    ctx = ptx(n, p)
    h, k, kh = hy.hyena_simd_params(n, p, 61)
    pattern = np.array([k] * (n // 2) + [p - k] * (n // 2), dtype=np.uint32)
    d_pat, d_w = to_dev(pattern), to_dev(np.zeros(n, dtype=np.uint32))
    hy.hyena_simd_encode(ctx, d_pat, d_w)
    w = from_dev(d_w)
    want = np.zeros(n, dtype=np.uint32)
    want[[n // 4, 3 * n // 4]] = kh
    assert np.array_equal(w, want)
    rng = np.random.default_rng(4)
    v = rng.integers(0, p, n).astype(np.uint32)
    d_v, d_m, d_o = to_dev(v), to_dev(np.zeros(n, np.uint32)), to_dev(np.zeros(n, np.uint32))
    hy.hyena_simd_encode(ctx, d_v, d_m)
    hy.hyena_pmult_sparse(ctx, d_m, [n // 4, 3 * n // 4], [kh, kh], d_o)
    d_s = to_dev(np.zeros(n, np.uint32))
    hy.hyena_simd_decode(ctx, d_o, d_s)
    got = from_dev(d_s).astype(np.int64)
    half = n // 2
    assert np.array_equal(got[:half], v[:half].astype(np.int64) * k % p)
    assert np.array_equal(got[half:], (-v[half:].astype(np.int64) * k) % p)
    hy.hyena_simd_encode(ctx, d_v, d_m)
    hy.hyena_automorphism(ctx, d_m, 3, d_o)
    hy.hyena_simd_decode(ctx, d_o, d_s)
    got = from_dev(d_s)
    assert np.array_equal(got[:half], np.roll(v[:half], -1)) and np.array_equal(got[half:], np.roll(v[half:], -1))


@pytest.mark.parametrize("N,L,bits", [(2048, 2, 30), (8192, 3, 31), (1024, 1, 31)])
def test_automorphism_matches_oracle(dev, N, L, bits):
    say(f"automorphism N={N} L={L}")
    ctx = ctx_for(N, L, bits)
    rng = np.random.default_rng(N + L)
    P = 2
    a = np.empty((P, L, N), dtype=np.uint32)
    for i, q in enumerate(ctx.primes):
        a[:, i, :] = rng.integers(0, q, size=(P, N))
        a[0, i, :3] = [0, q - 1, 1]
    d_a, d_o = to_dev(a), to_dev(np.zeros_like(a))
    for g in (3, 5, 2 * N - 1, pow(3, 123, 2 * N), 2 * N + 3):
        hy.hyena_automorphism(ctx, d_a, g, d_o)
        got = from_dev(d_o).reshape(P, L, N)
        for r in range(P):
            for i, q in enumerate(ctx.primes):
                assert np.array_equal(got[r, i], simd.automorphism(a[r, i], g % (2 * N), q)), (g, r, i)
    # arrays that are not 16-byte aligned take the coefficient-gather kernel
    import torch
    d_a4 = torch.zeros(a.size + 1, dtype=torch.int32, device="cuda")
    d_a4[1:] = d_a.reshape(-1)
    d_o4 = torch.zeros(a.size + 1, dtype=torch.int32, device="cuda")
    hy.hyena_automorphism(ctx, d_a4[1:], 5, d_o4[1:])
    got = from_dev(d_o4[1:]).reshape(P, L, N)
    for i, q in enumerate(ctx.primes):
        assert np.array_equal(got[1, i], simd.automorphism(a[1, i], 5, q))


@pytest.mark.parametrize("N,L,bits", [(2048, 2, 30), (8192, 3, 31)])
def test_pmult_sparse_matches_oracle(dev, N, L, bits):
    """The [k, -k] plaintext of the paper's parameters (two monomials), and a
    plaintext of 16 monomials with exponents up to 2N - 1 (signs)."""
    say(f"pmult_sparse N={N} L={L}")
    ctx = ctx_for(N, L, bits)
    rng = np.random.default_rng(N * L)
    P = 2
    a = np.empty((P, L, N), dtype=np.uint32)
    for i, q in enumerate(ctx.primes):
        a[:, i, :] = rng.integers(0, q, size=(P, N))
    d_a, d_o = to_dev(a), to_dev(np.zeros_like(a))
    _, _, kh = hy.hyena_simd_params(2048, 307201, 61)
    cases = [([N // 4, 3 * N // 4], [kh, kh]),
             (sorted(rng.choice(2 * N, 16, replace=False).tolist()), rng.integers(0, 307201, 16).tolist())]
    import torch
    d_a4 = torch.zeros(a.size + 1, dtype=torch.int32, device="cuda")
    d_a4[1:] = d_a.reshape(-1)
    d_o4 = torch.zeros(a.size + 1, dtype=torch.int32, device="cuda")
    for exps, coefs in cases:
        hy.hyena_pmult_sparse(ctx, d_a, exps, coefs, d_o)
        got = from_dev(d_o).reshape(P, L, N)
        # arrays that are not 16-byte aligned take the coefficient-gather kernel
        hy.hyena_pmult_sparse(ctx, d_a4[1:], exps, coefs, d_o4[1:])
        assert np.array_equal(from_dev(d_o4[1:]).reshape(P, L, N), got)
        for i, q in enumerate(ctx.primes):
            w = np.zeros(N, dtype=np.int64)
            for e, c in zip(exps, coefs):                 # X^e = -X^{e-N} for e >= N
                if e < N:
                    w[e] = (w[e] + c) % q
                else:
                    w[e - N] = (w[e - N] - c) % q
            for r in range(P):
                assert np.array_equal(got[r, i], simd.pmult(a[r, i], w, q)), (len(exps), r, i)


def test_simd_calls_reject_bad_arguments(dev):
    import torch
    ctx = ptx(2048, 307201)
    cctx = ctx_for(2048, 2, 30)
    buf = torch.zeros(4 * 2048 * 2, dtype=torch.int32, device="cuda")
    with pytest.raises(hy.HyenaError):                    # encode needs a single-prime context
        hy.hyena_simd_encode(cctx, buf[:2 * 2048], buf[4 * 2048:6 * 2048])
    with pytest.raises(hy.HyenaError):                    # overlapping arrays
        hy.hyena_simd_encode(ctx, buf[:2048], buf[1024:3072])
    with pytest.raises(hy.HyenaError):                    # even g
        hy.hyena_automorphism(cctx, buf[:2 * 2048], 4, buf[4 * 2048:6 * 2048])
    with pytest.raises(hy.HyenaError):                    # exponent not below 2N
        hy.hyena_pmult_sparse(cctx, buf[:2 * 2048], [4096], [1], buf[4 * 2048:6 * 2048])
    with pytest.raises(hy.HyenaError):                    # more than 16 monomials
        hy.hyena_pmult_sparse(cctx, buf[:2 * 2048], list(range(17)), [1] * 17, buf[4 * 2048:6 * 2048])


def _hrot_setup(N, L, b, gs, n_ct, seed, bits=30):
    import torch
    ctx = ctx_for(N, L, bits)
    primes = ctx.primes
    s = orc.keygen(N, seed)
    rng = np.random.default_rng(seed)
    t = 1 << 20
    msg = rng.integers(-t // 2 + 1, t // 2 + 1, size=(n_ct, N))
    ct = orc.encrypt(primes, 20, s, msg, seed + 1)
    keys = np.stack([hy.hyena_galois_keygen(ctx, s, g, b, 500 + g) for g in gs])
    d_k = to_dev(keys)
    hy.hyena_ksk_prepare(ctx, d_k)
    D = hy.n_digits(b)
    d_ct = to_dev(ct)
    d_work = torch.empty(n_ct * (L * D + 1) * L * N, dtype=torch.int32, device="cuda")
    d_out = torch.empty(n_ct * len(gs) * 2 * L * N, dtype=torch.int32, device="cuda")
    hy.hyena_hrot_hoisted(ctx, d_ct, gs, b, d_k, d_work, d_out)
    return ctx, s, msg, ct, keys, from_dev(d_out).reshape(n_ct, len(gs), 2, L, N)


@pytest.mark.parametrize("b", [8, 16, 29])
def test_hrot_hoisted_matches_oracle(dev, b):
    """Every rotated ciphertext equals the oracle's hoisted HRot bit for bit and
    decrypts to the automorphism of its message."""
    N, L = 1024, 2
    gs = [3, 2 * N - 1, 9, 1]
    say(f"hrot hoisted N={N} L={L} b={b}")
    ctx, s, msg, ct, keys, got = _hrot_setup(N, L, b, gs, 2, 40 + b)
    t = 1 << 20
    for m in range(2):
        for r, g in enumerate(gs):
            assert np.array_equal(got[m, r], simd.hrot(ctx.primes, ct[m], g, keys[r], b)), (m, g)
            want = simd.automorphism(msg[m] % t, g, t).astype(np.int64)
            want = np.where(want > t // 2, want - t, want)
            assert np.array_equal(orc.decrypt(ctx.primes, 20, s, got[m, r][None])[0], want), (m, g)


def test_hrot_hoisted_papers_parameters_nine_rotations(dev):
    """n = 2048 with a 60-bit q (two 30-bit primes), the 3x3 kernel's nine
    rotations (powers of 3, with the row swap), 4 ciphertexts: sampled
    (ciphertext, rotation) pairs against the oracle, every one by decryption."""
    N, L, b = 2048, 2, 16
    gs = [pow(3, r, 2 * N) for r in range(8)] + [2 * N - 1]
    say("hrot hoisted n=2048, 9 rotations")
    ctx, s, msg, ct, keys, got = _hrot_setup(N, L, b, gs, 4, 7)
    for m, r in [(0, 0), (3, 8), (2, 5)]:
        assert np.array_equal(got[m, r], simd.hrot(ctx.primes, ct[m], gs[r], keys[r], b)), (m, r)
    t = 1 << 20
    dec = hy.hyena_decrypt(ctx, s, got.reshape(-1, 2, L, N)).reshape(4, len(gs), N)
    for m in range(4):
        for r, g in enumerate(gs):
            want = simd.automorphism(msg[m] % t, g, t).astype(np.int64)
            assert np.array_equal(dec[m, r], np.where(want > t // 2, want - t, want)), (m, r)


def test_hrot_hoisted_ragged_ciphertext_groups(dev):
    """11 ciphertexts (groups of eight and a ragged three) under three
    rotations at b = 11: every output equals the oracle's hoisted HRot bit
    for bit."""
    N, L, b = 1024, 2, 11
    gs = [5, 2 * N - 3, 3]
    say(f"hrot hoisted N={N} L={L} b={b}, 11 ciphertexts")
    ctx, s, msg, ct, keys, got = _hrot_setup(N, L, b, gs, 11, 23)
    for m in range(11):
        for r, g in enumerate(gs):
            assert np.array_equal(got[m, r], simd.hrot(ctx.primes, ct[m], g, keys[r], b)), (m, g)


@pytest.mark.parametrize("L,b", [(2, 16), (3, 8), (3, 11)])
def test_hrot_hoisted_31_bit_primes(dev, L, b):
    """Primes below 2^31, where the key switch's 64-bit sums are folded after
    every few products (L D = 4, 12 and 9 digit terms): every output equals
    the oracle's hoisted HRot bit for bit."""
    N = 1024
    gs = [3, 2 * N - 1, 25]
    say(f"hrot hoisted N={N} L={L} b={b}, primes < 2^31")
    ctx, s, msg, ct, keys, got = _hrot_setup(N, L, b, gs, 3, 60 + b, bits=31)
    for m in range(3):
        for r, g in enumerate(gs):
            assert np.array_equal(got[m, r], simd.hrot(ctx.primes, ct[m], g, keys[r], b)), (m, g)


@pytest.mark.parametrize("N,L,b", [(4096, 2, 16), (8192, 3, 11), (16384, 2, 16)])
def test_hrot_hoisted_larger_rings(dev, N, L, b):
    """n = 4096, 8192 and 16384 (primes below 2^31): every output equals the
    oracle's hoisted HRot bit for bit."""
    gs = [3, 2 * N - 1]
    say(f"hrot hoisted N={N} L={L} b={b}")
    ctx, s, msg, ct, keys, got = _hrot_setup(N, L, b, gs, 2, 80 + b, bits=31)
    for m in range(2):
        for r, g in enumerate(gs):
            assert np.array_equal(got[m, r], simd.hrot(ctx.primes, ct[m], g, keys[r], b)), (m, g)


def test_hrot_hoisted_many_ciphertexts_rotation_loop(dev):
    """2045 random ciphertexts (a ragged last group of five) under three
    rotations, enough that the key switch loops over the rotations inside the
    thread, with primes below 2^31 (sums folded after every few products):
    sampled outputs equal the oracle's hoisted HRot bit for bit (keys from the
    oracle's key generation)."""
    import torch
    N, L, b = 1024, 2, 11
    gs = [3, 5, 2 * N - 1]
    n_ct = 2045
    say(f"hrot hoisted N={N} L={L} b={b}, {n_ct} ciphertexts")
    ctx = ctx_for(N, L, 31)
    primes = ctx.primes
    s = orc.keygen(N, 31)
    rng = np.random.default_rng(31)
    ct = np.empty((n_ct, 2, L, N), dtype=np.uint32)
    for k, q in enumerate(primes):
        ct[:, :, k, :] = rng.integers(0, q, size=(n_ct, 2, N), dtype=np.uint64).astype(np.uint32)
    keys = np.stack([simd.galois_keygen(primes, s, g, b, 700 + g) for g in gs])
    d_k = to_dev(keys)
    hy.hyena_ksk_prepare(ctx, d_k)
    D = hy.n_digits(b)
    d_work = torch.empty(n_ct * (L * D + 1) * L * N, dtype=torch.int32, device="cuda")
    d_out = torch.empty(n_ct * len(gs) * 2 * L * N, dtype=torch.int32, device="cuda")
    hy.hyena_hrot_hoisted(ctx, to_dev(ct), gs, b, d_k, d_work, d_out)
    got = from_dev(d_out).reshape(n_ct, len(gs), 2, L, N)
    for m in (0, 7, 8, 1001, 2039, 2040, 2044):
        for r, g in enumerate(gs):
            assert np.array_equal(got[m, r], simd.hrot(primes, ct[m], g, keys[r], b)), (m, g)


def test_hrot_rejects_bad_arguments(dev):
    import torch
    ctx = ctx_for(1024, 2, 30)
    L, N = 2, 1024
    ct = torch.zeros(2 * L * N, dtype=torch.int32, device="cuda")
    k = torch.zeros(2 * 2 * L * N * 2, dtype=torch.int32, device="cuda")
    work = torch.zeros((2 * 2 + 1) * L * N, dtype=torch.int32, device="cuda")
    out = torch.zeros(2 * L * N, dtype=torch.int32, device="cuda")
    with pytest.raises(hy.HyenaError):                     # even g
        hy.hyena_hrot_hoisted(ctx, ct, [4], 16, k, work, out)
    with pytest.raises(hy.HyenaError):                     # base out of range
        hy.hyena_hrot_hoisted(ctx, ct, [3], 30, k, work, out)
    with pytest.raises(hy.HyenaError):                     # output overlapping the workspace
        hy.hyena_hrot_hoisted(ctx, ct, [3], 16, k, work, work[:2 * L * N])


def test_simd_calls_on_empty_inputs(dev):
    """Degenerate sizes: no ciphertexts to rotate, no polynomials to permute
    or multiply, no output channels (nothing written, no error); no inputs to
    accumulate (every output is the zero ciphertext)."""
    import torch
    N, L = 1024, 2
    ctx = ctx_for(N, L, 30)
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    k = torch.zeros(2 * L * hy.n_digits(16) * 2 * L * N, dtype=torch.int32, device="cuda")   # two rotations' keys
    hy.hyena_hrot_hoisted(ctx, empty, [3, 5], 16, k, empty, empty)
    hy.hyena_automorphism(ctx, empty, 3, empty)
    hy.hyena_pmult_sparse(ctx, empty, [1], [1], empty)
    hy.hyena_cmult_accumulate(ctx, empty, torch.zeros((0, 0), dtype=torch.int32, device="cuda"), empty)
    sentinel = torch.full((3 * 2 * L * N,), 12345, dtype=torch.int32, device="cuda")
    hy.hyena_cmult_accumulate(ctx, empty, torch.zeros((3, 0), dtype=torch.int32, device="cuda"), sentinel)
    assert not from_dev(sentinel).any()
    torch.cuda.synchronize()


def test_simd_conv_cn2_on_gpu_matches_oracle(dev):
    """The paper's SIMD convolution with c_n = 2 at its parameters (n = 2048,
    p = 307201, k = 11), composed from the library's calls (hoisted HRot,
    CMult-accumulate, PMult by the [k, -k] plaintext, row-swap HRot, HAdd): the
    output ciphertexts equal the oracle's composition bit for bit and decrypt
    to 2k conv(x) at every image position."""
    import torch
    n, L, p, b = 2048, 3, 307201, 8
    fh, fw, Co = 32, 32, 4
    say("simd conv c_n=2 n=2048")
    ctx = ctx_for(n, L, 30)
    primes = ctx.primes
    s = orc.keygen(n, 8)
    h, k, kh = hy.hyena_simd_params(n, p, 61)
    rng = np.random.default_rng(21)
    H, W = fh - 2, fw - 2
    x = rng.integers(-8, 8, size=(2, H, W))
    w = rng.integers(-8, 8, size=(Co, 2, 3, 3))
    ct = simd.encrypt_p(primes, p, s, simd.encode(simd.frame_slots(x, fh, fw), p, n)[None], 5)[0]
    gs = simd.conv_rotations(n, fw)
    keys = np.stack([hy.hyena_galois_keygen(ctx, s, g, b, 300 + i) for i, g in enumerate(gs)])
    skey = hy.hyena_galois_keygen(ctx, s, 2 * n - 1, b, 399)
    want = simd.simd_conv_cn2(primes, ct, w, k, kh, fw, {g: keys[i] for i, g in enumerate(gs)}, skey, b)
    LN, D = L * n, hy.n_digits(b)
    dk, dsk = to_dev(keys), to_dev(skey)
    hy.hyena_ksk_prepare(ctx, dk)
    hy.hyena_ksk_prepare(ctx, dsk)
    i32 = dict(dtype=torch.int32, device="cuda")
    rots = torch.empty(9 * 2 * LN, **i32)
    work = torch.empty(max(1, Co) * (L * D + 1) * LN, **i32)
    hy.hyena_hrot_hoisted(ctx, to_dev(ct), gs, b, dk, work, rots)
    f0, f1 = w[:, 0].reshape(Co, 9), w[:, 1].reshape(Co, 9)
    Wab = torch.from_numpy(np.concatenate([k * (f0 + f1), f0 - f1]).astype(np.int32)).cuda()   # A block, B block
    AB = torch.empty(2 * Co * 2 * LN, **i32)
    hy.hyena_cmult_accumulate(ctx, rots, Wab, AB)
    PB = torch.empty(Co * 2 * LN, **i32)
    hy.hyena_pmult_sparse(ctx, AB[Co * 2 * LN:], [n // 4, 3 * n // 4], [kh, kh], PB)
    pair = torch.from_numpy(np.concatenate([np.eye(Co), np.eye(Co)], axis=1).astype(np.int32)).cuda()
    ZP = torch.cat([AB[:Co * 2 * LN], PB])
    Z = torch.empty(Co * 2 * LN, **i32)
    hy.hyena_cmult_accumulate(ctx, ZP, pair, Z)
    Zs = torch.empty(Co * 2 * LN, **i32)
    hy.hyena_hrot_hoisted(ctx, Z, [2 * n - 1], b, dsk, work, Zs)
    out = torch.empty(Co * 2 * LN, **i32)
    hy.hyena_cmult_accumulate(ctx, torch.cat([Z, Zs]), pair, out)
    got = from_dev(out).reshape(Co, 2, L, n)
    assert np.array_equal(got, want)
    y = orc.direct_conv(x, w, 3)
    for o in range(Co):
        slots = simd.decode(simd.decrypt_p(primes, p, s, got[o][None])[0], p, n).astype(np.int64)
        for row in range(2):
            frame = slots[row * (n // 2):(row + 1) * (n // 2)].reshape(fh, fw)
            assert np.array_equal(frame[1:1 + H, 1:1 + W], (2 * k * y[o]) % p), (o, row)


@pytest.mark.parametrize("Co", [3, 23, 45])
def test_simd_conv_cn2_entry_point(dev, Co):
    """hyena_simd_conv_cn2 over two input ciphertexts (4 channels -> Co outputs)
    at the paper's parameters: equal to the oracle's convolution bit for bit,
    decrypting to 2k conv(x); a too-small workspace is refused. The output
    counts take the CMult-accumulate's one, two and four outputs per thread,
    the last two with a ragged final group (23 = 11 x 2 + 1, 45 = 11 x 4 + 1)."""
    import torch
    n, L, p, b = 2048, 3, 307201, 8
    fh, fw, G = 32, 32, 2
    say(f"hyena_simd_conv_cn2 n=2048, 2 inputs, {Co} outputs")
    ctx = ctx_for(n, L, 30)
    primes = ctx.primes
    s = orc.keygen(n, 19)
    h, k, kh = hy.hyena_simd_params(n, p, 61)
    rng = np.random.default_rng(33)
    H, W = fh - 2, fw - 2
    x = rng.integers(-8, 8, size=(2 * G, H, W))
    w = rng.integers(-8, 8, size=(Co, 2 * G, 3, 3))
    msgs = np.stack([simd.encode(simd.frame_slots(x[2 * g:2 * g + 2], fh, fw), p, n) for g in range(G)])
    ct = simd.encrypt_p(primes, p, s, msgs, 6)
    gs = simd.conv_rotations(n, fw)
    keys = np.stack([hy.hyena_galois_keygen(ctx, s, g, b, 600 + i) for i, g in enumerate(gs)])
    skey = hy.hyena_galois_keygen(ctx, s, 2 * n - 1, b, 699)
    want = simd.simd_conv_cn2(primes, ct, w, k, kh, fw, {g: keys[i] for i, g in enumerate(gs)}, skey, b)
    dk, dsk = to_dev(keys), to_dev(skey)
    hy.hyena_ksk_prepare(ctx, dk)
    hy.hyena_ksk_prepare(ctx, dsk)
    wa, wb = hy.hyena_simd_conv_weights(w.astype(np.int8), k)
    d_wa, d_wb = torch.from_numpy(wa).cuda(), torch.from_numpy(wb).cuda()
    words = hy.hyena_simd_conv_workspace(ctx, G, Co, b)
    work = torch.empty(words, dtype=torch.int32, device="cuda")
    out = torch.empty(Co * 2 * L * n, dtype=torch.int32, device="cuda")
    d_ct = to_dev(ct)
    hy.hyena_simd_conv_cn2(ctx, d_ct, fw, d_wa, d_wb, kh, b, dk, dsk, work, out)
    got = from_dev(out).reshape(Co, 2, L, n)
    assert np.array_equal(got, want)
    y = orc.direct_conv(x, w, 3)
    for o in sorted({0, 1, Co - 1}):
        slots = simd.decode(simd.decrypt_p(primes, p, s, got[o][None])[0], p, n).astype(np.int64)
        for row in range(2):
            frame = slots[row * (n // 2):(row + 1) * (n // 2)].reshape(fh, fw)
            assert np.array_equal(frame[1:1 + H, 1:1 + W], (2 * k * y[o]) % p), (o, row)
    with pytest.raises(hy.HyenaError):
        hy.hyena_simd_conv_cn2(ctx, d_ct, fw, d_wa, d_wb, kh, b, dk, dsk, work[:words - 4], out)


def test_simd_conv_cn1_from_library_calls(dev):
    """c_n = 1 at the paper's parameters: hoisted HRot of 4 single-channel
    ciphertexts by the nine offsets, then one CMult-accumulate (the paper's
    CMult and HAdd with lazy reduction) per output channel; decrypts to
    conv(x) in the first row."""
    import torch
    n, L, p, b = 2048, 3, 307201, 8
    fh, fw, Ci, Co = 32, 32, 4, 3
    say("simd conv c_n=1 n=2048")
    ctx = ctx_for(n, L, 30)
    primes = ctx.primes
    s = orc.keygen(n, 23)
    rng = np.random.default_rng(44)
    H, W = fh - 2, fw - 2
    x = rng.integers(-8, 8, size=(Ci, H, W))
    w = rng.integers(-8, 8, size=(Co, Ci, 3, 3))
    rows = [simd.frame_slots(np.stack([x[c], np.zeros_like(x[c])]), fh, fw) for c in range(Ci)]
    ct = simd.encrypt_p(primes, p, s, np.stack([simd.encode(r, p, n) for r in rows]), 4)
    gs = simd.conv_rotations(n, fw)
    keys = to_dev(np.stack([hy.hyena_galois_keygen(ctx, s, g, b, 80 + i) for i, g in enumerate(gs)]))
    hy.hyena_ksk_prepare(ctx, keys)
    LN, D = L * n, hy.n_digits(b)
    rots = torch.empty(Ci * 9 * 2 * LN, dtype=torch.int32, device="cuda")
    work = torch.empty(Ci * (L * D + 1) * LN, dtype=torch.int32, device="cuda")
    hy.hyena_hrot_hoisted(ctx, to_dev(ct), gs, b, keys, work, rots)
    out = torch.empty(Co * 2 * LN, dtype=torch.int32, device="cuda")
    hy.hyena_cmult_accumulate(ctx, rots, torch.from_numpy(w.reshape(Co, Ci * 9).astype(np.int32)).cuda(), out)
    got = from_dev(out).reshape(Co, 2, L, n)
    y = orc.direct_conv(x, w, 3)
    for o in range(Co):
        slots = simd.decode(simd.decrypt_p(primes, p, s, got[o][None])[0], p, n).astype(np.int64)
        frame = slots[:n // 2].reshape(fh, fw)
        assert np.array_equal(frame[1:1 + H, 1:1 + W], y[o] % p), o


def test_simd_conv_packed_entry_point(dev):
    """hyena_simd_conv_packed (output channel packing) over two input
    ciphertexts, 4 -> 4 channels: two output ciphertexts equal to the oracle's
    bit for bit, each decrypting to two output channels."""
    import torch
    n, L, p, b = 2048, 3, 307201, 8
    fh, fw, G, Co = 32, 32, 2, 4
    say("hyena_simd_conv_packed n=2048, 2 inputs, 4 outputs")
    ctx = ctx_for(n, L, 30)
    primes = ctx.primes
    s = orc.keygen(n, 29)
    h, k, kh = hy.hyena_simd_params(n, p, 61)
    rng = np.random.default_rng(55)
    H, W = fh - 2, fw - 2
    x = rng.integers(-8, 8, size=(2 * G, H, W))
    w = rng.integers(-8, 8, size=(Co, 2 * G, 3, 3))
    msgs = np.stack([simd.encode(simd.frame_slots(x[2 * g:2 * g + 2], fh, fw), p, n) for g in range(G)])
    ct = simd.encrypt_p(primes, p, s, msgs, 8)
    gs = simd.conv_rotations(n, fw)
    keys = np.stack([hy.hyena_galois_keygen(ctx, s, g, b, 700 + i) for i, g in enumerate(gs)])
    skey = hy.hyena_galois_keygen(ctx, s, 2 * n - 1, b, 799)
    want = simd.simd_conv_cn2_packed(primes, ct, w, k, kh, fw, {g: keys[i] for i, g in enumerate(gs)}, skey, b)
    dk, dsk = to_dev(keys), to_dev(skey)
    hy.hyena_ksk_prepare(ctx, dk)
    hy.hyena_ksk_prepare(ctx, dsk)
    wa, wb = hy.hyena_simd_conv_weights_packed(w.astype(np.int8), k)
    work = torch.empty(hy.hyena_simd_conv_packed_workspace(ctx, G, Co, b), dtype=torch.int32, device="cuda")
    out = torch.empty(Co // 2 * 2 * L * n, dtype=torch.int32, device="cuda")
    hy.hyena_simd_conv_packed(ctx, to_dev(ct), fw, torch.from_numpy(wa).cuda(), torch.from_numpy(wb).cuda(), kh, b,
                              dk, dsk, work, out)
    got = from_dev(out).reshape(Co // 2, 2, L, n)
    assert np.array_equal(got, want)
    y = orc.direct_conv(x, w, 3)
    for o2 in range(Co // 2):
        slots = simd.decode(simd.decrypt_p(primes, p, s, got[o2][None])[0], p, n).astype(np.int64)
        for row in range(2):
            frame = slots[row * (n // 2):(row + 1) * (n // 2)].reshape(fh, fw)
            assert np.array_equal(frame[1:1 + H, 1:1 + W], (2 * k * y[2 * o2 + row]) % p), (o2, row)


def test_simd_conv_packed_full_layer_at_the_noise_chosen_base(dev):
    """The benchmark's layer at full size (30x30, 64 -> 64 channels, n = 2048,
    three primes below 2^30) with output channel packing, at the base
    hyena_simd_conv_choose_base returns: sampled output ciphertexts decrypt to
    2k conv(x) for both of their output channels at every image position (a
    property that holds at any size; bit equality with the oracle's
    composition is checked on the smaller cases above)."""
    import torch
    n, L, p = 2048, 3, 307201
    fh, fw, Ci, Co = 32, 32, 64, 64
    say("hyena_simd_conv_packed, 64 -> 64 at the chosen base")
    ctx = ctx_for(n, L, 30)
    primes = ctx.primes
    s = orc.keygen(n, 61)
    h, k, kh = hy.hyena_simd_params(n, p, 61)
    rng = np.random.default_rng(62)
    H, W = fh - 2, fw - 2
    x = rng.integers(-8, 8, size=(Ci, H, W))
    w = rng.integers(-8, 8, size=(Co, Ci, 3, 3))
    wa, wb = hy.hyena_simd_conv_weights_packed(w.astype(np.int8), k)
    b, margin = hy.hyena_simd_conv_choose_base(ctx, p, kh, wa, wb, packed=True)
    say(f"  chosen base 2^{b} (margin {margin:.2f} bits)")
    G = Ci // 2
    msgs = np.stack([simd.encode(simd.frame_slots(x[2 * g:2 * g + 2], fh, fw), p, n) for g in range(G)])
    ct = simd.encrypt_p(primes, p, s, msgs, 63)
    gs = simd.conv_rotations(n, fw)
    keys = to_dev(np.stack([hy.hyena_galois_keygen(ctx, s, g, b, 640 + i) for i, g in enumerate(gs)]))
    skey = to_dev(hy.hyena_galois_keygen(ctx, s, 2 * n - 1, b, 649))
    hy.hyena_ksk_prepare(ctx, keys)
    hy.hyena_ksk_prepare(ctx, skey)
    work = torch.empty(hy.hyena_simd_conv_packed_workspace(ctx, G, Co, b), dtype=torch.int32, device="cuda")
    out = torch.empty(Co // 2 * 2 * L * n, dtype=torch.int32, device="cuda")
    hy.hyena_simd_conv_packed(ctx, to_dev(ct), fw, torch.from_numpy(wa).cuda(), torch.from_numpy(wb).cuda(), kh, b,
                              keys, skey, work, out)
    got = from_dev(out).reshape(Co // 2, 2, L, n)
    y = orc.direct_conv(x, w, 3)
    for o2 in (0, 7, 19, 31):
        slots = simd.decode(simd.decrypt_p(primes, p, s, got[o2][None])[0], p, n).astype(np.int64)
        for row in range(2):
            frame = slots[row * (n // 2):(row + 1) * (n // 2)].reshape(fh, fw)
            assert np.array_equal(frame[1:1 + H, 1:1 + W], (2 * k * y[2 * o2 + row]) % p), (o2, row)
