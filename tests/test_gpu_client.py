"""GPU parity of the batched client operations (hyena_secret_prepare,
hyena_encrypt_device, hyena_decrypt_device) through the C ABI.

Ciphertexts must equal the oracle's encryption with the same secret and seed
bit for bit (the randomness is drawn from the same counter-based generator);
decrypted messages must equal the encrypted ones, the oracle's exact rounding
on valid ciphertexts, and the host library's decryption on arbitrary residues
(same integer rounding steps, compared everywhere, including fractions near
one half)."""
import math
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_12519_amd as hy

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_CTX = {}


def ctx_for(N, L, bits):
    key = (N, L, bits)
    if key not in _CTX:
        flags = (hy.HYENA_PRIMES_30BIT if bits == 30 else 0) | (hy.HYENA_ALLOW_INSECURE if N < 4096 else 0)
        _CTX[key] = hy.hyena_create(N, L, flags=flags)
    return _CTX[key]


def messages(rng, n, N, log2_t=20):
    t = 1 << log2_t
    m = rng.integers(-t // 2 + 1, t // 2 + 1, size=(n, N)).astype(np.int32)
    m[0, :4] = [t // 2, -t // 2 + 1, 0, -1]         # the ends of (-t/2, t/2]
    return m


def prepared(ctx, sk):
    import torch
    d_sk = torch.from_numpy(sk.astype(np.int8)).cuda()
    d_s_hat = torch.empty(ctx.L * ctx.N, dtype=torch.int32, device="cuda")
    hy.hyena_secret_prepare(ctx, d_sk, d_s_hat)
    return d_s_hat


def encrypt_dev(ctx, d_s_hat, msg, seed):
    import torch
    d_msg = torch.from_numpy(np.ascontiguousarray(msg, dtype=np.int32)).cuda()
    d_ct = torch.full((msg.shape[0] * 2 * ctx.L * ctx.N,), -1, dtype=torch.int32, device="cuda")
    d_work = torch.full((msg.shape[0] * ctx.L * ctx.N,), -1, dtype=torch.int32, device="cuda")
    hy.hyena_encrypt_device(ctx, d_s_hat, d_msg, seed, d_work, d_ct)
    torch.cuda.synchronize()
    return d_ct, d_ct.cpu().numpy().view(np.uint32).reshape(msg.shape[0], 2, ctx.L, ctx.N)


def decrypt_dev(ctx, d_s_hat, d_ct):
    import torch
    n = d_ct.numel() // (2 * ctx.L * ctx.N)
    d_work = torch.empty(n * ctx.L * ctx.N, dtype=torch.int32, device="cuda")
    d_msg = torch.full((n, ctx.N), 7, dtype=torch.int32, device="cuda")
    hy.hyena_decrypt_device(ctx, d_s_hat, d_ct, d_work, d_msg)
    torch.cuda.synchronize()
    return d_msg.cpu().numpy()


@pytest.mark.parametrize("N,L,bits", [(1024, 1, 31), (4096, 2, 30), (8192, 3, 31), (16384, 4, 31)])
def test_secret_prepare_matches_oracle(dev, N, L, bits):
    say(f"secret_prepare N={N} L={L} bits={bits}")
    ctx = ctx_for(N, L, bits)
    sk = orc.keygen(N, 5 + N)
    got = prepared(ctx, sk).cpu().numpy().view(np.uint32).reshape(L, N)
    for i, q in enumerate(ctx.primes):
        s_hat = orc.ntt(np.mod(sk.astype(np.int64), q).astype(np.uint32), q, ctx.psi[i]).astype(object)
        want = np.array([(int(x) << 32) % q for x in s_hat], dtype=np.uint64)
        assert np.array_equal(got[i].astype(np.uint64), want), i


# (N, L, prime bits, messages): one and several chunks per polynomial, one and
# several messages, both prime sizes
ORACLE_CASES = [(1024, 1, 31, 1), (1024, 2, 31, 3), (4096, 2, 30, 2), (8192, 3, 31, 2)]


@pytest.mark.parametrize("N,L,bits,n", ORACLE_CASES)
def test_encrypt_device_matches_oracle(dev, N, L, bits, n):
    say(f"encrypt_device N={N} L={L} bits={bits} n={n}")
    ctx = ctx_for(N, L, bits)
    rng = np.random.default_rng(N * 7 + n)
    sk = orc.keygen(N, 11 + n)
    msg = messages(rng, n, N)
    seed = 0xF00DFACE12345678 + n                    # above 2^63: the whole 64-bit seed is used
    d_s_hat = prepared(ctx, sk)
    d_ct, got = encrypt_dev(ctx, d_s_hat, msg, seed)
    want = orc.encrypt(ctx.primes, 20, sk, msg, seed)
    assert np.array_equal(got, want)
    dec = decrypt_dev(ctx, d_s_hat, d_ct)
    assert np.array_equal(dec.astype(np.int64), orc.decrypt(ctx.primes, 20, sk, want))
    if math.prod(int(q) for q in ctx.primes) > 1 << 41:
        # q > 2 t^2: Delta = floor(q/t) loses less than 1/4 on any message, so
        # decryption is the identity (with one 31-bit prime it is not, for
        # messages near t/2, on any implementation)
        assert np.array_equal(dec, msg)


@pytest.mark.parametrize("N,L,bits,n", [(8192, 3, 31, 50), (16384, 4, 31, 3), (4096, 3, 30, 97)])
def test_encrypt_device_matches_host_at_scale(dev, N, L, bits, n):
    """Many ciphertexts per call: equal to the host encryption (itself pinned to
    the oracle) on every coefficient, and decrypting back to the messages."""
    say(f"encrypt_device at scale N={N} L={L} n={n}")
    ctx = ctx_for(N, L, bits)
    rng = np.random.default_rng(n)
    sk = hy.hyena_keygen(ctx, 99 + n)
    msg = messages(rng, n, N)
    d_s_hat = prepared(ctx, sk)
    d_ct, got = encrypt_dev(ctx, d_s_hat, msg, 4242 + n)
    assert np.array_equal(got, hy.hyena_encrypt(ctx, sk, msg, 4242 + n))
    assert np.array_equal(decrypt_dev(ctx, d_s_hat, d_ct), msg)
    if n <= 3:                                       # the oracle too, where it is quick
        assert np.array_equal(got, orc.encrypt(ctx.primes, 20, sk, msg, 4242 + n))


@pytest.mark.parametrize("N,L,bits,n", [(1024, 2, 31, 4), (8192, 3, 31, 3), (4096, 2, 30, 5), (2048, 1, 31, 3),
                                        (16384, 4, 31, 2), (8192, 5, 30, 2)])
def test_decrypt_device_matches_host_on_arbitrary_residues(dev, N, L, bits, n):
    """Uniform residues put the rounded fraction everywhere in [0, 1); the
    device must take every rounding decision the host takes."""
    import torch
    say(f"decrypt_device arbitrary N={N} L={L} n={n}")
    ctx = ctx_for(N, L, bits)
    rng = np.random.default_rng(3 * N + n)
    ct = np.empty((n, 2, L, N), dtype=np.uint32)
    for i, q in enumerate(ctx.primes):
        ct[:, :, i, :] = rng.integers(0, q, size=(n, 2, N))
        ct[0, 0, i, :3] = [0, q - 1, q // 2]
    sk = hy.hyena_keygen(ctx, 31)
    d_s_hat = prepared(ctx, sk)
    d_ct = torch.from_numpy(ct.view(np.int32)).cuda()
    got = decrypt_dev(ctx, d_s_hat, d_ct.reshape(-1))
    assert np.array_equal(got, hy.hyena_decrypt(ctx, sk, ct))
    # and the oracle's exact rounding round(t v / q): the library takes the
    # fractions of the RNS terms in 0.64 fixed point, each short by less than
    # 2^-33, so it may round down only where frac(t v / q) lies in
    # [1/2, 1/2 + L 2^-33); every coefficient outside that window must equal
    # the oracle's
    q = math.prod(int(p) for p in ctx.primes)
    t = 1 << 20
    want = orc.decrypt(ctx.primes, 20, sk, ct)
    outside = 0
    for m in range(n):
        v = orc.decrypt_phase(ctx.primes, sk, ct[m])
        for j, x in enumerate(v):
            r = (t * x) % q                           # frac(t v / q) = r / q
            in_window = 2 * r >= q and (2 * r - q) * (1 << 32) < L * q
            if in_window:
                assert (int(got[m, j]) - int(want[m, j])) % t in (0, t - 1)
            else:
                assert got[m, j] == want[m, j], (m, j)
                outside += 1
    assert outside >= n * N - 4


def test_decrypt_device_many_ciphertexts(dev):
    """300 ciphertexts of arbitrary residues at n = 4096: the device
    decryption equals the host library's on every coefficient, and so does
    the allocation-free entry point in two calls of 128 and 172."""
    import torch
    N, L, n = 4096, 2, 300
    say(f"decrypt_device N={N} L={L} n={n}")
    ctx = ctx_for(N, L, 31)
    rng = np.random.default_rng(17)
    ct = np.empty((n, 2, L, N), dtype=np.uint32)
    for i, q in enumerate(ctx.primes):
        ct[:, :, i, :] = rng.integers(0, q, size=(n, 2, N))
    sk = hy.hyena_keygen(ctx, 5)
    d_s_hat = prepared(ctx, sk)
    d_ct = torch.from_numpy(ct.view(np.int32)).cuda().reshape(-1)
    got = decrypt_dev(ctx, d_s_hat, d_ct)
    assert np.array_equal(got, hy.hyena_decrypt(ctx, sk, ct))
    for lo, hi in ((0, 128), (128, 300)):   # within the scratch size (n L N <= 2^22)
        d_msg = torch.full((hi - lo, N), 7, dtype=torch.int32, device="cuda")
        hy.hyena_decrypt_device_noalloc(ctx, d_s_hat, d_ct[lo * 2 * L * N:hi * 2 * L * N], d_msg)
        torch.cuda.synchronize()
        assert np.array_equal(d_msg.cpu().numpy(), got[lo:hi])


def test_decrypt_device_of_convolution_output(dev):
    """Decrypting a homomorphic convolution's output (noise far above fresh
    encryption noise) on the device gives the plain convolution."""
    import torch
    import workloads as wl
    say("decrypt_device of a convolution output")
    ctx = ctx_for(4096, 2, 30)
    lay = wl.Layer("t", 12, 12, 8, 8, 3)
    d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k)
    rng = np.random.default_rng(8)
    x = rng.integers(-8, 9, size=(lay.Ci, lay.H, lay.W)).astype(np.int8)
    w = rng.integers(-128, 128, size=(lay.Co, lay.Ci, 3, 3)).astype(np.int8)
    sk = hy.hyena_keygen(ctx, 3)
    d_s_hat = prepared(ctx, sk)
    msg = hy.hyena_pack_input(d, ctx.N, x).reshape(-1, ctx.N)
    d_ct, _ = encrypt_dev(ctx, d_s_hat, msg, 77)
    d_out = torch.empty(d.n_out * 2 * ctx.L * ctx.N, dtype=torch.int32, device="cuda")
    hy.hyena_conv_direct(ctx, d, d_ct, torch.from_numpy(w).cuda(), d_out)
    got = decrypt_dev(ctx, d_s_hat, d_out)
    out_ct = d_out.cpu().numpy().view(np.uint32).reshape(-1, 2, ctx.L, ctx.N)
    assert np.array_equal(got, hy.hyena_decrypt(ctx, sk, out_ct))
    y = hy.hyena_unpack_output(d, ctx.N, got.reshape(d.tiles, lay.Co, ctx.N))
    assert np.array_equal(y, orc.direct_conv(x, w, 3))


def test_client_device_rejects_bad_arguments(dev):
    import torch
    ctx = ctx_for(1024, 2, 31)
    N, L = ctx.N, ctx.L
    d_s_hat = prepared(ctx, orc.keygen(N, 1))
    buf = torch.zeros(4 * 2 * L * N + 4, dtype=torch.int32, device="cuda")
    msg = torch.zeros(2 * N, dtype=torch.int32, device="cuda")
    work = torch.zeros(2 * L * N + 4, dtype=torch.int32, device="cuda")
    with pytest.raises(hy.HyenaError):               # workspace not 16-byte aligned
        hy.hyena_encrypt_device(ctx, d_s_hat, msg, 1, work[1:1 + 2 * L * N], buf[:2 * 2 * L * N])
    with pytest.raises(hy.HyenaError):               # d_ct overlapping d_msg
        hy.hyena_encrypt_device(ctx, d_s_hat, buf[:2 * N], 1, work[:2 * L * N], buf[:2 * 2 * L * N])
    with pytest.raises(hy.HyenaError):               # workspace overlapping d_ct
        hy.hyena_encrypt_device(ctx, d_s_hat, msg, 1, buf[2 * L * N:4 * L * N], buf[:2 * 2 * L * N])
    ct = buf[:2 * 2 * L * N]
    with pytest.raises(hy.HyenaError):               # workspace overlapping the ciphertexts
        hy.hyena_decrypt_device(ctx, d_s_hat, ct, buf[2 * 2 * L * N - 4 * L:], msg)
    with pytest.raises(ValueError):                  # workspace too small (caught by the binding)
        hy.hyena_decrypt_device(ctx, d_s_hat, ct, buf[:L * N], msg)
    # no messages: nothing is launched, nothing written
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    hy.hyena_encrypt_device(ctx, d_s_hat, empty, 1, empty, empty)
    hy.hyena_decrypt_device(ctx, d_s_hat, empty, empty, empty)
