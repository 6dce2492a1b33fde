"""Pins of the oracle against facts other than the oracle itself.

Each test ties an oracle function to something the paper or mathematics fixes:
a value the paper prints, a published test vector, an independent algorithm
(brute force, big-integer arithmetic, a library routine), a closed form or an
invariant. A plausible slip in the oracle (dropped term, wrong sign or index,
transposed operand) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import sympy
import torch

import oracle as orc
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = [l.split() for l in open(os.path.join(GOLDEN, name)) if l.strip() and not l.startswith("#")]
    return np.array([[int(v) for v in r] for r in rows], dtype=np.int64)


# ---------------------------------------------------------------- random numbers

def test_splitmix64_published_vectors():
    # SplitMix64 (Steele, Lea & Flood 2014) seeded with 0 and with 1234567:
    # the first outputs quoted with the reference C implementation.
    assert [int(v) for v in orc.sm64(0, [0, 1, 2])] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [int(v) for v in orc.sm64(1234567, [0, 1, 2, 3, 4])] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_uniform_mod_exact_against_bigint():
    r = orc.sm64(99, np.arange(2000, dtype=np.uint64))
    for q in (2147352577, 1073692673):
        got = orc._uniform_mod(r, q)
        want = [(int(x) * q) >> 64 for x in r]
        assert [int(v) for v in got] == want


def test_error_sampler_distribution():
    # rounded Gaussian, sigma = 3.2, bounded by B = 10 sigma (the "Homomorphic Operations in BFV" section)
    e = orc.sample_error(5, np.arange(400_000, dtype=np.uint64))
    assert e.min() >= -orc.B_ERR and e.max() <= orc.B_ERR
    assert abs(e.mean()) < 0.03
    assert abs(e.var() - orc.SIGMA ** 2) < 0.15
    # P(|e| > 4 sigma) is about 6e-5 for the discrete Gaussian
    assert np.mean(np.abs(e) > 13) < 3e-4


def test_keygen_is_ternary_and_balanced():
    s = orc.keygen(8192, 3)
    assert set(np.unique(s)) <= {-1, 0, 1}
    counts = np.bincount(s.astype(np.int64) + 1, minlength=3)
    assert np.all(np.abs(counts - 8192 / 3) < 200)


# ---------------------------------------------------------------- parameters

@pytest.mark.parametrize("N,L,bits", [(4096, 2, 30), (8192, 3, 31), (16384, 4, 31)])
def test_ntt_primes_are_the_largest(N, L, bits):
    ps = orc.ntt_primes(N, L, bits)
    assert len(ps) == L and ps == sorted(ps, reverse=True)
    for q in ps:
        assert sympy.isprime(q) and q % (2 * N) == 1 and q < 2 ** bits
    # no candidate above the smallest chosen prime was skipped
    cand = range(ps[-1], 2 ** bits, 2 * N)
    assert [q for q in cand if sympy.isprime(q)][::-1] == ps


@pytest.mark.parametrize("N,q", [(4096, 1073692673), (8192, 2147352577), (16384, 2146041857)])
def test_psi_is_smallest_primitive_2n_root(N, q):
    psi = orc.find_psi(q, N)
    assert pow(psi, N, q) == q - 1 and pow(psi, 2 * N, q) == 1
    # by exhaustion: nothing in [2, psi) has x^N = -1
    assert all(pow(x, N, q) != q - 1 for x in range(2, psi, max(1, (psi - 2) // 4000) if psi > 10**6 else 1))


def test_security_table_is_the_published_one():
    # the HE Security Standard's 128-bit ceilings for a uniform ternary secret
    # (tests/golden/he_standard_ternary_128.txt, with its citation)
    table = {int(n): int(b) for n, b in _golden("he_standard_ternary_128.txt")}
    assert orc.SECURITY_LOGQ_128 == table


# ---------------------------------------------------------------- ring arithmetic

def _brute_negacyclic(a, b, q):
    """Full polynomial product, then fold X^N = -1 (independent of the oracle)."""
    N = len(a)
    full = [0] * (2 * N)
    for i in range(N):
        for j in range(N):
            full[i + j] += int(a[i]) * int(b[j])
    return [(full[k] - full[k + N]) % q for k in range(N)]


def test_negacyclic_mul_brute_force_small():
    rng = np.random.default_rng(0)
    for N, q in [(8, 17), (32, 193), (64, 2147352577)]:
        a = rng.integers(0, q, N).astype(np.uint32)
        b = rng.integers(0, q, N).astype(np.uint32)
        assert list(orc.negacyclic_mul(a, b, q)) == _brute_negacyclic(a, b, q)


def test_negacyclic_mul_kronecker_bigint():
    # Kronecker substitution with Python big integers at N = 1024
    N, q = 1024, 2147352577
    rng = np.random.default_rng(1)
    a = rng.integers(0, q, N)
    b = rng.integers(0, q, N)
    bits = 80
    A = sum(int(v) << (bits * i) for i, v in enumerate(a))
    B = sum(int(v) << (bits * i) for i, v in enumerate(b))
    P = A * B
    mask = (1 << bits) - 1
    coeffs = [(P >> (bits * k)) & mask for k in range(2 * N)]
    want = [(coeffs[k] - coeffs[k + N]) % q for k in range(N)]
    got = orc.negacyclic_mul(a.astype(np.uint32), b.astype(np.uint32), q)
    assert list(got) == want


def test_monomial_product_is_signed_rotation():
    N, q = 256, 2147352577
    rng = np.random.default_rng(2)
    a = rng.integers(0, q, N).astype(np.uint32)
    for s in (0, 1, 77, 255):
        mono = np.zeros(N, dtype=np.uint32)
        mono[s] = 1
        want = np.concatenate([(q - a[N - s:].astype(np.int64)) % q, a[:N - s]]).astype(np.uint32)
        assert np.array_equal(orc.negacyclic_mul(a, mono, q), want)


# ---------------------------------------------------------------- NTT

def test_ntt_convolution_theorem_and_roundtrip():
    N, q = 64, 7681  # 7681 = 1 mod 128
    psi = orc.find_psi(q, N)
    rng = np.random.default_rng(3)
    a = rng.integers(0, q, N).astype(np.uint32)
    b = rng.integers(0, q, N).astype(np.uint32)
    A, B = orc.ntt(a, q, psi), orc.ntt(b, q, psi)
    assert np.array_equal(orc.intt(A, q, psi), a)
    C = (A.astype(np.uint64) * B.astype(np.uint64) % q).astype(np.uint32)
    assert list(orc.intt(C, q, psi)) == _brute_negacyclic(a, b, q)


def test_ntt_points_are_the_roots_of_x_n_plus_1():
    # NTT(X) lists the evaluation points: all distinct roots of X^N + 1
    N, q = 256, 2147352577
    psi = orc.find_psi(q, N)
    x = np.zeros(N, dtype=np.uint32)
    x[1] = 1
    pts = [int(v) for v in orc.ntt(x, q, psi)]
    assert len(set(pts)) == N
    assert all(pow(p, N, q) == q - 1 for p in pts)
    assert pts[0] == psi  # k = 0: psi^(2*0+1)
    ones = orc.ntt(np.eye(1, N, 0, dtype=np.uint32)[0], q, psi)
    assert np.all(ones == 1)


def test_ntt_sampled_indices_match_full():
    N, q = 512, 2147352577
    psi = orc.find_psi(q, N)
    a = np.random.default_rng(4).integers(0, q, N).astype(np.uint32)
    full = orc.ntt(a, q, psi)
    ks = np.array([0, 1, 100, 511], dtype=np.uint32)
    assert np.array_equal(orc.ntt(a, q, psi, ks), full[ks])


# ---------------------------------------------------------------- BFV (the "Homomorphic Operations in BFV" section)

@pytest.mark.parametrize("N,L,bits", [(1024, 2, 30), (4096, 3, 31)])
def test_encrypt_decrypt_roundtrip_and_fresh_noise(N, L, bits):
    primes = orc.ntt_primes(N, L, bits)
    s = orc.keygen(N, 11)
    rng = np.random.default_rng(5)
    t = 1 << 20
    m = rng.integers(-t // 2 + 1, t // 2 + 1, size=(2, N))
    m[0, :4] = [t // 2, -t // 2 + 1, 0, 1]
    ct = orc.encrypt(primes, 20, s, m, 99)
    assert np.array_equal(orc.decrypt(primes, 20, s, ct), m)
    # fresh noise v = e satisfies ||v|| <= B
    for j in range(2):
        assert orc.noise_inf(primes, 20, s, ct[j], m[j]) <= orc.B_ERR
    # c1 = -a is uniform per limb
    for i, q in enumerate(primes):
        assert abs(ct[:, 1, i].astype(np.float64).mean() / q - 0.5) < 0.02


def test_decrypt_detects_overflowing_noise():
    # noise beyond Delta/2 breaks decryption (correctness condition of the "Homomorphic Operations in BFV" section)
    N = 1024
    primes = orc.ntt_primes(N, 1, 31)
    q = primes[0]
    delta = q // (1 << 20)
    s = orc.keygen(N, 1)
    m = np.zeros((1, N), dtype=np.int64)
    ct = orc.encrypt(primes, 20, s, m, 5)
    ct[0, 0, 0, 0] = (int(ct[0, 0, 0, 0]) + delta // 2 + 64) % q  # push one coefficient
    assert orc.decrypt(primes, 20, s, ct)[0, 0] != 0


# ---------------------------------------------------------------- convolution

@pytest.mark.parametrize("k,dw", [(3, False), (1, False), (3, True)])
def test_direct_conv_matches_torch_conv2d(k, dw):
    x = wl.activations(1, 6, 9, 7)
    lay = wl.Layer("t", 9, 7, 6, 6 if dw else 5, k, depthwise=dw)
    w = wl.weights(2, lay)
    y = orc.direct_conv(x, w, k, dw)
    ref = torch.nn.functional.conv2d(torch.tensor(x, dtype=torch.float64)[None],
                                     torch.tensor(w, dtype=torch.float64),
                                     padding=(k - 1) // 2, groups=6 if dw else 1)[0]
    assert np.array_equal(y, ref.numpy().astype(np.int64))


def test_sparse_taps_equal_dense_kernel_product():
    N, L = 1024, 2
    primes = orc.ntt_primes(N, L, 31)
    pl = orc.plan(N, 6, 6, 5, 3, 3)
    rng = np.random.default_rng(6)
    ct = np.stack([rng.integers(0, q, size=(pl.tiles, pl.n_groups, 2, N)) for q in primes],
                  axis=3).astype(np.uint32)
    w = wl.weights(7, wl.Layer("t", 6, 6, 5, 3, 3))
    got = orc.conv_products(pl, ct, w, primes)
    for o in range(pl.Co):
        for p in range(2):
            for i, q in enumerate(primes):
                acc = np.zeros(N, dtype=np.int64)
                for g in range(pl.n_groups):
                    K = orc._lift(orc.kernel_poly(pl, w, o, g), q)
                    acc = (acc + orc.negacyclic_mul(ct[0, g, p, i], K, q)) % q
                assert np.array_equal(got[o, p, i], acc.astype(np.uint32))


CASES = [
    # (N, L, bits, H, W, Ci, Co, k, depthwise, ci_req)
    (4096, 2, 30, 16, 16, 16, 16, 3, False, None),   # the single-layer workload
    (1024, 2, 31, 40, 40, 3, 4, 3, False, None),     # row tiles with halo (42*42 > 1024)
    (1024, 2, 31, 8, 8, 7, 5, 3, False, None),       # short last channel group
    (1024, 2, 31, 8, 8, 6, 6, 3, True, None),        # depthwise
    (1024, 2, 31, 9, 9, 10, 4, 1, False, None),      # 1x1
    (1024, 2, 31, 8, 8, 9, 4, 3, False, 2),          # lowered channel partition
]


@pytest.mark.parametrize("case", CASES)
def test_he_conv_decrypts_to_plain_conv(case):
    # lossless claim: decrypting the HE convolution gives the plaintext
    # convolution exactly (the introduction and the "Optimal Parameter Selection" section)
    N, L, bits, H, W, Ci, Co, k, dw, cir = case
    primes = orc.ntt_primes(N, L, bits)
    pl = orc.plan(N, H, W, Ci, Co, k, dw, cir)
    lay = wl.Layer("t", H, W, Ci, Co, k, depthwise=dw)
    x = wl.activations(11, Ci, H, W)
    w = wl.weights(12, lay)
    assert orc.noise_ok(pl, w, primes)
    s = orc.keygen(N, 13)
    msgs = orc.pack_input(pl, x).reshape(-1, N)
    ct = orc.encrypt(primes, 20, s, msgs, 14).reshape(pl.tiles, pl.n_groups, 2, L, N)
    Y = orc.conv_products(pl, ct, w, primes)
    dec = orc.decrypt(primes, 20, s, Y).reshape(pl.tiles, pl.Co, N)
    y = orc.unpack_output(pl, dec)
    assert np.array_equal(y, orc.direct_conv(x, w, k, dw))


STRIDED = [
    # (N, L, H, W, Ci, Co, depthwise): MobileNetV1's stride-2 layer kinds,
    # scaled down (conv0: 3 -> 32 channels, 3x3, stride 2; dw: depthwise 3x3,
    # stride 2), with even and odd input sizes
    (1024, 2, 12, 12, 3, 8, False),
    (1024, 2, 13, 11, 3, 4, False),
    (1024, 2, 10, 10, 6, 6, True),
    (2048, 2, 9, 9, 8, 8, True),
]


@pytest.mark.parametrize("case", STRIDED)
def test_he_conv_subsampled_equals_strided_conv(case):
    # stride-2 layers (MobileNetV1, the "End-to-end Evaluation" section): the
    # server computes the stride-1 product; the decrypted, unpacked output
    # taken at every second row and column must be torch's stride-2
    # convolution with the same padding
    N, L, H, W, Ci, Co, dw = case
    primes = orc.ntt_primes(N, L, 31)
    pl = orc.plan(N, H, W, Ci, Co, 3, dw)
    lay = wl.Layer("t", H, W, Ci, Co, 3, stride=2, depthwise=dw)
    x = wl.activations(21, Ci, H, W)
    w = wl.weights(22, lay)
    s = orc.keygen(N, 23)
    ct = orc.encrypt(primes, 20, s, orc.pack_input(pl, x).reshape(-1, N), 24)
    Y = orc.conv_products(pl, ct.reshape(pl.tiles, pl.n_groups, 2, L, N), w, primes)
    y = orc.unpack_output(pl, orc.decrypt(primes, 20, s, Y).reshape(pl.tiles, pl.Co, N))
    got = orc.subsample(y, 2)
    ref = torch.nn.functional.conv2d(torch.tensor(x, dtype=torch.float64)[None],
                                     torch.tensor(w, dtype=torch.float64), stride=2,
                                     padding=1, groups=Ci if dw else 1)[0]
    assert got.shape == tuple(ref.shape)
    assert np.array_equal(got, ref.numpy().astype(np.int64))


def test_plan_vgg16_ciphertext_counts_by_hand():
    # Input ciphertexts per VGG-16 image at N = 8192, worked out by hand:
    # 224 (Wp 226, R 34, 7 tiles): 7*3 + 7*64; 112 (Wp 114, R 69, 2 tiles):
    # 2*64 + 2*128; 56 (58^2 = 3364, 2 ch): 64 + 128 + 128; 28 (900, 9 ch):
    # 29 + 57 + 57; 14 (256, 32 ch): 16 * 3.  Total 1364.
    pls = [orc.plan(8192, l.H, l.W, l.Ci, l.Co, l.k) for l in wl.vgg16_layers()]
    assert [p.tiles * p.n_groups for p in pls] == [21, 448, 128, 256, 64, 128, 128, 29, 57, 57, 16, 16, 16]
    assert sum(p.tiles * p.n_groups for p in pls) == 1364
    assert sum(p.tiles * p.Co for p in pls) == 5248
    assert pls[1].tiles == 7 and pls[1].R == 34


def test_noise_bound_rejects_single_limb():
    pl = orc.plan(4096, 16, 16, 16, 16, 3)
    w = np.full((16, 16, 3, 3), -8, dtype=np.int8)
    assert orc.noise_ok(pl, w, orc.ntt_primes(4096, 2, 30))
    assert not orc.noise_ok(pl, w, orc.ntt_primes(4096, 1, 31))


def test_noise_overflow_breaks_decryption():
    # L = 1 (Delta ~ 2^11): a 3x3x128 layer of maximal weights overflows
    N = 1024
    primes = orc.ntt_primes(N, 1, 31)
    pl = orc.plan(N, 4, 4, 128, 1, 3)
    x = np.full((128, 4, 4), 7, dtype=np.int8)
    w = np.full((1, 128, 3, 3), 7, dtype=np.int8)
    assert not orc.noise_ok(pl, w, primes)
    s = orc.keygen(N, 1)
    ct = orc.encrypt(primes, 20, s, orc.pack_input(pl, x).reshape(-1, N), 2)
    ct = ct.reshape(pl.tiles, pl.n_groups, 2, 1, N)
    dec = orc.decrypt(primes, 20, s, orc.conv_products(pl, ct, w, primes)).reshape(pl.tiles, 1, N)
    assert not np.array_equal(orc.unpack_output(pl, dec), orc.direct_conv(x, w, 3))


# ---------------------------------------------------------------- Walsh-Hadamard (the "Enabling Output Channel Packing" section)

def test_walsh_basis_c4_is_the_printed_one():
    assert np.array_equal(orc.walsh_matrix(4), _golden("walsh_basis_c4.txt"))


@pytest.mark.parametrize("c_n", [1, 2, 4, 8, 16, 32, 64])
def test_walsh_orthogonality(c_n):
    H = orc.walsh_matrix(c_n)
    assert np.array_equal(H @ H, c_n * np.eye(c_n, dtype=np.int64))
    assert np.array_equal(H, H.T) and set(np.unique(H)) <= {-1, 1}


def test_hadamard2_equation():
    rows = _golden("hadamard2_example.txt")
    for f0, f1, s, d in rows:
        assert (f0 + f1, f0 - f1) == (s, d)
        g = orc.walsh_weights(np.array([[f0], [f1]]), 2)[:, 0]
        assert list(g) == [s, d]
        assert list(orc.walsh_matrix(2) @ g) == [2 * f0, 2 * f1]


def test_walsh_kernel_is_kernel_of_walsh_weights_for_standard_layers():
    # linearity: for a standard layer the Walsh kernel equals the kernel
    # polynomial built from the Walsh weights g = H f
    N = 1024
    primes = orc.ntt_primes(N, 1, 31)
    pl = orc.plan(N, 6, 6, 5, 8, 3)
    w = wl.weights(3, wl.Layer("t", 6, 6, 5, 8, 3))
    gw = orc.walsh_weights(w, 4)
    q = primes[0]
    inv = pow(4, -1, q)
    for G in range(2):
        for j in range(4):
            want = (orc._lift(orc.kernel_poly(pl, gw, G * 4 + j, 0), q).astype(np.uint64) * inv) % q
            got = orc.walsh_kernel_residues(pl, w, 4, primes, G, j, 0)[0]
            assert np.array_equal(got, want.astype(np.uint32))


def test_walsh_weights_invert():
    w = wl.weights(3, wl.Layer("t", 4, 4, 5, 16, 3)).astype(np.int64)
    for c_n in (2, 4, 16):
        g = orc.walsh_weights(w, c_n)
        back = orc.walsh_weights(g, c_n)
        assert np.array_equal(back, c_n * w)


@pytest.mark.parametrize("c_n,dw", [(2, False), (4, False), (2, True), (4, True)])
def test_walsh_kernels_reproduce_plain_product(c_n, dw):
    # sum_j H[b][j] sum_g ct_g * (c_n^-1 Kw_{G,j,g}) == sum_g ct_g * K_{G c_n + b, g}
    N, L = 1024, 2
    primes = orc.ntt_primes(N, L, 31)
    C = 8
    pl = orc.plan(N, 6, 6, 5 if not dw else C, C, 3, dw)
    rng = np.random.default_rng(8)
    ct = np.stack([rng.integers(0, q, size=(pl.tiles, pl.n_groups, 2, N)) for q in primes],
                  axis=3).astype(np.uint32)
    w = wl.weights(9, wl.Layer("t", 6, 6, pl.Ci, C, 3, depthwise=dw))
    plain = orc.conv_products(pl, ct, w, primes)
    H = orc.walsh_matrix(c_n)
    for G in range(pl.Co // c_n):
        A = np.zeros((c_n, 2, L, N), dtype=np.int64)
        for j in range(c_n):
            for g in range(pl.n_groups):
                if dw and g != (G * c_n) // pl.ci:
                    continue
                Kw = orc.walsh_kernel_residues(pl, w, c_n, primes, G, j, g)
                for p in range(2):
                    for i, q in enumerate(primes):
                        A[j, p, i] = (A[j, p, i] + orc.negacyclic_mul(ct[0, g, p, i], Kw[i], q)) % q
        for b in range(c_n):
            for i, q in enumerate(primes):
                Y = sum(int(H[b, j]) * A[j, :, i] for j in range(c_n)) % q
                assert np.array_equal(Y, plain[G * c_n + b, :, i].astype(np.int64))
