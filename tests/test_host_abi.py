"""CPU tests of the C ABI: exported symbols and the host-side calls
(parameters, key generation, encryption, decryption, planning, packing)
against the oracle. No GPU is touched: contexts are created host-only."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as orc
import paper_2311_12519_amd as hy
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = hy.HYENA_HOST_ONLY


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|void|const char \*|uint32_t|size_t)\s*(hyena_\w+)\s*\(", src, re.M))
    return names


def test_library_exports_every_declared_symbol():
    L = hy.lib()
    names = _declared_symbols()
    assert len(names) >= 14
    for n in sorted(names):
        assert hasattr(L, n), n


def test_no_internal_symbols_exported():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", hy.LIB_PATH], capture_output=True, text=True).stdout
    syms = [l.split()[-1] for l in out.splitlines() if " T " in l]
    assert syms and all(s.startswith("hyena_") for s in syms), syms


@pytest.mark.parametrize("N,L,bits,flags", [(4096, 2, 30, hy.HYENA_PRIMES_30BIT), (8192, 3, 31, 0),
                                            (16384, 4, 31, 0)])
def test_params_match_oracle(N, L, bits, flags):
    ctx = hy.hyena_create(N, L, flags=flags | HOST)
    assert ctx.primes == orc.ntt_primes(N, L, bits)
    assert ctx.psi == [orc.find_psi(q, N) for q in ctx.primes]


@pytest.mark.parametrize("N", [4096, 8192, 16384])
def test_security_ceiling_enforced_at_its_edge(N):
    # the published 128-bit ceilings (tests/golden/he_standard_ternary_128.txt):
    # the default primes give the largest L whose sum of log2 q_i fits, one
    # limb more is refused unless HYENA_ALLOW_INSECURE
    table = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "he_standard_ternary_128.txt")):
        if line.strip() and not line.startswith("#"):
            n, b = line.split()
            table[int(n)] = int(b)
    primes = orc.ntt_primes(N, 16, 31)
    L = 0
    while sum(math.log2(q) for q in primes[:L + 1]) <= table[N]:
        L += 1
    assert L == {4096: 3, 8192: 7, 16384: 14}[N]
    hy.hyena_create(N, L, flags=HOST)
    with pytest.raises(hy.HyenaError) as e:
        hy.hyena_create(N, L + 1, flags=HOST)
    assert e.value.code == hy.HYENA_EUNSUPPORTED
    hy.hyena_create(N, L + 1, flags=HOST | hy.HYENA_ALLOW_INSECURE)


def test_bad_primes_rejected():
    with pytest.raises(hy.HyenaError):
        hy.hyena_create(4096, 1, primes=[2147352577 + 2], flags=HOST)  # not prime
    with pytest.raises(hy.HyenaError):
        hy.hyena_create(8192, 1, primes=[1073668097], flags=HOST)      # 1 mod 8192 only


@pytest.mark.parametrize("N,L,flags", [(4096, 2, hy.HYENA_PRIMES_30BIT), (8192, 3, 0)])
def test_keygen_encrypt_bit_exact_with_oracle(N, L, flags):
    ctx = hy.hyena_create(N, L, flags=flags | HOST)
    sk = hy.hyena_keygen(ctx, 4242)
    assert np.array_equal(sk, orc.keygen(N, 4242))
    rng = np.random.default_rng(0)
    m = rng.integers(-(1 << 19) + 1, (1 << 19) + 1, size=(3, N))
    ct = hy.hyena_encrypt(ctx, sk, m, 777)
    assert np.array_equal(ct, orc.encrypt(ctx.primes, 20, orc.keygen(N, 4242), m, 777))


def test_decrypt_matches_oracle_on_noisy_ciphertexts():
    N, L = 4096, 3
    ctx = hy.hyena_create(N, L, flags=HOST)
    s = orc.keygen(N, 5)
    pl = orc.plan(N, 16, 16, 16, 4, 3)
    x = wl.activations(1, 16, 16, 16)
    w = wl.weights(2, wl.Layer("t", 16, 16, 16, 4, 3))
    ct = orc.encrypt(ctx.primes, 20, s, orc.pack_input(pl, x).reshape(-1, N), 3)
    Y = orc.conv_products(pl, ct.reshape(pl.tiles, pl.n_groups, 2, L, N), w, ctx.primes)
    assert np.array_equal(hy.hyena_decrypt(ctx, s, Y), orc.decrypt(ctx.primes, 20, s, Y))


@pytest.mark.parametrize("N,L,flags", [(1024, 2, hy.HYENA_ALLOW_INSECURE), (4096, 3, hy.HYENA_PRIMES_30BIT)])
def test_decrypt_rounding_window_on_arbitrary_residues(N, L, flags):
    """Uniform residues put frac(t v / q) everywhere in [0, 1): the library's
    RNS rounding (fractions in 0.64 fixed point) equals the oracle's exact
    round(t v / q) on every coefficient whose fraction lies outside
    [1/2, 1/2 + L 2^-33), and is at most one less inside it."""
    import math
    ctx = hy.hyena_create(N, L, flags=HOST | flags)
    rng = np.random.default_rng(N + L)
    ct = np.empty((2, 2, L, N), dtype=np.uint32)
    for i, q in enumerate(ctx.primes):
        ct[:, :, i, :] = rng.integers(0, q, size=(2, 2, N))
    s = orc.keygen(N, 9)
    got = hy.hyena_decrypt(ctx, s, ct)
    want = orc.decrypt(ctx.primes, 20, s, ct)
    q = math.prod(int(p) for p in ctx.primes)
    t = 1 << 20
    outside = 0
    for m in range(2):
        v = orc.decrypt_phase(ctx.primes, s, ct[m])
        for j, x in enumerate(v):
            r = (t * x) % q
            if 2 * r >= q and (2 * r - q) * (1 << 32) < L * q:
                assert (int(got[m, j]) - int(want[m, j])) % t in (0, t - 1)
            else:
                assert got[m, j] == want[m, j], (m, j)
                outside += 1
    assert outside >= 2 * N - 2


def test_decrypt_rejects_noncanonical_residue():
    ctx = hy.hyena_create(4096, 2, flags=HOST | hy.HYENA_PRIMES_30BIT)
    ct = np.zeros((1, 2, 2, 4096), dtype=np.uint32)
    ct[0, 0, 1, 7] = ctx.primes[1]
    with pytest.raises(hy.HyenaError):
        hy.hyena_decrypt(ctx, np.zeros(4096, np.int8), ct)


def _all_layers():
    out = []
    for w in wl.WORKLOADS.values():
        for l in w.layers:
            out.append((w.N, w.L, w.prime_bits, l))
    return out


@pytest.mark.parametrize("N,L,bits,layer", _all_layers(), ids=lambda v: getattr(v, "name", str(v)))
def test_plan_matches_oracle(N, L, bits, layer):
    ctx = hy.hyena_create(N, L, flags=HOST | (hy.HYENA_PRIMES_30BIT if bits == 30 else 0))
    d = hy.hyena_conv_plan(ctx, layer.H, layer.W, layer.Ci, layer.Co, layer.k, stride=layer.stride,
                           depthwise=layer.depthwise)
    p = orc.plan(N, layer.H, layer.W, layer.Ci, layer.Co, layer.k, layer.depthwise)
    assert (d.pad, d.Wp, d.R, d.tiles, d.ci, d.Bt, d.O, d.n_groups) == (
        p.pad, p.Wp, p.R, p.tiles, p.ci, p.Bt, p.O, p.n_groups)
    assert d.n_in == p.tiles * p.n_groups and d.n_out == p.tiles * p.Co


@pytest.mark.parametrize("shape", [(4096, 16, 16, 16, 16, 3), (1024, 40, 40, 3, 2, 3), (1024, 9, 9, 10, 3, 1),
                                   (1024, 41, 39, 2, 3, 3)])
def test_pack_unpack_match_oracle(shape):
    N, H, W, Ci, Co, k = shape
    ctx = hy.hyena_create(N, 2, flags=HOST | hy.HYENA_ALLOW_INSECURE)
    d = hy.hyena_conv_plan(ctx, H, W, Ci, Co, k)
    p = orc.plan(N, H, W, Ci, Co, k)
    x = wl.activations(9, Ci, H, W)
    msg = hy.hyena_pack_input(d, N, x)
    assert np.array_equal(msg, orc.pack_input(p, x))
    rng = np.random.default_rng(1)
    out = rng.integers(-1000, 1000, size=(p.tiles, Co, N)).astype(np.int32)
    assert np.array_equal(hy.hyena_unpack_output(d, N, out), orc.unpack_output(p, out))
    # a stride-2 descriptor unpacks every second row and column
    d2 = hy.hyena_conv_plan(ctx, H, W, Ci, Co, k, stride=2)
    assert np.array_equal(hy.hyena_unpack_output(d2, N, out), orc.subsample(orc.unpack_output(p, out), 2))


def test_plan_noise_and_shape_errors():
    ctx1 = hy.hyena_create(4096, 1, flags=HOST)
    with pytest.raises(hy.HyenaError) as e:
        hy.hyena_conv_plan(ctx1, 16, 16, 16, 16, 3)
    assert e.value.code == hy.HYENA_ENOISE
    ctx = hy.hyena_create(4096, 2, flags=HOST | hy.HYENA_PRIMES_30BIT)
    for kw in (dict(c_n=3), dict(c_n=32), dict(k=5)):
        args = dict(H=16, W=16, Ci=16, Co=16, k=3)
        args.update(kw)
        with pytest.raises(hy.HyenaError) as e:
            hy.hyena_conv_plan(ctx, args.pop("H"), args.pop("W"), args.pop("Ci"), args.pop("Co"),
                               args.pop("k"), **args)
        assert e.value.code == hy.HYENA_EINVAL
    # |y| bound: 3x3 over 1024 channels of 4-bit values exceeds t/2 = 2^19
    ctxb = hy.hyena_create(16384, 4, flags=HOST)
    with pytest.raises(hy.HyenaError) as e:
        hy.hyena_conv_plan(ctxb, 8, 8, 1024, 8, 3)
    assert e.value.code == hy.HYENA_ENOISE


def test_device_calls_refused_on_host_only_context():
    ctx = hy.hyena_create(4096, 2, flags=HOST | hy.HYENA_PRIMES_30BIT)
    rc = hy.lib().hyena_ntt(ctx.handle, ctypes.c_void_p(0), 0, ctypes.c_void_p(0))
    assert rc == hy.HYENA_EINVAL


def test_client_device_calls_refused_on_host_only_context():
    """The batched client entry points check their arguments before any launch:
    NULL arrays and host-only contexts are refused, n = 0 is a no-op."""
    ctx = hy.hyena_create(4096, 2, flags=HOST | hy.HYENA_PRIMES_30BIT)
    L = hy.lib()
    fake = ctypes.c_void_p(0x10000)      # never dereferenced: every call below fails its checks first
    null = ctypes.c_void_p(0)
    assert L.hyena_secret_prepare(ctx.handle, null, fake, null) == hy.HYENA_EINVAL
    assert L.hyena_secret_prepare(ctx.handle, fake, fake, null) == hy.HYENA_EINVAL   # host-only
    assert L.hyena_encrypt_device(ctx.handle, fake, null, 1, 5, fake, fake, null) == hy.HYENA_EINVAL
    assert L.hyena_encrypt_device(ctx.handle, fake, fake, 1, 5, fake, fake, null) == hy.HYENA_EINVAL
    assert L.hyena_decrypt_device(ctx.handle, fake, fake, 1, null, fake, null) == hy.HYENA_EINVAL
    assert L.hyena_decrypt_device(ctx.handle, fake, fake, 1, fake, fake, null) == hy.HYENA_EINVAL
    assert "host-only" in L.hyena_last_error().decode()


def test_synth_weights_refusals():
    """hyena_synth_weights checks its arguments before any launch: NULL arrays,
    depthwise layers (EUNSUPPORTED) and host-only contexts are refused."""
    ctx = hy.hyena_create(4096, 2, flags=HOST | hy.HYENA_PRIMES_30BIT)
    L = hy.lib()
    fake = ctypes.c_void_p(0x10000)      # never dereferenced: every call below fails its checks first
    null = ctypes.c_void_p(0)
    d = hy.hyena_conv_plan(ctx, 16, 16, 16, 16, 3)
    dd = hy.hyena_conv_plan(ctx, 16, 16, 16, 16, 3, depthwise=True)
    assert L.hyena_synth_weights(ctx.handle, ctypes.byref(d), null, fake, null) == hy.HYENA_EINVAL
    assert L.hyena_synth_weights(ctx.handle, ctypes.byref(dd), fake, fake, null) == hy.HYENA_EUNSUPPORTED
    assert L.hyena_synth_weights(ctx.handle, ctypes.byref(d), fake, fake, null) == hy.HYENA_EINVAL
    assert "host-only" in L.hyena_last_error().decode()
    # a c_n that is not a power of two (which hyena_conv_plan never returns)
    d3 = hy.hyena_conv_plan(ctx, 16, 16, 16, 12, 3)
    d3.c_n = 3
    assert L.hyena_synth_weights(ctx.handle, ctypes.byref(d3), fake, fake, null) == hy.HYENA_EINVAL
    assert "power of two" in L.hyena_last_error().decode()


def test_simd_params_match_the_papers_example_and_the_oracle():
    """hyena_simd_params (closed form h = (w + w^3)^-1, w = zeta^(n/4)) against
    the paper's worked example and the oracle's brute-force encoding."""
    import os
    from oracle import simd
    g = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "simd_parameter_example.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            g[k] = v
    h, k, kh = hy.hyena_simd_params(int(g["n"]), int(g["p"]), 61)
    assert (h, k) == (int(g["h"]), int(g["k"])) and kh == k * h % int(g["p"])
    for n, p in [(1024, 12289), (4096, 65537), (1024, 307201)]:
        h, k, kh = hy.hyena_simd_params(n, p, 200)
        assert h == simd.h_pn(n, p)
        assert (k, kh) == simd.best_k(h, p, 200)
    for bad in [(2048, 307203, 61), (4096, 12289, 61), (6, 13, 5), (2048, 307201, 0)]:
        with pytest.raises(hy.HyenaError):
            hy.hyena_simd_params(*bad)


def test_plaintext_prime_context_and_simd_calls_on_host_only_context():
    ctx = hy.hyena_create(2048, 1, primes=[307201], flags=HOST | hy.HYENA_PLAINTEXT_PRIME)
    assert ctx.primes == [307201] and ctx.psi == [41]     # the least primitive 4096-th root
    with pytest.raises(hy.HyenaError):                    # without the flag the prime is refused
        hy.hyena_create(2048, 1, primes=[307201], flags=HOST)
    with pytest.raises(hy.HyenaError):                    # the flag needs the prime
        hy.hyena_create(2048, 1, flags=HOST | hy.HYENA_PLAINTEXT_PRIME)
    L = hy.lib()
    fake = ctypes.c_void_p(0x10000)
    null = ctypes.c_void_p(0)
    assert L.hyena_simd_encode(ctx.handle, fake, 1, fake, null) == hy.HYENA_EINVAL
    assert L.hyena_simd_decode(ctx.handle, fake, 1, fake, null) == hy.HYENA_EINVAL
    assert L.hyena_automorphism(ctx.handle, fake, 1, 3, fake, null) == hy.HYENA_EINVAL
    e = (ctypes.c_uint32 * 1)(512)
    assert L.hyena_pmult_sparse(ctx.handle, fake, 1, 1, e, e, fake, null) == hy.HYENA_EINVAL


def test_galois_keygen_matches_oracle():
    """Host key-switching keys equal the oracle's bit for bit (same draws)."""
    from oracle import simd
    primes = orc.ntt_primes(1024, 2, 30)
    ctx = hy.hyena_create(1024, 2, primes=primes, flags=HOST | hy.HYENA_ALLOW_INSECURE)
    s = orc.keygen(1024, 12)
    for g, b in [(3, 16), (2047, 29), (9, 8)]:
        assert np.array_equal(hy.hyena_galois_keygen(ctx, s, g, b, 77 + g), simd.galois_keygen(primes, s, g, b, 77 + g))
    for g, b in [(4, 16), (3, 0), (3, 30)]:
        with pytest.raises(hy.HyenaError):
            hy.hyena_galois_keygen(ctx, s, g, b, 1)


def test_simd_conv_weights():
    rng = np.random.default_rng(1)
    f = rng.integers(-8, 8, size=(3, 4, 3, 3)).astype(np.int8)
    wa, wb = hy.hyena_simd_conv_weights(f, 11)
    for o in range(3):
        for g in range(2):
            f0, f1 = f[o, 2 * g].reshape(9).astype(np.int32), f[o, 2 * g + 1].reshape(9).astype(np.int32)
            assert np.array_equal(wa[o, g * 9:(g + 1) * 9], 11 * (f0 + f1))
            assert np.array_equal(wb[o, g * 9:(g + 1) * 9], f0 - f1)
    with pytest.raises(hy.HyenaError):                    # odd channel count
        hy.hyena_simd_conv_weights(f[:, :3], 11)
    with pytest.raises(hy.HyenaError):                    # scalars would exceed 2^16
        hy.hyena_simd_conv_weights(f, 256)


def test_cmult_accumulate_refuses_null_output_even_without_inputs():
    """R = 0 still writes O (zero) outputs, so a NULL output is refused before
    anything else (a host-only context would refuse next)."""
    ctx = hy.hyena_create(4096, 2, flags=HOST | hy.HYENA_PRIMES_30BIT)
    null = ctypes.c_void_p(0)
    assert hy.lib().hyena_cmult_accumulate(ctx.handle, null, 0, null, 3, null, null) == hy.HYENA_EINVAL
    assert "NULL" in hy.lib().hyena_last_error().decode()


def test_simd_conv_weights_packed():
    rng = np.random.default_rng(2)
    f = rng.integers(-8, 8, size=(4, 4, 3, 3)).astype(np.int8)
    wa, wb = hy.hyena_simd_conv_weights_packed(f, 11)
    G = 2
    for o2 in range(2):
        o = 2 * o2
        for h in range(2):
            for g in range(G):
                a = f[o, 2 * g + h].reshape(9).astype(np.int32)
                b = f[o + 1, 2 * g + 1 - h].reshape(9).astype(np.int32)
                sl = slice((h * G + g) * 9, (h * G + g + 1) * 9)
                assert np.array_equal(wa[o2, sl], 11 * (a + b)) and np.array_equal(wb[o2, sl], a - b)
    with pytest.raises(hy.HyenaError):                    # odd output count
        hy.hyena_simd_conv_weights_packed(f[:3], 11)


def test_synth_taps_and_conv_synth_refusals():
    """The integer-tap calls check their arguments before any launch: NULL
    arrays, unplanned descriptors, depthwise layers (EUNSUPPORTED), more than
    18 taps per word (EUNSUPPORTED) and host-only contexts are refused."""
    ctx = hy.hyena_create(8192, 3, flags=HOST)
    L = hy.lib()
    fake = ctypes.c_void_p(0x10000)      # never dereferenced: every call below fails its checks first
    null = ctypes.c_void_p(0)
    d = hy.hyena_conv_plan(ctx, 64, 64, 3, 8, 3)                      # 9 taps per word
    dd = hy.hyena_conv_plan(ctx, 14, 14, 32, 32, 3, depthwise=True)
    big = hy.hyena_conv_plan(ctx, 14, 14, 64, 32, 3)                  # 288 taps per word
    assert L.hyena_synth_taps(ctx.handle, ctypes.byref(d), null, fake, null) == hy.HYENA_EINVAL
    assert L.hyena_synth_taps(ctx.handle, ctypes.byref(dd), fake, fake, null) == hy.HYENA_EUNSUPPORTED
    assert L.hyena_synth_taps(ctx.handle, ctypes.byref(d), fake, fake, null) == hy.HYENA_EINVAL
    assert "host-only" in L.hyena_last_error().decode()
    assert L.hyena_conv_synth(ctx.handle, ctypes.byref(d), fake, null, fake, null) == hy.HYENA_EINVAL
    assert L.hyena_conv_synth(ctx.handle, ctypes.byref(dd), fake, fake, fake, null) == hy.HYENA_EUNSUPPORTED
    assert L.hyena_conv_synth(ctx.handle, ctypes.byref(big), fake, fake, fake, null) == hy.HYENA_EUNSUPPORTED
    assert L.hyena_conv_synth(ctx.handle, ctypes.byref(d), fake, fake, fake, null) == hy.HYENA_EINVAL
    assert "host-only" in L.hyena_last_error().decode()
    # schedule table: the streaming schedules report 0, the synthesizing ones their tap bound
    taps = [hy.hyena_conv_schedule_taps(s) for s in range(len(hy.hyena_conv_schedules()))]
    assert taps.count(0) >= 25 and sorted(set(taps) - {0}) == [9, 18]
    assert hy.synth_taps_words(d) == 8 * 3 * 12
