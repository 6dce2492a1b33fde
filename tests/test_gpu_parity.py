"""GPU parity: every HIP kernel against the oracle, bit for bit.

Inputs come from the seeded generators and the oracle's encryption; expected
values come from the oracle only. Outputs are compared on every coefficient of
every limb and ciphertext part (ring elements are exact integers, so the bar
is bit equality)."""
import sys

import numpy as np
import pytest

import oracle as orc
import paper_2311_12519_amd as hy
import workloads as wl

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


def rand_res(rng, shape, primes):
    """uint32 [..., L, N] uniform residues per limb."""
    out = np.empty(shape, dtype=np.uint32)
    for i, q in enumerate(primes):
        out[..., i, :] = rng.integers(0, q, size=shape[:-2] + (shape[-1],))
    return out


_CTX = {}


def ctx_for(N, L, bits):
    key = (N, L, bits)
    if key not in _CTX:
        flags = (hy.HYENA_PRIMES_30BIT if bits == 30 else 0) | (hy.HYENA_ALLOW_INSECURE if N < 4096 else 0)
        _CTX[key] = hy.hyena_create(N, L, flags=flags)
    return _CTX[key]


# ---------------------------------------------------------------- NTT

@pytest.mark.parametrize("N,L,bits", [(1024, 2, 31), (2048, 2, 31), (4096, 2, 30), (8192, 3, 31), (16384, 4, 31),
                                     (8192, 3, 30), (16384, 2, 30)])
def test_ntt_matches_oracle(dev, N, L, bits):
    say(f"ntt N={N} L={L}")
    ctx = ctx_for(N, L, bits)
    rng = np.random.default_rng(N)
    a = rand_res(rng, (2, L, N), ctx.primes)
    for i, q in enumerate(ctx.primes):           # edge residues
        a[0, i, :4] = [0, q - 1, 1, q - 2]
    d = to_dev(a)
    hy.hyena_ntt(ctx, d)
    got = from_dev(d)
    for p in range(2):
        for i, q in enumerate(ctx.primes):
            assert np.array_equal(got[p, i], orc.ntt(a[p, i], q, ctx.psi[i])), (p, i)
    hy.hyena_intt(ctx, d)
    assert np.array_equal(from_dev(d), a)


@pytest.mark.parametrize("N,L,bits", [(4096, 2, 30), (8192, 3, 31), (16384, 4, 31), (8192, 3, 30)])
def test_intt_matches_oracle(dev, N, L, bits):
    say(f"intt N={N}")
    ctx = ctx_for(N, L, bits)
    rng = np.random.default_rng(N + 1)
    A = rand_res(rng, (1, L, N), ctx.primes)
    d = to_dev(A)
    hy.hyena_intt(ctx, d)
    got = from_dev(d)
    for i, q in enumerate(ctx.primes):
        assert np.array_equal(got[0, i], orc.intt(A[0, i], q, ctx.psi[i]))


def test_ntt_many_polys_roundtrip_and_empty(dev):
    import torch
    ctx = ctx_for(8192, 3, 31)
    rng = np.random.default_rng(3)
    a = rand_res(rng, (97, 3, 8192), ctx.primes)
    d = to_dev(a)
    hy.hyena_ntt(ctx, d)
    mid = from_dev(d)
    k = 57  # spot-check one polynomial in the middle of the launch
    for i, q in enumerate(ctx.primes):
        assert np.array_equal(mid[k, i], orc.ntt(a[k, i], q, ctx.psi[i]))
    hy.hyena_intt(ctx, d)
    assert np.array_equal(from_dev(d), a)
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    hy.hyena_ntt(ctx, empty)


# ---------------------------------------------------------------- weights

@pytest.mark.parametrize("c_n,dw", [(1, False), (2, False), (4, False), (1, True), (2, True)])
def test_encode_weights_matches_oracle(dev, c_n, dw):
    import torch
    say(f"encode c_n={c_n} dw={dw}")
    N, L = 4096, 2
    ctx = ctx_for(N, L, 30)
    lay = wl.Layer("t", 16, 16, 16, 16, 3, depthwise=dw)
    d = hy.hyena_conv_plan(ctx, 16, 16, 16, 16, 3, depthwise=dw, c_n=c_n)
    pl = orc.plan(N, 16, 16, 16, 16, 3, dw)
    w = wl.weights(21, lay)
    dw_t = torch.from_numpy(w).cuda()
    out = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device="cuda")
    hy.hyena_encode_weights(ctx, d, dw_t, out)
    got = from_dev(out).reshape(16, d.w_groups, L, N)
    for o in range(16):
        G, j = divmod(o, c_n)
        gs = [o // pl.ci] if dw else range(pl.n_groups)
        for slot, g in enumerate(gs):
            Kw = orc.walsh_kernel_residues(pl, w, c_n, ctx.primes, G, j, g)
            for i, q in enumerate(ctx.primes):
                # the encoding is documented as 2^32 times the NTT (Montgomery form)
                want = (orc.ntt(Kw[i], q, ctx.psi[i]).astype(np.uint64) << np.uint64(32)) % np.uint64(q)
                assert np.array_equal(got[o, 0 if dw else slot, i], want.astype(np.uint32)), (o, g, i)


@pytest.mark.parametrize("N,L,bits,H,Ci,Co,k,c_n", [
    (4096, 2, 30, 16, 16, 16, 3, 1),     # ci = 12: two input groups, the second ragged
    (4096, 2, 30, 16, 16, 16, 3, 4),     # Walsh-combined taps
    (8192, 3, 31, 64, 3, 20, 3, 1),      # ci = 1 (9 taps per word), 60 polynomials
    (8192, 3, 31, 14, 64, 32, 1, 2),     # 1x1 kernel
    (16384, 2, 31, 7, 100, 8, 3, 8),     # many taps per word
])
def test_synth_weights_equals_encode_weights(dev, N, L, bits, H, Ci, Co, k, c_n):
    """hyena_synth_weights (evaluation-domain synthesis, no NTT) against
    hyena_encode_weights on every word, and against the oracle's kernel
    polynomials on the first and last output channel."""
    import torch
    say(f"synth N={N} L={L} H={H} Ci={Ci} Co={Co} k={k} c_n={c_n}")
    ctx = ctx_for(N, L, bits)
    lay = wl.Layer("t", H, H, Ci, Co, k)
    d = hy.hyena_conv_plan(ctx, H, H, Ci, Co, k, c_n=c_n)
    w = wl.weights(5 + c_n, lay)
    dw_t = torch.from_numpy(w).cuda()
    n = hy.wntt_words(ctx, d)
    enc = torch.empty(n, dtype=torch.int32, device="cuda")
    syn = torch.full((n,), -1, dtype=torch.int32, device="cuda")   # every word must be written
    hy.hyena_encode_weights(ctx, d, dw_t, enc)
    hy.hyena_synth_weights(ctx, d, dw_t, syn)
    a, b = from_dev(enc), from_dev(syn)
    assert np.array_equal(a, b), int(np.count_nonzero(a != b))
    pl = orc.plan(N, H, H, Ci, Co, k)
    got = b.reshape(Co, d.w_groups, L, N)
    for o in (0, Co - 1):
        G, j = divmod(o, c_n)
        for g in range(pl.n_groups):
            Kw = orc.walsh_kernel_residues(pl, w, c_n, ctx.primes, G, j, g)
            for i, q in enumerate(ctx.primes):
                want = (orc.ntt(Kw[i], q, ctx.psi[i]).astype(np.uint64) << np.uint64(32)) % np.uint64(q)
                assert np.array_equal(got[o, g, i], want.astype(np.uint32)), (o, g, i)


@pytest.mark.parametrize("pattern", ["all_min", "alternating", "all_max"])
def test_synth_weights_full_int8_range_at_cn64(dev, pattern):
    """The synthesis kernel's overflow argument at its edge: full-range int8
    weights at c_n = 64 make Walsh weights of magnitude up to 64 * 128 = 2^13
    (all -128: the first Walsh row is -8192; -128/127 alternating along the
    output channels: rows of +-8160), over 576 taps per word (ci = 64 at
    N = 16384). Every word must equal the scatter + NTT encoding, and the
    first and last output channels the oracle's NTT of the Walsh kernel."""
    import torch
    say(f"synth full int8 range c_n=64 {pattern}")
    N, L, H, Ci, Co, c_n = 16384, 2, 14, 64, 64, 64
    ctx = ctx_for(N, L, 31)
    d = hy.hyena_conv_plan(ctx, H, H, Ci, Co, 3, c_n=c_n)
    assert d.ci == 64 and d.w_groups == 1
    if pattern == "all_min":
        w = np.full((Co, Ci, 3, 3), -128, dtype=np.int8)
    elif pattern == "all_max":
        w = np.full((Co, Ci, 3, 3), 127, dtype=np.int8)
    else:
        w = np.where((np.arange(Co) % 2 == 0)[:, None, None, None], -128, 127) * np.ones((1, Ci, 3, 3))
        w = w.astype(np.int8)
    dw_t = torch.from_numpy(w).cuda()
    n = hy.wntt_words(ctx, d)
    enc = torch.empty(n, dtype=torch.int32, device="cuda")
    syn = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    hy.hyena_encode_weights(ctx, d, dw_t, enc)
    hy.hyena_synth_weights(ctx, d, dw_t, syn)
    a, b = from_dev(enc), from_dev(syn)
    assert np.array_equal(a, b), int(np.count_nonzero(a != b))
    pl = orc.plan(N, H, H, Ci, Co, 3)
    got = b.reshape(Co, d.w_groups, L, N)
    for o in (0, 1, Co - 1):
        G, j = divmod(o, c_n)
        Kw = orc.walsh_kernel_residues(pl, w, c_n, ctx.primes, G, j, 0)
        for i, q in enumerate(ctx.primes):
            want = (orc.ntt(Kw[i], q, ctx.psi[i]).astype(np.uint64) << np.uint64(32)) % np.uint64(q)
            assert np.array_equal(got[o, 0, i], want.astype(np.uint32)), (o, i)


# ---------------------------------------------------------------- Walsh-Hadamard

@pytest.mark.parametrize("c_n", [2, 4, 8, 64])
def test_wht_pack_matches_oracle(dev, c_n):
    N, L = 4096, 2
    ctx = ctx_for(N, L, 30)
    G = 3
    rng = np.random.default_rng(c_n)
    x = rand_res(rng, (G, c_n, 2, L, N), ctx.primes)
    x[0, :, 0, 0, 0] = ctx.primes[0] - 1
    d = to_dev(x)
    hy.hyena_wht_pack(ctx, c_n, d, d, G)          # in place
    got = from_dev(d)
    H = orc.walsh_matrix(c_n)
    for i, q in enumerate(ctx.primes):
        want = np.einsum("bj,Gjpn->Gbpn", H, x[:, :, :, i, :].astype(np.int64)) % q
        assert np.array_equal(got[:, :, :, i, :], want.astype(np.uint32))


# ---------------------------------------------------------------- end to end

def run_layer(ctx, lay, c_n, seed, batch=1, fuse=True, ci_req=0, check_decrypt=True):
    """Oracle-encrypted inputs -> GPU ntt, conv, (wht), intt -> compare with
    oracle products on every coefficient, then decrypt and compare with the
    plaintext convolution."""
    import torch
    N, L = ctx.N, ctx.L
    flags = hy.HYENA_FUSE_WHT if fuse else 0
    d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, stride=lay.stride, depthwise=lay.depthwise,
                           c_n=c_n, flags=flags, batch=batch, ci_req=ci_req)
    pl = orc.plan(N, lay.H, lay.W, lay.Ci, lay.Co, lay.k, lay.depthwise, ci_req or None)
    w = wl.weights(seed, lay)
    s = orc.keygen(N, wl.crypto_seed(seed))
    xs, cts = [], []
    for b in range(batch):
        x = wl.activations(seed + 100 * b, lay.Ci, lay.H, lay.W)
        ct = orc.encrypt(ctx.primes, 20, s, orc.pack_input(pl, x).reshape(-1, N), wl.crypto_seed(seed) + b)
        xs.append(x)
        cts.append(ct.reshape(pl.tiles, pl.n_groups, 2, L, N))
    ct_all = np.stack(cts)
    d_ct = to_dev(ct_all)
    d_w = torch.from_numpy(w).cuda()
    d_wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device="cuda")
    d_out = torch.empty(batch * pl.tiles * lay.Co * 2 * L * N, dtype=torch.int32, device="cuda")
    hy.hyena_encode_weights(ctx, d, d_w, d_wn)
    hy.hyena_ntt(ctx, d_ct)
    hy.hyena_conv(ctx, d, d_ct, d_wn, d_out)
    if not fuse and c_n > 1:
        hy.hyena_wht_pack(ctx, c_n, d_out, d_out, batch * pl.tiles * lay.Co // c_n)
    hy.hyena_intt(ctx, d_out)
    got = from_dev(d_out).reshape(batch, pl.tiles, lay.Co, 2, L, N)
    for b in range(batch):
        want = orc.conv_products(pl, cts[b], w, ctx.primes).reshape(pl.tiles, lay.Co, 2, L, N)
        bad = np.argwhere(got[b] != want)
        assert bad.size == 0, f"image {b}: {len(bad)} mismatches, first at {bad[:3].tolist()}"
        if check_decrypt:
            dec = hy.hyena_decrypt(ctx, s, got[b].reshape(-1, 2, L, N)).reshape(pl.tiles, lay.Co, N)
            y = hy.hyena_unpack_output(d, N, dec)
            want_y = orc.subsample(orc.direct_conv(xs[b], w, lay.k, lay.depthwise), lay.stride)
            assert np.array_equal(y, want_y)


CONFIGS = [
    # id, (N, L, bits), layer, c_n
    ("single16", (4096, 2, 30), wl.WORKLOADS[1].layers[0], 1),
    ("resnet32", (8192, 3, 31), wl.WORKLOADS[2].layers[0], 1),
    ("resnet56_cn4", (16384, 4, 31), wl.WORKLOADS[3].layers[0], 4),
    ("resnet14_cn64", (16384, 4, 31), wl.WORKLOADS[3].layers[1], 64),
]


@pytest.mark.parametrize("name,params,lay,c_n", CONFIGS, ids=[c[0] for c in CONFIGS])
def test_workload_layers_end_to_end(dev, name, params, lay, c_n):
    say(f"e2e {name}")
    run_layer(ctx_for(*params), lay, c_n, seed=1000 + len(name))


VARIANTS = [
    ("tiles_halo", (4096, 2, 30), wl.Layer("t", 70, 70, 3, 8, 3), 1, 1, True, 0),
    ("short_group", (4096, 2, 30), wl.Layer("t", 12, 12, 37, 8, 3), 2, 1, True, 0),
    ("depthwise", (8192, 3, 31), wl.Layer("t", 28, 28, 32, 32, 3, depthwise=True), 1, 1, True, 0),
    ("depthwise_cn2", (8192, 3, 31), wl.Layer("t", 14, 14, 64, 64, 3, depthwise=True), 2, 1, True, 0),
    ("pointwise", (8192, 3, 31), wl.Layer("t", 14, 14, 64, 40, 1), 8, 1, True, 0),
    ("unfused_cn4", (4096, 2, 30), wl.Layer("t", 16, 16, 16, 16, 3), 4, 1, False, 0),
    ("batch3_cn2", (4096, 2, 30), wl.Layer("t", 16, 16, 16, 16, 3), 2, 3, True, 0),
    ("ci_lowered", (4096, 2, 30), wl.Layer("t", 16, 16, 16, 8, 3), 1, 1, True, 5),
    ("cn32_unfusable", (8192, 3, 31), wl.Layer("t", 14, 14, 32, 32, 3), 32, 1, True, 0),
    ("primes30_batch8", (8192, 3, 30), wl.Layer("t", 28, 28, 64, 32, 3), 1, 8, True, 0),
    # MobileNetV1's stride-2 layer kinds (conv0 3 -> 32 at 56x56, a depthwise
    # 3x3 at 28x28): stride-1 server work, every second row and column unpacked
    ("stride2_conv0", (8192, 3, 31), wl.Layer("t", 56, 56, 3, 32, 3, stride=2), 1, 2, True, 0),
    ("stride2_depthwise", (8192, 3, 31), wl.Layer("t", 28, 28, 64, 64, 3, stride=2, depthwise=True), 1, 1, True, 0),
    # the largest ring and the most limbs the 128-bit ceiling allows (14 x 31 bits)
    ("n16384_max_limbs", (16384, 14, 31), wl.Layer("t", 14, 14, 16, 8, 3), 2, 1, True, 0),
]


@pytest.mark.parametrize("name,params,lay,c_n,batch,fuse,ci_req", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_layer_variants_end_to_end(dev, name, params, lay, c_n, batch, fuse, ci_req):
    say(f"variant {name}")
    run_layer(ctx_for(*params), lay, c_n, seed=2000 + len(name), batch=batch, fuse=fuse, ci_req=ci_req)


def test_vgg_conv1_2_full_size_sampled(dev):
    """VGG-16 conv1_2 (224x224, 64 -> 64, 7 row tiles) at N = 8192, two images,
    in the default launch configuration; sampled output ciphertexts are checked
    against the oracle on every coefficient."""
    import torch
    say("vgg conv1_2 full size")
    ctx = ctx_for(8192, 3, 31)
    lay = wl.vgg16_layers()[1]
    N, L, batch = 8192, 3, 2
    d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, 3, batch=batch, flags=hy.HYENA_FUSE_WHT)
    pl = orc.plan(N, lay.H, lay.W, lay.Ci, lay.Co, 3)
    rng = np.random.default_rng(12)
    ct = rand_res(rng, (batch, pl.tiles, pl.n_groups, 2, L, N), ctx.primes)
    w = wl.weights(4001, lay)
    d_ct = to_dev(ct)
    d_wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device="cuda")
    d_out = torch.empty(batch * pl.tiles * lay.Co * 2 * L * N, dtype=torch.int32, device="cuda")
    hy.hyena_encode_weights(ctx, d, torch.from_numpy(w).cuda(), d_wn)
    hy.hyena_ntt(ctx, d_ct)
    hy.hyena_conv(ctx, d, d_ct, d_wn, d_out)
    hy.hyena_intt(ctx, d_out)
    got = from_dev(d_out).reshape(batch, pl.tiles, lay.Co, 2, L, N)
    sel = [(0, 0), (3, 17), (6, 63)]
    for b in range(batch):
        want = orc.conv_products(pl, ct[b], w, ctx.primes, outputs=sel)
        for u, (tau, o) in enumerate(sel):
            assert np.array_equal(got[b, tau, o], want[u]), (b, tau, o)


@pytest.mark.parametrize("lay,c_n,batch", [
    (wl.Layer("t", 14, 14, 64, 48, 3), 4, 3),   # rows = 6, partial row and output blocks
    (wl.Layer("t", 28, 28, 40, 24, 3), 2, 8),   # rows = 16, 5 input groups (stage tail)
    (wl.Layer("t", 14, 14, 32, 32, 3, depthwise=True), 2, 2),
], ids=["std_rows6", "std_rows16", "depthwise"])
def test_every_mac_schedule_matches_oracle(dev, lay, c_n, batch):
    """All MAC schedules (register-only and LDS-pipelined) give the oracle's
    output on every coefficient."""
    import torch
    ctx = ctx_for(8192, 3, 31)
    N, L = 8192, 3
    d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, depthwise=lay.depthwise, c_n=c_n,
                           flags=hy.HYENA_FUSE_WHT, batch=batch)
    pl = orc.plan(N, lay.H, lay.W, lay.Ci, lay.Co, lay.k, lay.depthwise)
    rng = np.random.default_rng(31)
    ct = rand_res(rng, (batch, pl.tiles, pl.n_groups, 2, L, N), ctx.primes)
    w = wl.weights(77, lay)
    d_ct = to_dev(ct)
    d_wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device="cuda")
    d_out = torch.empty(batch * pl.tiles * lay.Co * 2 * L * N, dtype=torch.int32, device="cuda")
    hy.hyena_encode_weights(ctx, d, torch.from_numpy(w).cuda(), d_wn)
    hy.hyena_ntt(ctx, d_ct)
    want = [orc.conv_products(pl, ct[b], w, ctx.primes).reshape(pl.tiles, lay.Co, 2, L, N) for b in range(batch)]
    ran = 0
    streamed = [sid for sid in range(len(hy.hyena_conv_schedules())) if hy.hyena_conv_schedule_taps(sid) == 0]
    for sid, info in enumerate(hy.hyena_conv_schedules()):
        if sid not in streamed:
            continue   # synthesizing schedules read integer taps (test_conv_synth_equals_streamed_weights)
        try:
            hy.hyena_conv_tiled(ctx, d, d_ct, d_wn, d_out, sid)
        except hy.HyenaError as e:
            assert lay.depthwise and e.code == hy.HYENA_EINVAL, (sid, info)
            continue
        o = d_out.clone()
        hy.hyena_intt(ctx, o)
        got = from_dev(o).reshape(batch, pl.tiles, lay.Co, 2, L, N)
        for b in range(batch):
            assert np.array_equal(got[b], want[b]), (sid, info, b)
        ran += 1
    assert ran >= (4 if lay.depthwise else len(streamed))


@pytest.mark.parametrize("N,L,bits", [(2048, 2, 30), (2048, 1, 31), (4096, 2, 30), (8192, 3, 31), (8192, 2, 30),
                                      (16384, 2, 31)])
def test_every_ntt_schedule_matches_oracle(dev, N, L, bits):
    ctx = ctx_for(N, L, bits)
    rng = np.random.default_rng(N + bits)
    a = rand_res(rng, (2, L, N), ctx.primes)
    want = [orc.ntt(a[1, i], q, ctx.psi[i]) for i, q in enumerate(ctx.primes)]
    for sid in hy.hyena_ntt_schedules(N):
        d = to_dev(a)
        hy.hyena_ntt_sched(ctx, d, False, sid)
        got = from_dev(d)
        for i in range(L):
            assert np.array_equal(got[1, i], want[i]), (sid, i)
        hy.hyena_ntt_sched(ctx, d, True, sid)
        assert np.array_equal(from_dev(d), a), sid


@pytest.mark.parametrize("N,L,bits", [(2048, 2, 31), (8192, 2, 31), (4096, 2, 30)])
def test_every_ntt_schedule_on_extreme_residues(dev, N, L, bits):
    """Inputs that keep the butterflies' intermediate values at the top of
    their ranges (every residue q - 1, alternating 0 and q - 1, q - 1 at one
    end, zero), forward and inverse, through every schedule, against the
    oracle's transforms."""
    ctx = ctx_for(N, L, bits)
    pats = []
    for kind in range(4):
        a = np.zeros((L, N), dtype=np.uint64)
        for i, q in enumerate(ctx.primes):
            if kind == 0:
                a[i] = q - 1
            elif kind == 1:
                a[i, 1::2] = q - 1
            elif kind == 2:
                a[i, -1] = q - 1
        pats.append(a)
    a = np.stack(pats)                                   # [4][L][N]
    want_f = np.stack([[orc.ntt(a[k, i], q, ctx.psi[i]) for i, q in enumerate(ctx.primes)] for k in range(4)])
    want_i = np.stack([[orc.intt(a[k, i], q, ctx.psi[i]) for i, q in enumerate(ctx.primes)] for k in range(4)])
    for sid in hy.hyena_ntt_schedules(N):
        d = to_dev(a)
        hy.hyena_ntt_sched(ctx, d, False, sid)
        assert np.array_equal(from_dev(d), want_f), ("forward", sid)
        d = to_dev(a)
        hy.hyena_ntt_sched(ctx, d, True, sid)
        assert np.array_equal(from_dev(d), want_i), ("inverse", sid)


@pytest.mark.parametrize("N,L,bits", [(8192, 3, 31), (4096, 2, 30), (16384, 2, 31), (2048, 2, 31)])
def test_ntt_schedules_many_polys(dev, N, L, bits):
    """Every schedule on more limb-polynomials than a persistent grid holds
    (so persistent blocks loop and prefetch), against the default schedule
    and, on sampled polynomials, against the oracle."""
    ctx = ctx_for(N, L, bits)
    rng = np.random.default_rng(N * 7 + bits)
    P = 2600 // L + 1                      # > 4 blocks x 256 CUs limb-polynomials
    a = rand_res(rng, (P, L, N), ctx.primes)
    d = to_dev(a)
    hy.hyena_intt(ctx, d)
    want_inv = from_dev(d)
    d = to_dev(a)
    hy.hyena_ntt(ctx, d)
    want_fwd = from_dev(d)
    for pi in (0, P // 2, P - 1):          # the default schedule against the oracle
        for i, q in enumerate(ctx.primes):
            assert np.array_equal(want_inv[pi, i], orc.intt(a[pi, i], q, ctx.psi[i])), (pi, i)
    for sid in hy.hyena_ntt_schedules(N):
        d = to_dev(a)
        hy.hyena_ntt_sched(ctx, d, True, sid)
        assert np.array_equal(from_dev(d), want_inv), ("inverse", sid)
        d = to_dev(a)
        hy.hyena_ntt_sched(ctx, d, False, sid)
        assert np.array_equal(from_dev(d), want_fwd), ("forward", sid)


def test_misaligned_device_arrays_rejected(dev):
    """16-byte alignment is checked on the host before any launch (EINVAL)."""
    import torch
    N, L = 8192, 3
    ctx = ctx_for(N, L, 31)
    d = hy.hyena_conv_plan(ctx, 16, 16, 16, 16, 3, c_n=1, flags=hy.HYENA_FUSE_WHT)
    ct = torch.zeros(d.n_in * 2 * L * N + 4, dtype=torch.int32, device="cuda")
    w = torch.zeros(hy.wntt_words(ctx, d) + 4, dtype=torch.int32, device="cuda")
    out = torch.zeros(d.n_out * 2 * L * N + 4, dtype=torch.int32, device="cuda")
    n_ct, n_w, n_out = ct.numel() - 4, w.numel() - 4, out.numel() - 4
    with pytest.raises(hy.HyenaError, match="aligned"):
        hy.hyena_conv(ctx, d, ct[1:1 + n_ct], w[:n_w], out[:n_out])
    with pytest.raises(hy.HyenaError, match="aligned"):
        hy.hyena_conv(ctx, d, ct[:n_ct], w[:n_w], out[1:1 + n_out])
    with pytest.raises(hy.HyenaError, match="aligned"):
        hy.hyena_ntt(ctx, ct[1:1 + 2 * L * N])
    with pytest.raises(hy.HyenaError, match="aligned"):
        hy.hyena_encode_weights(ctx, d, torch.zeros(16 * 16 * 9, dtype=torch.int8, device="cuda"), w[1:1 + n_w])
    torch.cuda.synchronize()


# ---------------------------------------------------------------- direct (coefficient domain)

DIRECT_CASES = [
    # (name, (N, L, bits), layer, batch)
    ("depthwise", (8192, 3, 31), wl.Layer("t", 28, 28, 32, 32, 3, depthwise=True), 2),
    ("depthwise_30bit", (4096, 2, 30), wl.Layer("t", 14, 14, 64, 64, 3, depthwise=True), 1),
    ("small_std", (4096, 2, 30), wl.Layer("t", 16, 16, 16, 16, 3), 1),
    ("tiles_halo", (4096, 2, 30), wl.Layer("t", 70, 70, 3, 8, 3), 1),
    ("short_group", (4096, 2, 30), wl.Layer("t", 12, 12, 37, 8, 3), 3),
    ("pointwise", (8192, 3, 31), wl.Layer("t", 14, 14, 64, 40, 1), 1),
]


@pytest.mark.parametrize("name,params,lay,batch", DIRECT_CASES, ids=[c[0] for c in DIRECT_CASES])
def test_conv_direct_matches_oracle(dev, name, params, lay, batch):
    """The coefficient-domain direct convolution equals the oracle's sparse-tap
    schoolbook products on every coefficient of every output, part and limb."""
    import torch
    say(f"direct {name}")
    ctx = ctx_for(*params)
    N, L = params[0], params[1]
    d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, depthwise=lay.depthwise, batch=batch)
    pl = orc.plan(N, lay.H, lay.W, lay.Ci, lay.Co, lay.k, lay.depthwise)
    rng = np.random.default_rng(31 + len(name))
    ct = rand_res(rng, (batch, pl.tiles, pl.n_groups, 2, L, N), ctx.primes)
    w = wl.weights(3100 + len(name), lay)
    d_out = torch.empty(batch * pl.tiles * lay.Co * 2 * L * N, dtype=torch.int32, device="cuda")
    hy.hyena_conv_direct(ctx, d, to_dev(ct), torch.from_numpy(w).cuda(), d_out)
    got = from_dev(d_out).reshape(batch, pl.tiles, lay.Co, 2, L, N)
    for b in range(batch):
        want = orc.conv_products(pl, ct[b], w, ctx.primes).reshape(pl.tiles, lay.Co, 2, L, N)
        assert np.array_equal(got[b], want), (name, b)


def test_conv_direct_equals_ntt_path(dev):
    """Direct result == inverse NTT of the NTT-domain product with the Walsh
    packing (c_n = 2, fused), on a layer with row tiles and a short group."""
    import torch
    ctx = ctx_for(8192, 3, 31)
    N, L = 8192, 3
    lay = wl.Layer("t", 28, 28, 40, 24, 3)
    d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, c_n=2, flags=hy.HYENA_FUSE_WHT, batch=2)
    pl = orc.plan(N, lay.H, lay.W, lay.Ci, lay.Co, lay.k)
    rng = np.random.default_rng(77)
    ct = rand_res(rng, (2, pl.tiles, pl.n_groups, 2, L, N), ctx.primes)
    w = wl.weights(7700, lay)
    d_w = torch.from_numpy(w).cuda()
    n_out = 2 * pl.tiles * lay.Co * 2 * L * N
    direct = torch.empty(n_out, dtype=torch.int32, device="cuda")
    hy.hyena_conv_direct(ctx, d, to_dev(ct), d_w, direct)
    d_ct = to_dev(ct)
    d_wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device="cuda")
    hy.hyena_encode_weights(ctx, d, d_w, d_wn)
    via_ntt = torch.empty(n_out, dtype=torch.int32, device="cuda")
    hy.hyena_ntt(ctx, d_ct)
    hy.hyena_conv(ctx, d, d_ct, d_wn, via_ntt)
    hy.hyena_intt(ctx, via_ntt)
    assert torch.equal(direct, via_ntt)


def test_conv_direct_rejects_overlap_and_unplanned(dev):
    import torch
    ctx = ctx_for(4096, 2, 30)
    lay = wl.Layer("t", 16, 16, 16, 16, 3)
    d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k)
    n_in = d.n_in * 2 * 2 * 4096
    n_out = d.n_out * 2 * 2 * 4096
    buf = torch.zeros(n_in + n_out, dtype=torch.int32, device="cuda")
    w = torch.zeros(16 * 16 * 9, dtype=torch.int8, device="cuda")
    with pytest.raises(hy.HyenaError):       # output overlapping the input
        hy.hyena_conv_direct(ctx, d, buf[:n_in], w, buf[n_in // 2:n_in // 2 + n_out])
    bad = hy.ConvDesc()
    with pytest.raises(hy.HyenaError):       # descriptor never planned
        hy.hyena_conv_direct(ctx, bad, buf[:n_in], w, buf[n_in:])


# ---------------------------------------------------------------- weights synthesized in the MAC

SYNTH_CASES = [
    # id, (N, L, bits), layer, c_n, batch, fused, ci_req
    ("ci1_k3", (8192, 3, 31), wl.Layer("t", 64, 64, 3, 20, 3), 1, 1, True, 0),          # 9 taps, 3 groups
    ("ci2_k3_cn4", (8192, 3, 31), wl.Layer("t", 56, 56, 64, 64, 3), 4, 2, True, 0),     # 18 taps, 32 groups
    ("rowtiles_cn2", (4096, 2, 30), wl.Layer("t", 70, 70, 3, 8, 3), 2, 3, True, 0),     # 2 row tiles, batch 3
    ("k1_ci16_cn8", (8192, 3, 31), wl.Layer("t", 14, 14, 64, 40, 1), 8, 1, True, 16),   # 1x1, 16 taps, 4 groups
    ("unfused_cn4", (8192, 3, 31), wl.Layer("t", 28, 28, 10, 16, 3), 4, 2, False, 2),   # Walsh components out
    ("short_group", (8192, 3, 31), wl.Layer("t", 20, 20, 7, 12, 1), 1, 5, True, 4),     # ragged last group
]


def _synth_setup(ctx, lay, c_n, batch, fuse, ci_req, seed):
    import torch
    N, L = ctx.N, ctx.L
    flags = hy.HYENA_FUSE_WHT if fuse else 0
    d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, c_n=c_n, flags=flags, batch=batch,
                           ci_req=ci_req)
    pl = orc.plan(N, lay.H, lay.W, lay.Ci, lay.Co, lay.k, False, ci_req or None)
    rng = np.random.default_rng(seed)
    ct = rand_res(rng, (batch, pl.tiles, pl.n_groups, 2, L, N), ctx.primes)
    w = wl.weights(seed, lay)
    d_w = torch.from_numpy(w).cuda()
    d_wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device="cuda")
    hy.hyena_encode_weights(ctx, d, d_w, d_wn)
    d_taps = torch.full((hy.synth_taps_words(d),), 12345, dtype=torch.int32, device="cuda")
    hy.hyena_synth_taps(ctx, d, d_w, d_taps)
    d_ct = to_dev(ct)
    hy.hyena_ntt(ctx, d_ct)
    return d, pl, ct, w, d_wn, d_taps, d_ct


@pytest.mark.parametrize("c_n", [1, 2, 4, 64])
def test_synth_taps_are_the_walsh_weights(dev, c_n):
    """The integer-tap table equals the oracle's Walsh weights (Eq. (hadamard2)
    generalised) arranged per output, input group and tap, zero past the last
    input channel and in the padding."""
    import torch
    say(f"synth taps c_n={c_n}")
    ctx = ctx_for(8192, 3, 31)
    lay = wl.Layer("t", 56, 56, 5, 64, 3)                       # ci = 2: 3 groups, the last one short
    d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, c_n=c_n)
    w = np.random.default_rng(c_n).integers(-128, 128, size=(64, 5, 3, 3)).astype(np.int8)
    d_taps = torch.full((hy.synth_taps_words(d),), 7, dtype=torch.int32, device="cuda")
    hy.hyena_synth_taps(ctx, d, torch.from_numpy(w).cuda(), d_taps)
    torch.cuda.synchronize()
    got = d_taps.cpu().numpy().reshape(64, d.w_groups, -1)
    gw = orc.walsh_weights(w, c_n)                              # [Co][Ci][3][3]
    T = d.ci * 9
    want = np.zeros_like(got)
    for g in range(d.w_groups):
        chans = gw[:, g * d.ci:(g + 1) * d.ci].reshape(64, -1)  # taps c' k^2 + di k + dj
        want[:, g, :chans.shape[1]] = chans
    assert got.shape[2] == (T + 3) // 4 * 4
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name,params,lay,c_n,batch,fuse,ci_req", SYNTH_CASES, ids=[c[0] for c in SYNTH_CASES])
def test_conv_synth_equals_streamed_weights(dev, name, params, lay, c_n, batch, fuse, ci_req):
    """hyena_conv_synth (weight words synthesized in the multiply-accumulate
    from the integer taps) against hyena_conv with the encoded weights, on every
    output word, by its default schedule and by every synthesizing schedule
    that fits the layer; the first case also against the oracle."""
    import torch
    say(f"conv synth {name}")
    ctx = ctx_for(*params)
    N, L = ctx.N, ctx.L
    d, pl, ct, w, d_wn, d_taps, d_ct = _synth_setup(ctx, lay, c_n, batch, fuse, ci_req, 7000 + len(name))
    n_out = batch * pl.tiles * lay.Co * 2 * L * N
    ref = torch.empty(n_out, dtype=torch.int32, device="cuda")
    hy.hyena_conv(ctx, d, d_ct, d_wn, ref)
    out = torch.full((n_out,), -1, dtype=torch.int32, device="cuda")
    hy.hyena_conv_synth(ctx, d, d_ct, d_taps, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref), int((out != ref).sum())
    T = d.ci * d.k * d.k
    tried = 0
    for sid in range(len(hy.hyena_conv_schedules())):
        tm = hy.hyena_conv_schedule_taps(sid)
        if tm == 0 or tm < T:
            continue
        out.fill_(-1)
        hy.hyena_conv_tiled(ctx, d, d_ct, d_taps, out, sid)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (sid, int((out != ref).sum()))
        tried += 1
    assert tried >= 2
    if name == "ci1_k3":
        hy.hyena_intt(ctx, out)
        got = from_dev(out).reshape(batch, pl.tiles, lay.Co, 2, L, N)
        want = orc.conv_products(pl, ct[0], w, ctx.primes).reshape(pl.tiles, lay.Co, 2, L, N)
        assert np.array_equal(got[0], want)


def test_conv_synth_refusals(dev):
    import torch
    ctx = ctx_for(8192, 3, 31)
    big = hy.hyena_conv_plan(ctx, 14, 14, 64, 32, 3)             # ci = 32: 288 taps per word
    dw = hy.hyena_conv_plan(ctx, 14, 14, 32, 32, 3, depthwise=True)
    buf = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
    for d, code in ((big, hy.HYENA_EUNSUPPORTED), (dw, hy.HYENA_EUNSUPPORTED)):
        with pytest.raises(hy.HyenaError) as e:
            hy.hyena_conv_synth(ctx, d, buf, buf, buf)
        assert e.value.code == code
    # a streaming schedule cannot run on taps alone, nor a synthesizing one on a 288-tap layer
    sid = next(s for s in range(len(hy.hyena_conv_schedules())) if hy.hyena_conv_schedule_taps(s) == 18)
    with pytest.raises(hy.HyenaError):
        hy.hyena_conv_tiled(ctx, big, buf, buf, buf, sid)
