"""GPU tests of the batched path (segmented NTTs, persistent multiply-
accumulate over uneven layers, hipGraph replay, autotuner): outputs equal the
oracle's on every coefficient, for every flag combination and every replay."""
import os

import numpy as np
import pytest

import oracle as orc
import paper_2311_12519_amd as hy
import workloads as wl

pytestmark = pytest.mark.gpu

LAYERS = [
    # uneven input-ciphertext counts, tiles, Walsh groups and a depthwise layer
    (wl.Layer("a", 70, 70, 3, 8, 3), 1),     # 2 row tiles, 3 groups
    (wl.Layer("b", 28, 28, 40, 24, 3), 2),   # 5 groups (9 channels per ciphertext)
    (wl.Layer("c", 14, 14, 64, 32, 3), 32),  # c_n wider than the fused epilogue
    (wl.Layer("d", 14, 14, 32, 32, 3, depthwise=True), 1),
    (wl.Layer("e", 14, 14, 16, 16, 1), 4),   # 1x1
]
N, L, BATCH = 8192, 3, 2


@pytest.fixture(scope="module")
def setup():
    import torch
    ctx = hy.hyena_create(N, L)
    rng = np.random.default_rng(5)
    items = []
    for i, (lay, c_n) in enumerate(LAYERS):
        d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, depthwise=lay.depthwise, c_n=c_n,
                               flags=hy.HYENA_FUSE_WHT, batch=BATCH)
        pl = orc.plan(N, lay.H, lay.W, lay.Ci, lay.Co, lay.k, lay.depthwise)
        ct = np.empty((BATCH, pl.tiles, pl.n_groups, 2, L, N), dtype=np.uint32)
        for li, q in enumerate(ctx.primes):
            ct[..., li, :] = rng.integers(0, q, size=ct[..., li, :].shape)
        w = wl.weights(300 + i, lay)
        d_wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device="cuda")
        hy.hyena_encode_weights(ctx, d, torch.from_numpy(w).cuda(), d_wn)
        want = [orc.conv_products(pl, ct[b], w, ctx.primes).reshape(pl.tiles, lay.Co, 2, L, N)
                for b in range(BATCH)]
        items.append(dict(d=d, pl=pl, ct=ct, w=w, d_wn=d_wn, want=want))
    return ctx, items


def _buffers(items):
    import torch
    bufs = []
    for it in items:
        d_ct = torch.from_numpy(it["ct"].reshape(-1).view(np.int32)).cuda()
        d_out = torch.empty(BATCH * it["pl"].tiles * it["d"].Co * 2 * L * N, dtype=torch.int32, device="cuda")
        bufs.append((d_ct, d_out))
    return bufs


def _check(items, bufs, tag):
    import torch
    torch.cuda.synchronize()
    for i, (it, (d_ct, d_out)) in enumerate(zip(items, bufs)):
        got = d_out.cpu().numpy().view(np.uint32).reshape(BATCH, it["pl"].tiles, it["d"].Co, 2, L, N)
        for b in range(BATCH):
            assert np.array_equal(got[b], it["want"][b]), (tag, i, b)


@pytest.mark.parametrize("flags", [0, hy.HYENA_BATCH_PERSISTENT, hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH,
                                   hy.HYENA_BATCH_GRAPH,
                                   hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH | hy.HYENA_BATCH_TIMING,
                                   hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_TIMING])
def test_batch_matches_oracle(dev, setup, flags):
    import torch
    ctx, items = setup
    bufs = _buffers(items)
    pristine = [d_ct.clone() for d_ct, _ in bufs]
    b = hy.hyena_batch_create(ctx, [(it["d"], d_ct, it["d_wn"], d_out) for it, (d_ct, d_out) in zip(items, bufs)],
                              flags)
    for rep in range(3):
        for (d_ct, d_out), p in zip(bufs, pristine):
            d_ct.copy_(p)
            d_out.fill_(0)
        torch.cuda.synchronize()
        hy.hyena_batch_run(b)
        if flags & hy.HYENA_BATCH_TIMING:
            ms = hy.hyena_batch_phase_ms(b)
            assert all(m > 0 for m in ms)
        _check(items, bufs, (flags, rep))
    info = hy.hyena_batch_info(b)
    if flags & hy.HYENA_BATCH_PERSISTENT:
        assert info["persistent_launches"] >= 1
    hy.hyena_batch_destroy(b)


def test_batch_tuned_uses_cache(dev, setup, tmp_path, monkeypatch):
    import torch
    ctx, items = setup
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HYENA_TUNE_CACHE", str(cache))
    bufs = _buffers(items)
    pristine = [d_ct.clone() for d_ct, _ in bufs]
    flags = hy.HYENA_BATCH_TUNE | hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH
    layers = [(it["d"], d_ct, it["d_wn"], d_out) for it, (d_ct, d_out) in zip(items, bufs)]
    b = hy.hyena_batch_create(ctx, layers, flags)
    info1 = hy.hyena_batch_info(b)
    # tuning timed on the buffers but left the inputs untouched
    for (d_ct, _), p in zip(bufs, pristine):
        assert torch.equal(d_ct, p)
    hy.hyena_batch_run(b)
    _check(items, bufs, "tuned")
    text = cache.read_text()
    assert "|mac|" in text and "|ntt|" in text
    b2 = hy.hyena_batch_create(ctx, layers, flags)   # second build reads the cache
    assert hy.hyena_batch_info(b2)["mac_sched"] == info1["mac_sched"]
    for (d_ct, d_out), p in zip(bufs, pristine):
        d_ct.copy_(p)
        d_out.fill_(0)
    hy.hyena_batch_run(b2)
    _check(items, bufs, "cached")


def test_batch_every_ntt_schedule_from_cache(dev, setup, tmp_path, monkeypatch):
    """Segmented NTT launches over all layers with every schedule, forced
    through the tuning cache (persistent inverse schedules cross segment
    boundaries inside one block's loop)."""
    import torch
    ctx, items = setup
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HYENA_TUNE_CACHE", str(cache))
    bufs = _buffers(items)
    pristine = [d_ct.clone() for d_ct, _ in bufs]
    flags = hy.HYENA_BATCH_TUNE | hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH
    layers = [(it["d"], d_ct, it["d_wn"], d_out) for it, (d_ct, d_out) in zip(items, bufs)]
    hy.hyena_batch_destroy(hy.hyena_batch_create(ctx, layers, flags))   # writes the cache
    lines = cache.read_text().splitlines()
    assert any("|ntt|" in ln for ln in lines)
    for sid in hy.hyena_ntt_schedules(N):
        text = "\n".join(ln.split("\t")[0] + "\t" + str(sid) if "|ntt|" in ln else ln for ln in lines) + "\n"
        cache.write_text(text)
        b = hy.hyena_batch_create(ctx, layers, flags)
        info = hy.hyena_batch_info(b)
        assert info["ntt_fwd"] == sid and info["ntt_inv"] == sid
        for (d_ct, d_out), p in zip(bufs, pristine):
            d_ct.copy_(p)
            d_out.fill_(0)
        hy.hyena_batch_run(b)
        _check(items, bufs, ("ntt schedule", sid))
        hy.hyena_batch_destroy(b)


@pytest.mark.parametrize("solo", [0, 1])
def test_batch_mac_launch_form_from_cache(dev, setup, tmp_path, monkeypatch, solo):
    """Both launch forms of the tuned multiply-accumulate phase (one persistent
    launch, or one launch per layer), forced through the tuning cache."""
    import torch
    ctx, items = setup
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HYENA_TUNE_CACHE", str(cache))
    bufs = _buffers(items)
    pristine = [d_ct.clone() for d_ct, _ in bufs]
    flags = hy.HYENA_BATCH_TUNE | hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH
    layers = [(it["d"], d_ct, it["d_wn"], d_out) for it, (d_ct, d_out) in zip(items, bufs)]
    hy.hyena_batch_destroy(hy.hyena_batch_create(ctx, layers, flags))   # writes the cache

    def rewrite(tag, value):
        lines = cache.read_text().splitlines()
        assert any(tag in ln for ln in lines), tag
        cache.write_text("\n".join(ln.split("\t")[0] + "\t" + str(value) if tag in ln else ln
                                   for ln in lines) + "\n")

    # an LDS schedule for every layer that admits one (the library re-tunes the
    # others), so that a persistent group exists and its launch form is tuned
    lds = [sid for sid, info in enumerate(hy.hyena_conv_schedules()) if info[0]][0]
    rewrite("|mac|", lds)
    hy.hyena_batch_destroy(hy.hyena_batch_create(ctx, layers, flags))   # tunes and caches the form
    rewrite("|macphase|", solo)
    b = hy.hyena_batch_create(ctx, layers, flags)
    info = hy.hyena_batch_info(b)
    assert (info["persistent_launches"] == 0) == bool(solo)
    for rep in range(2):
        for (d_ct, d_out), p in zip(bufs, pristine):
            d_ct.copy_(p)
            d_out.fill_(0)
        hy.hyena_batch_run(b)
        _check(items, bufs, ("launch form", solo, rep))
    hy.hyena_batch_destroy(b)


def test_vgg_full_size_tuned_batch_sampled(dev, tmp_path, monkeypatch):
    """Three VGG-16 layers at their full size (conv1_2: 7 row tiles, 64 input
    groups; conv4_2: 57 groups; conv5_1: 16 groups) for 8 images at N = 8192,
    L = 3, in the launch configuration the benchmark times: one tuned batch
    with the persistent multiply-accumulate and hipGraph replay. Sampled output
    ciphertexts equal the oracle's on every coefficient, after the first run
    and after a replay of the captured graph."""
    import torch
    monkeypatch.setenv("HYENA_TUNE_CACHE", str(tmp_path / "tune.txt"))
    n, l_, images = 8192, 3, 8
    ctx = hy.hyena_create(n, l_)
    by_name = {lay.name: lay for lay in wl.vgg16_layers()}
    gen = torch.Generator(device="cuda")
    items = []
    for i, name in enumerate(["conv1_2", "conv4_2", "conv5_1"]):
        lay = by_name[name]
        d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, c_n=1, flags=hy.HYENA_FUSE_WHT,
                               batch=images)
        pl = orc.plan(n, lay.H, lay.W, lay.Ci, lay.Co, lay.k)
        ct0 = torch.empty((images, pl.tiles, pl.n_groups, 2, l_, n), dtype=torch.int32, device="cuda")
        gen.manual_seed(700 + i)
        for li, q in enumerate(ctx.primes):
            ct0[..., li, :] = torch.randint(0, q, ct0[..., li, :].shape, generator=gen, device="cuda",
                                            dtype=torch.int64).to(torch.int32)
        w = wl.weights(7000 + i, lay)
        d_wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device="cuda")
        hy.hyena_encode_weights(ctx, d, torch.from_numpy(w).cuda(), d_wn)
        d_out = torch.empty(images * pl.tiles * lay.Co * 2 * l_ * n, dtype=torch.int32, device="cuda")
        # (image, tile, output channel): first, last and one in between
        sel = [(0, 0, 0), (3, pl.tiles // 2, lay.Co // 2 + 1), (images - 1, pl.tiles - 1, lay.Co - 1)]
        items.append(dict(d=d, pl=pl, ct0=ct0, d_ct=ct0.clone(), w=w, d_wn=d_wn, d_out=d_out, sel=sel))
    flags = hy.HYENA_BATCH_TUNE | hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH
    b = hy.hyena_batch_create(ctx, [(it["d"], it["d_ct"], it["d_wn"], it["d_out"]) for it in items], flags)
    assert hy.hyena_batch_info(b)["layers"] == 3
    want = []
    for it in items:
        pl = it["pl"]
        w_it = []
        for img, tau, o in it["sel"]:
            ct_img = it["ct0"][img].cpu().numpy().view(np.uint32)
            w_it.append(orc.conv_products(pl, ct_img, it["w"], ctx.primes, outputs=[(tau, o)])[0])
        want.append(w_it)
    for rep in range(2):
        for it in items:
            it["d_ct"].copy_(it["ct0"])
        torch.cuda.synchronize()
        hy.hyena_batch_run(b)
        torch.cuda.synchronize()
        for it, w_it in zip(items, want):
            pl = it["pl"]
            got = it["d_out"].view(images, pl.tiles, it["d"].Co, 2, l_, n)
            for (img, tau, o), wv in zip(it["sel"], w_it):
                g = got[img, tau, o].cpu().numpy().view(np.uint32)
                assert np.array_equal(g, wv), (rep, it["d"].Co, img, tau, o)
    hy.hyena_batch_destroy(b)


# ------------------------------------------------- weights synthesized in the MAC

@pytest.mark.parametrize("flags", [hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH,
                                   hy.HYENA_BATCH_TUNE | hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH, 0])
def test_batch_with_integer_taps_matches_oracle(dev, setup, flags, tmp_path, monkeypatch):
    """Layers given as integer taps only (no encoded weights: their words are
    synthesized in the multiply-accumulate), next to layers with encoded
    weights and layers with both (the autotuner then also times the
    synthesizing schedules): every output equals the oracle's, on every
    replay."""
    import torch
    monkeypatch.setenv("HYENA_TUNE_CACHE", str(tmp_path / "tune.txt"))
    ctx, items = setup
    bufs = _buffers(items)
    pristine = [d_ct.clone() for d_ct, _ in bufs]
    layers = []
    for i, (it, (d_ct, d_out)) in enumerate(zip(items, bufs)):
        d = it["d"]
        T = d.ci * d.k * d.k
        if d.depthwise or T > 18:
            layers.append((d, d_ct, it["d_wn"], d_out))
            continue
        d_taps = torch.empty(hy.synth_taps_words(d), dtype=torch.int32, device="cuda")
        hy.hyena_synth_taps(ctx, d, torch.from_numpy(it["w"]).cuda(), d_taps)
        # layer "a": taps only; layer "e": both forms
        layers.append((d, d_ct, None if i == 0 else it["d_wn"], d_out, d_taps))
    assert layers[0][2] is None and len(layers[4]) == 5
    b = hy.hyena_batch_create(ctx, layers, flags)
    info = hy.hyena_batch_info(b)
    assert hy.hyena_conv_schedule_taps(info["mac_sched"][0]) >= 9   # taps only: a synthesizing schedule
    for rep in range(3):
        for (d_ct, d_out), p in zip(bufs, pristine):
            d_ct.copy_(p)
            d_out.fill_(0)
        torch.cuda.synchronize()
        hy.hyena_batch_run(b)
        _check(items, bufs, ("taps", flags, rep))
    hy.hyena_batch_destroy(b)


def test_vgg_conv2_2_synthesized_in_the_batch_full_size(dev):
    """VGG-16 conv2_2 (112x112, 128 -> 128, 2 row tiles, 128 input groups, 9
    taps per weight word) for 8 images at N = 8192, L = 3, its weights given
    only as integer taps: the tuned persistent batch synthesizes every weight
    word in the multiply-accumulate. All outputs equal those of the same batch
    with encoded weights; sampled output ciphertexts equal the oracle's."""
    import torch
    lay = wl.vgg16_layers()[3]
    assert (lay.H, lay.Ci, lay.Co) == (112, 128, 128)
    ctx = hy.hyena_create(N, L)
    images = 8
    d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, 3, flags=hy.HYENA_FUSE_WHT, batch=images)
    pl = orc.plan(N, lay.H, lay.W, lay.Ci, lay.Co, 3)
    assert (pl.tiles, pl.n_groups, pl.ci) == (2, 128, 1)
    w = wl.weights(4003, lay)
    d_w = torch.from_numpy(w).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(44)
    ct0 = torch.empty((images, pl.tiles, pl.n_groups, 2, L, N), dtype=torch.int32, device="cuda")
    for i, q in enumerate(ctx.primes):
        ct0[..., i, :] = torch.randint(0, q, ct0[..., i, :].shape, generator=g, device="cuda",
                                       dtype=torch.int64).to(torch.int32)
    d_taps = torch.empty(hy.synth_taps_words(d), dtype=torch.int32, device="cuda")
    hy.hyena_synth_taps(ctx, d, d_w, d_taps)
    d_wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device="cuda")
    hy.hyena_encode_weights(ctx, d, d_w, d_wn)
    outs = []
    for form in ("taps", "encoded"):
        ct = ct0.clone().reshape(-1)
        out = torch.empty(images * pl.tiles * lay.Co * 2 * L * N, dtype=torch.int32, device="cuda")
        io = (d, ct, None, out, d_taps) if form == "taps" else (d, ct, d_wn, out)
        b = hy.hyena_batch_create(ctx, [io], hy.HYENA_BATCH_TUNE | hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH)
        if form == "taps":
            assert hy.hyena_conv_schedule_taps(hy.hyena_batch_info(b)["mac_sched"][0]) >= 9
        ct.copy_(ct0.reshape(-1))
        hy.hyena_batch_run(b)
        torch.cuda.synchronize()
        outs.append(out)
        hy.hyena_batch_destroy(b)
        del ct
    assert torch.equal(outs[0], outs[1])
    got = outs[0].view(images, pl.tiles, lay.Co, 2, L, N)
    host_ct = ct0[5].cpu().numpy().view(np.uint32)
    sel = [(0, 0), (1, 77), (1, 127)]
    want = orc.conv_products(pl, host_ct, w, ctx.primes, outputs=sel)
    for u, (tau, o) in enumerate(sel):
        assert np.array_equal(got[5, tau, o].cpu().numpy().view(np.uint32), want[u]), (tau, o)
    hy.hyena_destroy(ctx)
