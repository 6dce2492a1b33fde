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
