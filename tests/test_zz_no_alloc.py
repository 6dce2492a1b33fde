"""hyena_decrypt_device_noalloc (the decryption that uses the library's fixed
device workspace instead of a caller-allocated one) against
hyena_decrypt_device with a caller workspace: bit-equal messages on two calls
in a row, the second smaller than the first, and a clear refusal of a call
above the workspace's size. Runs alone in a fresh process or after the other
GPU tests."""
import sys

import numpy as np
import pytest

import paper_2311_12519_amd as hy

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _encrypted(ctx, d_s_hat, n, seed):
    import torch
    rng = np.random.default_rng(seed)
    t = 1 << 20
    msg = rng.integers(-t // 2 + 1, t // 2 + 1, size=(n, ctx.N)).astype(np.int32)
    d_msg = torch.from_numpy(msg).cuda()
    d_ct = torch.empty(n * 2 * ctx.L * ctx.N, dtype=torch.int32, device="cuda")
    d_work = torch.empty(n * ctx.L * ctx.N, dtype=torch.int32, device="cuda")
    hy.hyena_encrypt_device(ctx, d_s_hat, d_msg, seed, d_work, d_ct)
    return msg, d_ct


def _arbitrary(ctx, n, seed):
    """Uniform residues per limb: decryption's rounding sees every fraction."""
    import torch
    rng = np.random.default_rng(seed)
    ct = np.empty((n, 2, ctx.L, ctx.N), dtype=np.uint32)
    for i, q in enumerate(ctx.primes):
        ct[:, :, i, :] = rng.integers(0, q, size=(n, 2, ctx.N))
    return torch.from_numpy(ct.view(np.int32).reshape(-1)).cuda()


def _with_workspace(ctx, d_s_hat, d_ct):
    import torch
    n = d_ct.numel() // (2 * ctx.L * ctx.N)
    d_work = torch.empty(n * ctx.L * ctx.N, dtype=torch.int32, device="cuda")
    d_msg = torch.full((n * ctx.N,), 7, dtype=torch.int32, device="cuda")
    hy.hyena_decrypt_device(ctx, d_s_hat, d_ct, d_work, d_msg)
    torch.cuda.synchronize()
    return d_msg.cpu().numpy()


def _no_alloc(ctx, d_s_hat, d_ct):
    import torch
    n = d_ct.numel() // (2 * ctx.L * ctx.N)
    d_msg = torch.full((n * ctx.N,), -7, dtype=torch.int32, device="cuda")
    hy.hyena_decrypt_device_noalloc(ctx, d_s_hat, d_ct, d_msg)
    torch.cuda.synchronize()
    return d_msg.cpu().numpy()


@pytest.mark.parametrize("N,L,flags", [(8192, 3, 0), (4096, 2, hy.HYENA_PRIMES_30BIT)])
def test_noalloc_decrypt_equals_workspace_decrypt(N, L, flags):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say(f"noalloc decrypt N={N} L={L}")
    ctx = hy.hyena_create(N, L, flags=flags)
    sk = hy.hyena_keygen(ctx, 5 + N)
    d_s_hat = torch.empty(L * N, dtype=torch.int32, device="cuda")
    hy.hyena_secret_prepare(ctx, torch.from_numpy(sk).cuda(), d_s_hat)
    n_max = hy.HYENA_NOALLOC_SCRATCH_WORDS // (L * N)

    # first call: the largest batch the workspace holds, fresh encryptions
    msg, d_ct = _encrypted(ctx, d_s_hat, n_max, 11)
    got = _no_alloc(ctx, d_s_hat, d_ct)
    assert np.array_equal(got, _with_workspace(ctx, d_s_hat, d_ct))
    assert np.array_equal(got.reshape(n_max, N), msg)

    # second call, smaller, on arbitrary residues: the workspace holds the
    # first call's values; every rounding decision must still match
    d_ct2 = _arbitrary(ctx, 5, 12)
    got2 = _no_alloc(ctx, d_s_hat, d_ct2)
    assert np.array_equal(got2, _with_workspace(ctx, d_s_hat, d_ct2))

    # one ciphertext more than the workspace holds is refused, nothing written
    d_big = torch.zeros((n_max + 1) * 2 * L * N, dtype=torch.int32, device="cuda")
    d_msg = torch.full(((n_max + 1) * N,), 3, dtype=torch.int32, device="cuda")
    with pytest.raises(hy.HyenaError) as e:
        hy.hyena_decrypt_device_noalloc(ctx, d_s_hat, d_big, d_msg)
    assert e.value.code == hy.HYENA_EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((d_msg == 3).all())
    # n = 0 does nothing
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    hy.hyena_decrypt_device_noalloc(ctx, d_s_hat, empty, empty)
