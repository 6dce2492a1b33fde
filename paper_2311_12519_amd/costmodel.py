"""Learned cost model for the parameters of a homomorphic convolution layer.

The paper chooses the encryption parameters by hand per layer (the ring degree
by input size, the moduli for noise and speed; "Optimal Parameter Selection",
"Evaluation Setup"). Here the choice is searched: for every layer the
candidates are (ring degree N, RNS limb count L, channels per ciphertext c_i,
Walsh group c_n) computed through the NTT path, plus, for layers with at most
DIRECT_MAX_TAPS taps per output, (N, L, c_i) computed by the coefficient-domain
direct convolution; all restricted to parameter sets that meet the 128-bit
security ceiling and whose worst-case noise still decrypts (the library's
planner refuses the rest). Timing every candidate is the exhaustive search; a small
FP32 MLP (8 -> 64 -> 64 -> 1, trained and evaluated by the library's own HIP
kernels) predicts the log time of a candidate from its features and picks the
argmin instead. The exhaustive table stays as the reference for the model's regret.

Training data are timings of random layer shapes (never the evaluated
network's own shapes), drawn by the same timer. Everything that touches the GPU
goes through the library's C ABI.

Run ``python -m paper_2311_12519_amd.costmodel`` for the MobileNetV1 report.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass

import numpy as np

from . import (HYENA_FUSE_WHT, HYENA_HOST_ONLY, HyenaError, hyena_conv, hyena_conv_direct, hyena_conv_plan,
               hyena_create, hyena_intt, hyena_mlp_adam, hyena_mlp_forward, hyena_mlp_loss_grad,
               hyena_mlp_params, hyena_mlp_workspace_floats, hyena_ntt)

RING_DEGREES = (4096, 8192, 16384)
SECURITY_LOGQ_128 = {4096: 109, 8192: 218, 16384: 438}   # ternary secret, 128-bit
MAX_MACS = 1 << 32          # candidates above this many coeff-MACs are not searched
MAX_BYTES = 1 << 30         # nor those whose weight and ciphertext buffers exceed 1 GiB
# the direct path is a candidate up to this many taps per output: 3x3 and 5x5
# depthwise layers and a first layer over 3 input channels; with 32 taps and
# more (pointwise layers over 32+ channels) the NTT path was faster wherever
# timed, and offering the direct path there only made the model err
DIRECT_MAX_TAPS = 27


@dataclass(frozen=True)
class Cand:
    N: int
    L: int
    ci: int
    c_n: int
    direct: bool = False     # coefficient-domain direct convolution instead of the NTT path


@dataclass(frozen=True)
class Shape:
    H: int
    W: int
    Ci: int
    Co: int
    k: int
    depthwise: bool


def _max_limbs(N: int) -> int:
    return SECURITY_LOGQ_128[N] // 31


_HOST_CTX = {}


def _host_ctx(N: int, L: int):
    key = (N, L)
    if key not in _HOST_CTX:
        _HOST_CTX[key] = hyena_create(N, L, flags=HYENA_HOST_ONLY)
    return _HOST_CTX[key]


def _plan(N, L, s: Shape, ci, c_n):
    return hyena_conv_plan(_host_ctx(N, L), s.H, s.W, s.Ci, s.Co, s.k, depthwise=s.depthwise, c_n=c_n,
                           ci_req=ci, flags=HYENA_FUSE_WHT)


def _sizes(d, N, L):
    macs = d.tiles * (1 if d.depthwise else d.n_groups) * d.Co * 2 * L * N
    w_bytes = d.Co * d.w_groups * L * N * 4
    io_bytes = (d.n_in + d.n_out) * 2 * L * N * 4
    return macs, w_bytes, io_bytes


def _taps(s: Shape) -> int:
    """Taps per output coefficient of the direct path."""
    return s.k * s.k * (1 if s.depthwise else s.Ci)


def candidates(s: Shape, max_extra_limbs: int = 2):
    """Valid (N, L, c_i, c_n) for a layer shape: secure, decryptable, bounded."""
    out = []
    for N in RING_DEGREES:
        # smallest L whose worst-case noise decrypts (planner check)
        lmin = None
        for L in range(1, _max_limbs(N) + 1):
            try:
                _plan(N, L, s, 0, 1)
                lmin = L
                break
            except HyenaError:
                continue
        if lmin is None:
            continue
        base = _plan(N, lmin, s, 0, 1)
        cmax = base.ci
        cis = sorted({c for c in [1 << i for i in range(12)] if c <= cmax} | {cmax}) if base.tiles == 1 else [1]
        for L in range(lmin, min(lmin + max_extra_limbs, _max_limbs(N)) + 1):
            for ci in cis:
                for c_n in (1, 2, 4):
                    if s.Co % c_n or (s.depthwise and ci % c_n):
                        continue
                    try:
                        d = _plan(N, L, s, ci, c_n)
                    except HyenaError:
                        continue
                    macs, wb, iob = _sizes(d, N, L)
                    if macs > MAX_MACS or wb + iob > MAX_BYTES:
                        continue
                    out.append(Cand(N, L, ci, c_n))
                    # the direct path ignores c_n; its time hardly depends on
                    # c_i (outputs dominate), so one candidate per (N, L): the
                    # widest channel partition
                    if (c_n == 1 and ci == cis[-1] and _taps(s) <= DIRECT_MAX_TAPS and N % 1024 == 0
                            and iob <= MAX_BYTES):
                        out.append(Cand(N, L, ci, 1, True))
    return out


def default_candidate(s: Shape):
    """The method without the model: N = 8192, the fewest limbs that decrypt,
    as many channels per ciphertext as fit, no Walsh grouping."""
    for L in range(1, _max_limbs(8192) + 1):
        try:
            d = _plan(8192, L, s, 0, 1)
            return Cand(8192, L, d.ci, 1)
        except HyenaError:
            continue
    return None


def features(s: Shape, c: Cand) -> np.ndarray:
    """log2 N, L, log2 c_i, log2 c_n, log2 of the input and output ciphertext
    counts, log2 of the multiply-adds (pointwise coeff-MACs on the NTT path,
    tap multiply-adds of every output coefficient on the direct path) and the
    path: 0 NTT (standard layer), 1 NTT (depthwise layer), 2 direct."""
    d = _plan(c.N, c.L, s, c.ci, c.c_n)
    macs, _, _ = _sizes(d, c.N, c.L)
    if c.direct:
        macs = d.n_out * 2 * c.L * c.N * _taps(s)
    path = 2.0 if c.direct else float(s.depthwise)
    return np.array([math.log2(c.N), c.L, math.log2(c.ci), math.log2(c.c_n),
                     math.log2(d.n_in), math.log2(d.n_out), math.log2(macs), path],
                    dtype=np.float64)


class Timer:
    """Times one image of a layer configuration on the GPU: forward NTT of the
    input ciphertexts, multiply-accumulate (with Walsh recombination) and
    inverse NTT of the outputs, or the direct convolution for a direct
    candidate; best of `reps` after a warm-up."""

    def __init__(self, pool_words: int = MAX_BYTES // 4, reps: int = 3):
        import torch
        self.torch = torch
        self.reps = reps
        self.ctx = {}
        # residues below 2^29 are canonical for every prime in (2^29, 2^31)
        self.pool = torch.randint(0, 1 << 29, (pool_words,), dtype=torch.int32, device="cuda")
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def _ctx(self, N, L):
        if (N, L) not in self.ctx:
            self.ctx[(N, L)] = hyena_create(N, L)
        return self.ctx[(N, L)]

    def time_ms(self, s: Shape, c: Cand) -> float:
        ctx = self._ctx(c.N, c.L)
        d = hyena_conv_plan(ctx, s.H, s.W, s.Ci, s.Co, s.k, depthwise=s.depthwise, c_n=c.c_n, ci_req=c.ci,
                            flags=HYENA_FUSE_WHT)
        LN = c.L * c.N
        n_ct, n_out, n_w = d.n_in * 2 * LN, d.n_out * 2 * LN, d.Co * d.w_groups * LN
        if n_ct + n_out + n_w > self.pool.numel():
            raise ValueError("configuration larger than the timing pool")
        ct = self.pool[:n_ct]
        w = self.pool[n_ct:n_ct + n_w]
        out = self.pool[n_ct + n_w:n_ct + n_w + n_out]

        wi8 = self.pool.view(self.torch.int8)[4 * n_ct:4 * n_ct + d.Co * (1 if s.depthwise else s.Ci) * s.k * s.k]

        def run():
            if c.direct:
                hyena_conv_direct(ctx, d, ct, wi8, out)
                return
            hyena_ntt(ctx, ct)
            hyena_conv(ctx, d, ct, w, out)
            hyena_intt(ctx, out)

        run()
        best = 1e30
        for _ in range(self.reps):
            self.e0.record()
            run()
            self.e1.record()
            self.e1.synchronize()
            best = min(best, self.e0.elapsed_time(self.e1))
        return best


class MLP:
    """The cost model: standardised features -> log(ms), trained with Adam on
    the GPU by the library's forward / backward / Adam kernels."""

    def __init__(self, seed: int = 0, device: str = "cuda"):
        import torch
        self.torch = torch
        self.device = device
        n = hyena_mlp_params()
        rng = np.random.default_rng(seed)
        th = np.zeros(n, dtype=np.float32)
        # He initialisation of W1, W2, W3 (biases zero)
        th[0:512] = rng.normal(0, math.sqrt(2 / 8), 512)
        th[576:576 + 4096] = rng.normal(0, math.sqrt(2 / 64), 4096)
        th[4736:4800] = rng.normal(0, math.sqrt(1 / 64), 64)
        self.theta = torch.from_numpy(th).to(device)
        self.mu = self.sd = None
        self.y_mu = 0.0
        # Adam state, kept so that training can resume from a saved model
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step = 0

    def save(self, path: str) -> None:
        """Parameters, feature standardisation and Adam state in one .npz
        (plain arrays, no pickled objects)."""
        np.savez(path, theta=self.theta.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
                 step=np.int64(self.step), mu=np.asarray(self.mu, dtype=np.float64),
                 sd=np.asarray(self.sd, dtype=np.float64), y_mu=np.float64(self.y_mu))

    @classmethod
    def load(cls, path: str, device: str = "cuda") -> "MLP":
        z = np.load(path, allow_pickle=False)
        if z["theta"].shape != (hyena_mlp_params(),):
            raise ValueError(f"{path}: parameter count {z['theta'].shape} is not the library's MLP")
        mdl = cls(0, device)
        mdl.theta = mdl.torch.from_numpy(z["theta"].astype(np.float32)).to(device)
        mdl.m = mdl.torch.from_numpy(z["m"].astype(np.float32)).to(device)
        mdl.v = mdl.torch.from_numpy(z["v"].astype(np.float32)).to(device)
        mdl.step = int(z["step"])
        mdl.mu, mdl.sd, mdl.y_mu = z["mu"], z["sd"], float(z["y_mu"])
        return mdl

    def _std(self, X):
        return ((X - self.mu) / self.sd).astype(np.float32)

    def fit(self, X: np.ndarray, y: np.ndarray, steps: int = 4000, lr: float = 3e-3, log=None,
            resume: bool = False):
        """Full-batch Adam on the mean squared error of log(ms). With
        ``resume`` (a loaded model), training continues from the saved
        parameters, Adam moments and step count, with the saved feature
        standardisation; ``steps`` more steps are taken."""
        torch = self.torch
        if not resume or self.mu is None:
            self.mu = X.mean(axis=0)
            self.sd = X.std(axis=0) + 1e-6
            self.y_mu = float(y.mean())
            self.m.zero_()
            self.v.zero_()
            self.step = 0
        Xd = torch.from_numpy(self._std(X)).cuda()
        yd = torch.from_numpy((y - self.y_mu).astype(np.float32)).cuda()
        grad = torch.zeros_like(self.theta)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        work = torch.empty(hyena_mlp_workspace_floats(X.shape[0]), dtype=torch.float32, device="cuda")
        hist = []
        for i in range(1, steps + 1):
            self.step += 1
            hyena_mlp_loss_grad(self.theta, Xd, yd, grad, loss, work)
            hyena_mlp_adam(self.theta, grad, self.m, self.v, self.step,
                           lr * (0.1 if i > 0.75 * steps else 1.0))
            if i % 500 == 0 or i == 1:
                hist.append((self.step, float(loss.item())))
                if log:
                    log(f"  step {self.step}: mse {hist[-1][1]:.4f}")
        return hist

    def predict(self, X: np.ndarray) -> np.ndarray:
        torch = self.torch
        Xd = torch.from_numpy(self._std(X)).cuda()
        yd = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        hyena_mlp_forward(self.theta, Xd, yd)
        return yd.cpu().numpy().astype(np.float64) + self.y_mu


def random_shapes(seed: int, n: int, exclude=()):
    """Random conv layer shapes in the range of ImageNet CNNs."""
    rng = np.random.default_rng(seed)
    ex = set(exclude)
    out = []
    while len(out) < n:
        H = int(rng.choice([7, 10, 14, 20, 28, 40, 56, 80, 112, 160, 224]))
        dw = bool(rng.random() < 0.3)
        k = 3 if (dw or rng.random() < 0.6) else 1
        Ci = int(2 ** rng.uniform(1.5, 10))
        Co = Ci if dw else int(2 ** rng.uniform(3, 10))
        Co = max(4, Co // 4 * 4)
        if dw:
            Ci = Co
        s = Shape(H, H, Ci, Co, k, dw)
        if s in ex:
            continue
        out.append(s)
    return out


def mobilenet_shapes():
    # the workloads module lists the layer table; reproduced as shapes here so
    # that the library does not depend on the test-side input generators
    res, out = 224, [Shape(224, 224, 3, 32, 3, False)]
    h, c = 112, 32
    for co, st in [(64, 1), (128, 2), (128, 1), (256, 2), (256, 1), (512, 2), (512, 1), (512, 1), (512, 1),
                   (512, 1), (512, 1), (1024, 2), (1024, 1)]:
        out.append(Shape(h, h, c, c, 3, True))
        h //= st
        out.append(Shape(h, h, c, co, 1, False))
        c = co
    del res
    return out


def collect(timer: Timer, shapes, per_shape: int, seed: int, log=None):
    """Timed samples: `per_shape` random candidates of every shape."""
    rng = np.random.default_rng(seed)
    X, y = [], []
    for i, s in enumerate(shapes):
        cands = candidates(s)
        if not cands:
            continue
        pick = rng.choice(len(cands), min(per_shape, len(cands)), replace=False)
        for j in pick:
            c = cands[int(j)]
            X.append(features(s, c))
            y.append(math.log(timer.time_ms(s, c)))
        if log and (i + 1) % 100 == 0:
            log(f"  timed {len(y)} samples ({i + 1}/{len(shapes)} shapes)")
    return np.array(X), np.array(y)


def evaluate(timer: Timer, model: MLP, shapes, log=None):
    """Exhaustive timing of every candidate of every layer (the reference), the
    model's picks, and the default parameters."""
    rows = []
    t_search = 0.0
    t_model = 0.0
    for s in shapes:
        cands = candidates(s)
        t0 = time.perf_counter()
        times = [timer.time_ms(s, c) for c in cands]
        t_search += time.perf_counter() - t0
        t0 = time.perf_counter()
        pred = model.predict(np.array([features(s, c) for c in cands]))
        t_model += time.perf_counter() - t0
        ib, ip = int(np.argmin(times)), int(np.argmin(pred))
        dc = default_candidate(s)
        t_def = timer.time_ms(s, dc)
        rows.append({"shape": s.__dict__, "candidates": len(cands), "best": cands[ib].__dict__,
                     "best_ms": times[ib], "model": cands[ip].__dict__, "model_ms": times[ip],
                     "default": dc.__dict__, "default_ms": t_def})
        if log:
            log(f"  {s}: {len(cands)} cands, best {times[ib]:.3f} ms, model {times[ip]:.3f}, default {t_def:.3f}")
    tot = {k: sum(r[k] for r in rows) for k in ("best_ms", "model_ms", "default_ms")}
    return {"layers": rows, "total_best_ms": tot["best_ms"], "total_model_ms": tot["model_ms"],
            "total_default_ms": tot["default_ms"],
            "regret": tot["model_ms"] / tot["best_ms"] - 1.0,
            "gain_over_default": tot["default_ms"] / tot["model_ms"],
            "exhaustive_search_s": t_search, "model_search_s": t_model,
            "candidates": sum(r["candidates"] for r in rows)}


def run(train_shapes: int = 700, per_shape: int = 4, steps: int = 4000, seed: int = 0, log=None,
        save: str | None = None, load: str | None = None):
    """Collect timed samples of random shapes, train the MLP (or, with
    ``load``, continue training a saved one for ``steps`` more steps; with
    steps = 0 it is used as saved), optionally save it, and evaluate it on
    MobileNetV1 against exhaustive search and the default parameters."""
    timer = Timer()
    mob = mobilenet_shapes()
    shapes = random_shapes(seed, train_shapes, exclude=mob)
    t0 = time.perf_counter()
    X, y = collect(timer, shapes, per_shape, seed, log) if train_shapes else (np.zeros((0, 8)), np.zeros(0))
    t_collect = time.perf_counter() - t0
    if log:
        log(f"{len(y)} training samples in {t_collect:.1f} s")
    model = MLP.load(load) if load else MLP(seed)
    t0 = time.perf_counter()
    hist = model.fit(X, y, steps=steps, log=log, resume=bool(load)) if steps and len(y) else []
    t_train = time.perf_counter() - t0
    if save:
        model.save(save)
    report = evaluate(timer, model, mob, log)
    report.update({"train_samples": int(len(y)), "train_shapes": train_shapes, "collect_s": t_collect,
                   "train_s": t_train, "train_mse_history": hist, "mlp": "8-64-64-1 ReLU, fp32, Adam",
                   "adam_steps": model.step})
    return report


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-shapes", type=int, default=700)
    ap.add_argument("--per-shape", type=int, default=4)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--save", default=None, help="write the trained model (.npz) here")
    ap.add_argument("--load", default=None, help="start from this saved model (training resumes)")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    rep = run(a.train_shapes, a.per_shape, a.steps, a.seed, log, save=a.save, load=a.load)
    summary = {k: v for k, v in rep.items() if k != "layers"}
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rep, f, indent=1)
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
