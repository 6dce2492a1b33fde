"""Throughput of the Hyena HE-convolution hot path on one MI355X.

Workload: the 13 convolution layers of VGG-16 at 224x224 (widths 64, 128,
256, 512, 512; 3x3, pad 1) for a batch of 8 images, BFV ring N = 8192 with
three RNS primes below 2^31, plaintext modulus 2^20. One step is the whole
server-side path for every (image, layer): forward NTT of the input
ciphertexts, the multiply-accumulate over input ciphertexts with lazy
reduction, the Walsh-Hadamard recombination (c_n = 1 here: every VGG layer at
N = 8192 packs at most 32 channels, and the paper's choice is c_n <= 2; the
butterflies are exercised by the tests) and the inverse NTT of the output
ciphertexts. Weights are encoded once, before timing (the paper's offline
weight preparation). Inputs are uniform residues drawn on the GPU from a
seeded generator (distributed as fresh ciphertexts), resident in HBM before
the timed region.

Three schedules of the same arithmetic are timed:
  plain   - per image and layer: ntt, conv, intt through the C ABI with the
            default kernel schedules;
  batched - per layer, all 8 images in one launch of each kernel, so each
            encoded-weight word is read once per batch instead of per image;
  tuned   - the batched path object: NTT schedule per direction and MAC
            schedule per layer picked by the autotuner, every layer's
            multiply-accumulate in one persistent launch, the whole step
            captured in a hipGraph and replayed. Phase durations come from HIP
            events recorded on the launch stream between the graphs of the
            three phases (a timed run replays one graph per phase).
Before timing, one step of each schedule runs from pristine inputs and two
output ciphertexts per layer (every coefficient of both parts and all limbs)
are copied to the host; the cpu_baseline leg, the only part of this script
that runs the oracle, computes those outputs (timed as part of the baseline)
and checks every schedule's against them bit for bit.
`value` is the tuned schedule's throughput.

`--copy-calibration` instead times a plain 1 GiB device copy (the reference
kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters).

Prints one JSON line (rank 0, N=1 GPU).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# ALU roof of the integer kernels: 32-bit integer VALU instructions, the
# 64-bit multiply-add included, issue at 16 lanes per clock per SIMD:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s (measured
# 36.7-38.7 T/s by --alu-calibration; the fp32 vector peak of 157.3 TFLOP/s
# counts packed fp32 FMAs, which integer code has no form of). A coeff-MAC is
# one v_mad_u64_u32 plus its share of the accumulator folds: a v_mov and a
# v_mad_u64_u32 per accumulator after every F products (F from the primes,
# lazy_fold_interval; the instructions of the multiply-accumulate loop)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# integer VALU instructions of one exact butterfly with primes below 2^31: a
# Montgomery product (two v_mad_u64_u32, one v_mul_lo_u32) and seven adds,
# subtracts and minima (the modular sum, difference and corrections)
NTT_OPS_PER_BUTTERFLY = 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "mac_vgg16_b8_n8192_counters.md")
MAC_SOURCES = ["paper_2311_12519_amd/csrc/mac.h", "paper_2311_12519_amd/csrc/batch.hip",
               "paper_2311_12519_amd/csrc/conv.hip", "paper_2311_12519_amd/csrc/internal.h"]


def measured_traffic(kernel):
    """HBM bytes per step of the MAC kernel from the committed rocprofv3
    counter summary, or None when it was taken for another kernel or the MAC
    sources changed since."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in text.splitlines()
                if l.startswith(("traffic_bytes_per_step", "source_sha256_16", "kernel")))
    if vals.get("kernel", "").strip() != kernel:
        return None
    h = hashlib.sha256()
    for f in MAC_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if vals.get("source_sha256_16", "").strip() != h.hexdigest()[:16]:
        return None
    return int(vals["traffic_bytes_per_step"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--images", type=int, default=8)
    ap.add_argument("--layers", type=int, default=13, help="first n VGG layers (13 = all)")
    ap.add_argument("--mode", choices=["all", "plain", "batched", "tuned"], default="all")
    ap.add_argument("--primes", type=int, choices=[30, 31], default=31,
                    help="RNS primes below 2^31 (default) or below 2^30")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--alu-calibration", action="store_true",
                    help="measure the integer VALU rates (v_mad_u64_u32, v_mul_lo/hi_u32, v_add_u32)")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-alt-primes", action="store_true",
                    help="skip the supplementary tuned run with primes below 2^30")
    ap.add_argument("--no-direct", action="store_true",
                    help="skip the supplementary direct-versus-NTT run on MobileNetV1's depthwise layers")
    ap.add_argument("--no-client", action="store_true",
                    help="skip the supplementary client-side run (device encryption and decryption)")
    ap.add_argument("--no-simd", action="store_true",
                    help="skip the supplementary run of the SIMD-setting kernels (HRot, batch encoding, PMult)")
    ap.add_argument("--no-synth", action="store_true",
                    help="skip the supplementary run of the evaluation-domain weight synthesis")
    ap.add_argument("--no-walsh-vgg", action="store_true",
                    help="skip the supplementary VGG-16 step with Walsh-Hadamard packing (c_n = 2)")
    ap.add_argument("--no-config3", action="store_true",
                    help="skip the supplementary run of the ImageNet ResNet layers with Walsh-Hadamard packing")
    ap.add_argument("--no-costmodel", action="store_true",
                    help="skip the supplementary run of the learned cost model on MobileNetV1")
    ap.add_argument("--cm-shapes", type=int, default=700,
                    help="random layer shapes timed to train the cost model (4 candidates each)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


class Layer:
    pass


def lazy_fold_interval(primes):
    """Products the MAC adds between two folds of its 64-bit accumulator
    (one mad per fold): after a fold the accumulator is below 2^32 (r + 1),
    r = 2^32 mod q, and each product is at most (q - 1)^2."""
    f = 15
    for q in primes:
        r = (1 << 32) % q
        f = min(f, ((1 << 64) - 1 - ((r + 1) << 32)) // ((q - 1) ** 2))
    return max(1, f)


def setup(args, hy, wl, torch):
    N, L = 8192, 3
    ctx = hy.hyena_create(N, L, flags=hy.HYENA_PRIMES_30BIT if args.primes == 30 else 0)
    layers = []
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    for li, lay in enumerate(wl.vgg16_layers()[: args.layers]):
        o = Layer()
        o.lay = lay
        o.desc_b = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, c_n=1,
                                      flags=hy.HYENA_FUSE_WHT, batch=args.images)
        o.desc_1 = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, c_n=1,
                                      flags=hy.HYENA_FUSE_WHT, batch=1)
        d = o.desc_b
        seed = wl.layer_seed(4, li)
        o.w = wl.weights(seed, lay)
        o.d_wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device=dev)
        o.d_w = torch.from_numpy(o.w).to(dev)
        hy.hyena_encode_weights(ctx, d, o.d_w, o.d_wn)
        # layers with at most 18 taps per weight word also get their integer
        # taps, so the autotuner can weigh synthesizing the weight words in the
        # multiply-accumulate against streaming them
        o.d_taps = None
        if d.ci * d.k * d.k <= 18:
            o.d_taps = torch.empty(hy.synth_taps_words(d), dtype=torch.int32, device=dev)
            hy.hyena_synth_taps(ctx, d, o.d_w, o.d_taps)
        in_words = d.n_in * 2 * L * N
        out_words = d.n_out * 2 * L * N
        o.ct0 = torch.empty((args.images, in_words), dtype=torch.int32, device=dev)
        v = o.ct0.view(args.images, d.n_in, 2, L, N)
        g.manual_seed(seed)
        for i, q in enumerate(ctx.primes):
            v[:, :, :, i, :] = torch.randint(0, q, v[:, :, :, i, :].shape, generator=g, device=dev,
                                             dtype=torch.int64).to(torch.int32)
        o.ct = o.ct0.clone()
        o.out = torch.empty((args.images, out_words), dtype=torch.int32, device=dev)
        o.macs = d.n_groups * lay.Co * d.tiles * 2 * L * N   # coeff-MACs per image
        o.in_words, o.out_words = in_words, out_words
        layers.append(o)
    torch.cuda.synchronize()
    return ctx, layers


def step_batched(ctx, layers, hy, ev=None):
    for o in layers:
        if ev is not None:
            ev.rec("ntt")
        hy.hyena_ntt(ctx, o.ct)
        if ev is not None:
            ev.rec("ntt_end")
            ev.rec("mac")
        hy.hyena_conv(ctx, o.desc_b, o.ct, o.d_wn, o.out)
        if ev is not None:
            ev.rec("mac_end")
            ev.rec("intt")
        hy.hyena_intt(ctx, o.out)
        if ev is not None:
            ev.rec("intt_end")


def step_plain(ctx, layers, hy, images):
    for o in layers:
        for b in range(images):
            hy.hyena_ntt(ctx, o.ct[b])
            hy.hyena_conv(ctx, o.desc_1, o.ct[b], o.d_wn, o.out[b])
            hy.hyena_intt(ctx, o.out[b])


class Events:
    """HIP events on torch's current stream, the stream every call runs on."""

    def __init__(self, torch):
        self.torch = torch
        self.marks = []

    def rec(self, name):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.marks.append((name, e))

    def totals(self):
        self.torch.cuda.synchronize()
        out, open_ = {}, {}
        for name, e in self.marks:
            if name.endswith("_end"):
                k = name[:-4]
                out.setdefault(k, []).append(open_.pop(k).elapsed_time(e))
            else:
                open_[name] = e
        return out


def sample_outputs(ctx, layers, torch, images, step):
    """One step from pristine inputs; host copies of two sampled output
    ciphertexts per layer (the first and the last (tile, output channel) of
    image layer mod images) and of the inputs they depend on. Nothing here
    computes expected values: the cpu_baseline leg does, with the oracle."""
    N, L = ctx.N, ctx.L
    for o in layers:
        o.ct.copy_(o.ct0)
        o.out.fill_(0)
    torch.cuda.synchronize()
    step()
    torch.cuda.synchronize()
    got = []
    for li, o in enumerate(layers):
        b, tiles, co = li % images, o.desc_b.tiles, o.lay.Co
        out = o.out[b].view(tiles, co, 2, L, N)
        sel = [(0, 0), (tiles - 1, co - 1)]
        got.append((sel, [out[t, oc].cpu().numpy().view(np.uint32).copy() for t, oc in sel]))
    return got


def sampled_inputs(ctx, layers, images):
    """Host copies of the input ciphertexts (coefficient domain) and weights of
    the sampled image of every layer."""
    return [(o.lay, o.ct0[li % images].cpu().numpy().view(np.uint32).copy(), o.w) for li, o in enumerate(layers)]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(ctx, layers, orc, seconds, parity):
    """The oracle (sparse-tap schoolbook, OpenMP) on a bounded sample. It first
    computes the sampled outputs of every parity set (inputs, primes and the
    GPU outputs of each schedule, taken before timing) and checks each
    schedule's outputs against them bit for bit, then continues on whole
    output ciphertexts of random inputs until about `seconds` of CPU time.
    Returns the baseline and the number of output ciphertexts checked."""
    N, L = ctx.N, ctx.L
    done_macs, spent, outs, checked = 0, 0.0, 0, 0
    names = []
    for inputs, primes, by_mode in parity:
        for li, (lay, ct, w) in enumerate(inputs):
            pl = orc.plan(N, lay.H, lay.W, lay.Ci, lay.Co, lay.k)
            sel = next(iter(by_mode.values()))[li][0]
            t0 = time.perf_counter()
            want = orc.conv_products(pl, ct.reshape(pl.tiles, pl.n_groups, 2, L, N), w, primes, outputs=sel)
            spent += time.perf_counter() - t0
            done_macs += len(sel) * pl.n_groups * 2 * L * N
            outs += len(sel)
            names.append(lay.name)
            for mode, samples in by_mode.items():
                s_sel, got = samples[li]
                for u, (tau, oc) in enumerate(s_sel):
                    if not np.array_equal(got[u], want[u]):
                        raise SystemExit(f"parity failure: {mode} layer {lay.name} output {(tau, oc)} "
                                         f"primes {primes}")
                    checked += 1
    rng = np.random.default_rng(0)
    li = 0
    while spent < seconds and li < 64:
        o = layers[li % len(layers)]
        li += 1
        pl = orc.plan(N, o.lay.H, o.lay.W, o.lay.Ci, o.lay.Co, o.lay.k)
        ct = np.empty((pl.tiles, pl.n_groups, 2, L, N), dtype=np.uint32)
        for i, q in enumerate(ctx.primes):
            ct[:, :, :, i, :] = rng.integers(0, q, size=(pl.tiles, pl.n_groups, 2, N))
        n_out = 8
        sel = [(int(rng.integers(pl.tiles)), int(rng.integers(o.lay.Co))) for _ in range(n_out)]
        t0 = time.perf_counter()
        orc.conv_products(pl, ct, o.w, ctx.primes, outputs=sel)
        spent += time.perf_counter() - t0
        done_macs += n_out * pl.n_groups * 2 * L * N
        outs += n_out
        names.append(o.lay.name)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": done_macs / spent, "unit": "coeff-MAC/s", "cores": threads,
            "kind": "oracle", "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "sample": f"{outs} output ciphertexts (all coefficients, 2 parts x {L} limbs) of VGG layers "
                      f"{sorted(set(names))}, {spent:.1f} s"}, checked


def copy_calibration(args, torch):
    n = 1 << 28  # 1 GiB of int32
    a = torch.randint(0, 1 << 30, (n,), dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "ms": dt * 1e3,
                      "GBs": 2 * n * 4 / dt / 1e9}))


def alu_calibration(hy, torch):
    """Lane operations per second of the integer instructions the kernels are
    made of: eight independent chains per lane over 8192 blocks of 256 threads.
    The ALU roof of a coeff-MAC is the v_mad_u64_u32 rate."""
    blocks = 8192
    d = torch.zeros(blocks * 256, dtype=torch.int32, device="cuda")
    rates = {name: hy.hyena_valu_rate(i, d, blocks) / 1e12 for i, name in enumerate(hy.VALU_OPS)}
    print(json.dumps({"unit": "T lane-ops/s", "rates": rates,
                      "issue_peak_nominal": 256 * 4 * 32 * 2.4e9 / 1e12,
                      "valu_peak_tops_used": VALU_PEAK_TOPS}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2311_12519_amd as hy
    import workloads as wl

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_calibration:
        copy_calibration(args, torch)
        return
    if args.alu_calibration:
        alu_calibration(hy, torch)
        return
    hy.lib()
    log("setup ...")
    ctx, layers = setup(args, hy, wl, torch)
    n_img = args.images
    total_macs = sum(o.macs for o in layers) * n_img
    n_layer_runs = len(layers) * n_img

    modes = ["plain", "batched", "tuned"] if args.mode == "all" else [args.mode]
    batch = None
    if "tuned" in modes:
        log("autotuning + graph capture ...")
        flags = hy.HYENA_BATCH_TUNE | hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH | hy.HYENA_BATCH_TIMING
        batch = hy.hyena_batch_create(ctx, [(o.desc_b, o.ct, o.d_wn, o.out, o.d_taps) for o in layers], flags)

    steps = {
        "plain": lambda: step_plain(ctx, layers, hy, n_img),
        "batched": lambda: step_batched(ctx, layers, hy),
        "tuned": lambda: hy.hyena_batch_run(batch),
    }
    # outputs of one step of every schedule, sampled before timing; the
    # cpu_baseline leg checks them against the oracle
    parity = []
    if not args.no_check:
        parity.append((sampled_inputs(ctx, layers, n_img), ctx.primes,
                       {m: sample_outputs(ctx, layers, torch, n_img, steps[m]) for m in modes}))

    res = {}
    for mode in modes:
        fn = steps[mode]
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev = Events(torch) if mode == "batched" else None
        phases = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            if ev is not None:
                step_batched(ctx, layers, hy, ev)
            else:
                fn()
            if mode == "tuned":
                phases.append(hy.hyena_batch_phase_ms(batch))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[mode] = {"ms_per_step": dt * 1e3, "coeff_macs_per_s": total_macs / dt,
                     "layers_per_s": n_layer_runs / dt}
        if ev is not None:
            res[mode]["kernels_ms"] = {k: sum(v) / args.steps for k, v in ev.totals().items()}
        if mode == "tuned":
            ph = np.array(phases).mean(axis=0)
            res[mode]["kernels_ms"] = {"ntt": float(ph[0]), "mac": float(ph[1]), "intt": float(ph[2])}
            info = hy.hyena_batch_info(batch)
            res[mode]["schedules"] = info
        log(f"{mode}: {dt * 1e3:.2f} ms/step, {total_macs / dt / 1e12:.3f} T coeff-MAC/s")

    head_mode = "tuned" if "tuned" in res else ("batched" if "batched" in res else "plain")
    head = res[head_mode]
    # the offline weight preparation (integer Walsh weights -> kernel
    # polynomials -> NTT) of all layers, re-encoded into the same buffers
    enc = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for o in layers:
            hy.hyena_encode_weights(ctx, o.desc_b, o.d_w, o.d_wn)
        e1.record()
        torch.cuda.synchronize()
        enc.append(e0.elapsed_time(e1))
    synth = None if args.no_synth else weight_synthesis(ctx, layers, hy, torch)
    synth_mac = None if args.no_synth else synth_in_mac(ctx, layers, hy, torch)
    out = {
        "metric": "HE-conv coeff-MACs/s + layers/s at N=8192, batched/tuned vs plain; bit-exact",
        "value": head["coeff_macs_per_s"],
        "unit": "coeff-MAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"VGG-16 {len(layers)} conv layers at 224x224, {n_img} images, "
                               f"N=8192, 3 primes < 2^{args.primes}, t=2^20, c_n=1",
                   "images": n_img, "layers": len(layers), "N": 8192, "L": 3, "prime_bits": args.primes,
                   "schedule": head_mode},
        "layers_per_s": head["layers_per_s"],
        "parity_checked_outputs": 0,
        "encode_weights_ms": min(enc),
        "ms_per_step_with_encode": head["ms_per_step"] + min(enc),
        "schedules": res,
    }
    if synth is not None:
        out["weight_synthesis"] = synth
    if synth_mac is not None:
        out["synth_in_mac"] = synth_mac
    if head_mode == "tuned":
        out["synthesized_layers"] = [o.lay.name for o, sid in zip(layers, head["schedules"]["mac_sched"])
                                     if hy.hyena_conv_schedule_taps(sid) > 0]
    if "plain" in res:
        for m in ("batched", "tuned"):
            if m in res:
                out[f"speedup_{m}_vs_plain"] = res["plain"]["ms_per_step"] / res[m]["ms_per_step"]
    if "kernels_ms" in head:
        km = head["kernels_ms"]
        mac_ms = km["mac"]
        # layers whose multiply-accumulate synthesizes the weight words read
        # only their integer taps
        syn = [False] * len(layers)
        if head_mode == "tuned":
            syn = [hy.hyena_conv_schedule_taps(sid) > 0 for sid in head["schedules"]["mac_sched"]]
        w_bytes = sum((o.d_taps.numel() if sy else o.d_wn.numel()) * 4 for o, sy in zip(layers, syn))
        io_bytes = sum((o.in_words + o.out_words) * 4 for o in layers) * n_img
        mac_gbs = (w_bytes + io_bytes) / (mac_ms * 1e-3) / 1e9
        ach = total_macs / (mac_ms * 1e-3) / 1e12
        # VALU instructions per coeff-MAC: the multiply-add and the folds
        fold_f = lazy_fold_interval(ctx.primes)
        ops_per_mac = 1 + 2 / fold_f
        ach_ops = ach * ops_per_mac
        # the binding roof is the one whose time at peak is longer: the HBM
        # time of the algorithmic bytes or the VALU time of the
        # multiply-accumulate's instructions
        t_hbm = (w_bytes + io_bytes) / (HBM_PEAK_GBS * 1e9)
        t_alu = total_macs * ops_per_mac / (VALU_PEAK_TOPS * 1e12)
        # the tuned step runs the multiply-accumulate as one persistent launch
        # unless its autotuner found per-layer launches clearly faster
        persistent = head_mode == "tuned" and head["schedules"]["persistent_launches"] > 0
        kernel = "mac_persistent_kernel" if persistent else "mac_lds_kernel"
        launches = 1 if persistent else len(layers)
        common = {"kernel": kernel,
                  "traffic": measured_traffic(kernel) if head_mode == "tuned" and args.primes == 31 else None,
                  "traffic_unit": "HBM bytes per step (all launches of the kernel)",
                  "algorithmic_bytes_per_step": w_bytes + io_bytes,
                  "launches_per_step": launches,
                  "roof_ms": {"hbm": t_hbm * 1e3, "alu": t_alu * 1e3},
                  "alu_ops_per_coeff_mac": ops_per_mac, "fold_interval": fold_f,
                  "alu_achieved_TOPs": ach_ops, "alu_peak_TOPs": VALU_PEAK_TOPS, "alu_frac": ach_ops / VALU_PEAK_TOPS,
                  "hbm_achieved_GBs": mac_gbs, "hbm_peak_GBs": HBM_PEAK_GBS, "hbm_frac": mac_gbs / HBM_PEAK_GBS}
        if t_hbm >= t_alu:
            out["roofline"] = {"bound": "hbm", "achieved": mac_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": mac_gbs / HBM_PEAK_GBS, **common}
        else:
            out["roofline"] = {"bound": "alu", "achieved": ach_ops, "peak": VALU_PEAK_TOPS,
                               "unit": "T VALU instructions/s (1 + 2/F per coeff-MAC)",
                               "frac": ach_ops / VALU_PEAK_TOPS, **common}
        ntt_bytes = sum(o.in_words * 4 * 2 for o in layers) * n_img
        intt_bytes = sum(o.out_words * 4 * 2 for o in layers) * n_img

        def ntt_roof(ms, nbytes):
            # limb-polynomials of N words; N/2 log2 N butterflies each, every one
            # at least NTT_OPS_PER_BUTTERFLY integer VALU instructions
            polys = nbytes / 8 / 8192
            ops = polys * 4096 * 13 * NTT_OPS_PER_BUTTERFLY
            t_hbm = nbytes / (HBM_PEAK_GBS * 1e9) * 1e3
            t_alu = ops / (VALU_PEAK_TOPS * 1e12) * 1e3
            return {"ms": ms, "GBs": nbytes / (ms * 1e-3) / 1e9, "hbm_frac": t_hbm / ms,
                    "alu_Tops": ops / (ms * 1e-3) / 1e12, "alu_frac": t_alu / ms,
                    "roof_ms": {"hbm": t_hbm, "alu": t_alu}, "bound": "alu" if t_alu > t_hbm else "hbm"}

        out["kernels"] = {
            "ntt": ntt_roof(km["ntt"], ntt_bytes),
            "mac": {"ms": mac_ms, "GBs": mac_gbs, "Tcoeff_macs": ach},
            "intt": ntt_roof(km["intt"], intt_bytes),
        }
    if head_mode == "tuned":
        out["kernels"]["wht"] = wht_bandwidth(ctx, layers, hy, torch)
    if not args.no_client:   # before alt_primes, which releases this run's buffers
        out["client"] = client_side(args, ctx, layers, hy, torch, head["ms_per_step"], n_layer_runs)
    if head_mode == "tuned" and not args.no_walsh_vgg:
        out["walsh_vgg"] = walsh_vgg(args, ctx, layers, hy, torch, batch, head["ms_per_step"], total_macs)
    layers_host = [Layer() for _ in layers]   # what the random part of the baseline needs
    for h, o in zip(layers_host, layers):
        h.lay, h.w = o.lay, o.w
    if args.primes == 31 and args.mode in ("all", "tuned") and not args.no_alt_primes:
        out["primes_below_2^30"], alt_parity = alt_primes(args, hy, wl, torch, layers, n_img, total_macs)
        parity += alt_parity
    if args.mode in ("all", "tuned") and not args.no_direct:
        out["direct_depthwise"] = direct_depthwise(args, hy, wl, torch)
    if not args.no_simd:
        out["simd"] = simd_kernels(hy, torch)
    c3_parity = None
    if not args.no_config3:
        out["config3"], c3_parity = walsh_layers(args, hy, wl, torch)
    c5_parity = None
    if not args.no_costmodel:
        out["config5"], c5_parity = mobilenet_costmodel(args, hy, wl, torch)
    if not args.no_cpu_baseline:
        import oracle as orc
        log("cpu baseline (oracle), with the parity check of the sampled outputs ...")
        out["cpu_baseline"], checked = cpu_baseline(ctx, layers_host, orc, args.cpu_seconds, parity)
        n_alt = 0
        if "primes_below_2^30" in out and alt_parity:
            n_alt = sum(len(sel) for sel, _ in alt_parity[0][2]["tuned"])
            out["primes_below_2^30"]["parity_checked_outputs"] = n_alt
        out["parity_checked_outputs"] = checked - n_alt
        log(f"parity ok: {checked} sampled output ciphertexts bit-exact")
        if c3_parity is not None:
            out["config3"]["parity_checked_outputs"] = check_walsh_layers(orc, c3_parity)
        if c5_parity is not None:
            out["config5"]["end_to_end"]["parity_checked_outputs"] = check_mobilenet(orc, c5_parity)
    else:
        log("no oracle run: outputs not checked (--no-cpu-baseline)")
    print(json.dumps(out))


def walsh_vgg(args, ctx, layers, hy, torch, batch1, step_ms, total_macs):
    """Supplementary figure: the headline step with Walsh-Hadamard output
    packing over pairs of output channels (c_n = 2: Walsh kernels
    c_n^-1 (K_2G + K_2G+1) and c_n^-1 (K_2G - K_2G+1), butterflies fused into
    the MAC epilogue), tuned like the headline. The butterflies recombine the
    pair, so every output coefficient equals the c_n = 1 step's: one step of
    each from the same inputs is compared on all outputs (the c_n = 1 outputs
    are the ones the oracle checks)."""
    log("supplementary run: VGG-16 step with Walsh-Hadamard packing, c_n = 2 ...")
    n_img = args.images
    items = []
    for o in layers:
        lay = o.lay
        d2 = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, c_n=2, flags=hy.HYENA_FUSE_WHT,
                                batch=n_img)
        d1 = o.desc_b
        if (d2.n_in, d2.n_groups, d2.ci, d2.tiles) != (d1.n_in, d1.n_groups, d1.ci, d1.tiles):
            raise SystemExit(f"c_n = 2 plan of {lay.name} packs its inputs differently")
        wn2 = torch.empty(hy.wntt_words(ctx, d2), dtype=torch.int32, device="cuda")
        hy.hyena_encode_weights(ctx, d2, o.d_w, wn2)
        items.append((d2, wn2, torch.empty_like(o.out)))
    flags = hy.HYENA_BATCH_TUNE | hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH | hy.HYENA_BATCH_TIMING
    batch2 = hy.hyena_batch_create(ctx, [(d2, o.ct, wn2, out2) for o, (d2, wn2, out2) in zip(layers, items)],
                                   flags)
    for b in (batch1, batch2):
        for o in layers:
            o.ct.copy_(o.ct0)
        hy.hyena_batch_run(b)
        torch.cuda.synchronize()
    for o, (_, _, out2) in zip(layers, items):
        if not torch.equal(o.out, out2):
            raise SystemExit(f"c_n = 2 outputs of {o.lay.name} differ from the c_n = 1 outputs")
    for _ in range(args.warmup):
        hy.hyena_batch_run(batch2)
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        hy.hyena_batch_run(batch2)
        phases.append(hy.hyena_batch_phase_ms(batch2))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ph = np.array(phases).mean(axis=0)
    res = {"workload": f"VGG-16 {len(layers)} conv layers at 224x224, {n_img} images, N=8192, c_n=2 "
                       "(output-channel pairs, fused butterflies)",
           "c_n": 2, "ms_per_step": dt * 1e3, "coeff_macs_per_s": total_macs / dt,
           "over_c_n_1": dt * 1e3 / step_ms,
           "kernels_ms": {"ntt": float(ph[0]), "mac": float(ph[1]), "intt": float(ph[2])},
           "outputs_equal_to_c_n_1": True, "compared_output_words": sum(int(o.out.numel()) for o in layers),
           "schedules": hy.hyena_batch_info(batch2)}
    hy.hyena_batch_destroy(batch2)
    del items
    torch.cuda.empty_cache()
    log(f"c_n = 2: {dt * 1e3:.2f} ms/step ({res['over_c_n_1']:.3f} of c_n = 1), outputs equal")
    return res


def weight_synthesis(ctx, layers, hy, torch):
    """Every layer's NTT-domain weights made two ways: hyena_encode_weights
    (taps scattered into kernel polynomials, then the NTT) and
    hyena_synth_weights (each word evaluated from the integer taps, ci*k*k
    multiply-adds, no transform). The two must agree on every word."""
    log("supplementary run: evaluation-domain weight synthesis against scatter + NTT ...")
    big = max(o.d_wn.numel() for o in layers)
    scratch = torch.empty(big, dtype=torch.int32, device="cuda")

    def timed(fn):
        best = None
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        return best

    rows = []
    for o in layers:
        d, n = o.desc_b, o.d_wn.numel()
        dst = scratch[:n]
        t_enc = timed(lambda: hy.hyena_encode_weights(ctx, d, o.d_w, o.d_wn))
        t_syn = timed(lambda: hy.hyena_synth_weights(ctx, d, o.d_w, dst))
        if not torch.equal(dst, o.d_wn):
            raise SystemExit(f"synthesised and encoded weights differ on VGG layer {o.lay.name}")
        rows.append({"layer": o.lay.name, "taps_per_word": d.ci * d.k * d.k, "words": n,
                     "encode_ms": t_enc, "synth_ms": t_syn})
    del scratch
    tot_e = sum(r["encode_ms"] for r in rows)
    tot_s = sum(r["synth_ms"] for r in rows)
    c1 = [r for r in rows if r["taps_per_word"] <= 9]
    log(f"weights: scatter + NTT {tot_e:.2f} ms, synthesis {tot_s:.2f} ms for all layers (equal words); "
        f"layers with <= 9 taps per word: {sum(r['encode_ms'] for r in c1):.3f} against "
        f"{sum(r['synth_ms'] for r in c1):.3f} ms")
    return {"encode_ms": tot_e, "synth_ms": tot_s, "bit_exact": True, "layers": rows}


def synth_in_mac(ctx, layers, hy, torch):
    """Supplementary figure: the multiply-accumulate of every VGG-16 layer with
    at most 18 taps per weight word (conv1_1 ... conv3_3), streaming the
    NTT-domain weights against synthesizing them in the block from the integer
    taps (hyena_conv_synth's schedules), each at its fastest schedule, for the
    batch of 8 images and for one image. Both must give the same output words
    (the benchmark stops otherwise)."""
    log("supplementary run: weights synthesized in the multiply-accumulate against streamed ...")
    scheds = hy.hyena_conv_schedules()
    streamed = [sid for sid, info in enumerate(scheds) if info[0] and hy.hyena_conv_schedule_taps(sid) == 0]

    def timed(fn):
        fn()
        best = None
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        return best

    rows = []
    for o in layers:
        if o.d_taps is None:
            continue
        T = o.desc_b.ci * o.desc_b.k * o.desc_b.k
        synth = [sid for sid in range(len(scheds)) if hy.hyena_conv_schedule_taps(sid) >= T]
        row = {"layer": o.lay.name, "taps_per_word": T, "weight_bytes_streamed": o.d_wn.numel() * 4,
               "taps_bytes": o.d_taps.numel() * 4}
        for tag, d, ct, out in (("images_8", o.desc_b, o.ct, o.out), ("images_1", o.desc_1, o.ct[0], o.out[0])):
            ts = {sid: timed(lambda: hy.hyena_conv_tiled(ctx, d, ct, o.d_wn, out, sid)) for sid in streamed}
            bs = min(ts, key=ts.get)
            hy.hyena_conv_tiled(ctx, d, ct, o.d_wn, out, bs)
            ref = out.clone()
            ty = {sid: timed(lambda: hy.hyena_conv_tiled(ctx, d, ct, o.d_taps, out, sid)) for sid in synth}
            by = min(ty, key=ty.get)
            if not torch.equal(out, ref):
                raise SystemExit(f"synthesized and streamed weights give different outputs on {o.lay.name}")
            row[tag] = {"streamed_ms": ts[bs], "streamed_sched": bs, "synth_ms": ty[by], "synth_sched": by,
                        "synth_over_streamed": ty[by] / ts[bs]}
            del ref
        rows.append(row)
        log(f"  {o.lay.name}: 8 images streamed {row['images_8']['streamed_ms']:.3f} ms, synthesized "
            f"{row['images_8']['synth_ms']:.3f}; 1 image {row['images_1']['streamed_ms']:.3f} against "
            f"{row['images_1']['synth_ms']:.3f}")
    return {"layers": rows, "outputs_equal": True}


def wht_bandwidth(ctx, layers, hy, torch):
    """The unfused Walsh-Hadamard pass (hyena_wht_pack) over the largest output
    array of the step, in place, for c_n = 2 and 4 (every VGG-16 layer runs with
    c_n = 1, so the step itself does not run it): algorithmic bytes = read and
    write of every word once."""
    o = max(layers, key=lambda x: x.out.numel())
    res = {"array": o.lay.name, "bytes": o.out.numel() * 4}
    for cn in (2, 4):
        G = o.out.numel() // (cn * 2 * ctx.L * ctx.N)
        hy.hyena_wht_pack(ctx, cn, o.out, o.out, G)
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            hy.hyena_wht_pack(ctx, cn, o.out, o.out, G)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        gbs = 2 * o.out.numel() * 4 / (best * 1e-3) / 1e9
        res[f"c_n={cn}"] = {"ms": best, "GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    return res


def direct_depthwise(args, hy, wl, torch):
    """Supplementary figure: MobileNetV1's 13 depthwise 3x3 layers at 224x224
    for the same number of images, N = 8192, three primes below 2^31, computed
    two ways on the same inputs: the NTT path (forward NTT of the input
    ciphertexts, pointwise product with the encoded weights, inverse NTT; the
    weights encoded beforehand) and the coefficient-domain direct convolution
    from the integer taps (hyena_conv_direct). The two outputs must agree on
    every coefficient (the benchmark stops otherwise); times are per layer the
    best of 3 runs, summed."""
    N, L, n_img = 8192, 3, args.images
    log("supplementary run: direct versus NTT path, MobileNetV1 depthwise layers ...")
    ctx = hy.hyena_create(N, L)
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    t_ntt = t_dir = 0.0
    n_layers = 0
    for li, lay in enumerate(wl.mobilenet_v1_layers()):
        if not lay.depthwise:
            continue
        n_layers += 1
        d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, depthwise=True, c_n=1,
                               flags=hy.HYENA_FUSE_WHT, batch=n_img)
        ct0 = torch.empty(n_img * d.n_in * 2 * L * N, dtype=torch.int32, device=dev)
        v = ct0.view(-1, L, N)
        gen.manual_seed(wl.layer_seed(5, li))
        for i, q in enumerate(ctx.primes):
            v[:, i, :] = torch.randint(0, q, v[:, i, :].shape, generator=gen, device=dev,
                                       dtype=torch.int64).to(torch.int32)
        w = torch.from_numpy(wl.weights(wl.layer_seed(5, li), lay)).to(dev)
        wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device=dev)
        hy.hyena_encode_weights(ctx, d, w, wn)
        ct = torch.empty_like(ct0)
        out_ntt = torch.empty(n_img * d.n_out * 2 * L * N, dtype=torch.int32, device=dev)
        out_dir = torch.empty_like(out_ntt)
        best_n = best_d = 1e30
        for rep in range(4):
            ct.copy_(ct0)
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            hy.hyena_ntt(ctx, ct)
            hy.hyena_conv(ctx, d, ct, wn, out_ntt)
            hy.hyena_intt(ctx, out_ntt)
            e1.record()
            hy.hyena_conv_direct(ctx, d, ct0, w, out_dir)
            e2.record()
            torch.cuda.synchronize()
            if rep:
                best_n = min(best_n, e0.elapsed_time(e1))
                best_d = min(best_d, e1.elapsed_time(e2))
        if not torch.equal(out_ntt, out_dir):
            raise SystemExit(f"direct and NTT paths differ on MobileNetV1 layer {lay.name}")
        t_ntt += best_n
        t_dir += best_d
        del ct0, ct, out_ntt, out_dir, wn
    hy.hyena_destroy(ctx)
    log(f"depthwise layers: NTT path {t_ntt:.3f} ms, direct {t_dir:.3f} ms")
    return {"workload": f"MobileNetV1 13 depthwise 3x3 layers at 224x224, {n_img} images, N=8192, "
                        "3 primes < 2^31",
            "layers": n_layers, "images": n_img, "ntt_path_ms": t_ntt, "direct_ms": t_dir,
            "speedup_direct_vs_ntt": t_ntt / t_dir, "outputs_equal": True}


def client_side(args, ctx, layers, hy, torch, step_ms, n_layer_runs):
    """Supplementary figure: the client's share of one step. In the protocol
    the client holds each layer's input activations (after the nonlinear part)
    and receives each layer's output: it encrypts every layer's input and
    decrypts every layer's output, here on the same GPU
    (hyena_encrypt_device / hyena_decrypt_device: bit for bit the host
    library's ciphertexts and messages). Reported: ciphertexts and bytes each
    way (the step's communication), the device time of both sides (per layer
    the best of 3 runs, summed), layers/s with the client included, and the
    host library's rate on a sample for comparison. Check: every encrypted
    input decrypts back to its message, on every coefficient."""
    N, L, n_img = ctx.N, ctx.L, args.images
    log("supplementary run: client-side encryption and decryption on the device ...")
    dev = torch.device("cuda:0")
    words = 2 * L * N                      # uint32 words per ciphertext
    sk = hy.hyena_keygen(ctx, 2024)
    d_s_hat = torch.empty(L * N, dtype=torch.int32, device=dev)
    hy.hyena_secret_prepare(ctx, torch.from_numpy(sk).to(dev), d_s_hat)
    n_in = [o.ct.numel() // words for o in layers]
    n_out = [o.out.numel() // words for o in layers]
    t = 1 << 20
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    msg_in = torch.randint(-t // 2 + 1, t // 2 + 1, (max(n_in), N), generator=g, device=dev, dtype=torch.int32)
    msg_chk = torch.empty((max(n_in), N), dtype=torch.int32, device=dev)
    msg_out = torch.empty((max(n_out), N), dtype=torch.int32, device=dev)
    work = torch.empty(max(max(n_in), max(n_out)) * L * N, dtype=torch.int32, device=dev)

    def timed(fn):
        best = 1e30
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    t_enc = t_dec = 0.0
    for li, o in enumerate(layers):
        n, m = n_in[li], n_out[li]
        ct = o.ct.view(-1)
        t_enc += timed(lambda: hy.hyena_encrypt_device(ctx, d_s_hat, msg_in[:n], 1000 + li, work[:n * L * N], ct))
        hy.hyena_decrypt_device(ctx, d_s_hat, ct, work[:n * L * N], msg_chk[:n])
        if not torch.equal(msg_chk[:n], msg_in[:n]):
            raise SystemExit(f"device encryption of layer {o.lay.name} does not decrypt to its messages")
        t_dec += timed(lambda: hy.hyena_decrypt_device(ctx, d_s_hat, o.out.view(-1), work[:m * L * N],
                                                       msg_out[:m]))
        o.ct.copy_(o.ct0)
    # the host library (multithreaded C++) on a sample of 16 ciphertexts
    k = 16
    msg_h = msg_in[:k].cpu().numpy()
    t0 = time.perf_counter()
    ct_h = hy.hyena_encrypt(ctx, sk, msg_h, 5)
    t1 = time.perf_counter()
    hy.hyena_decrypt(ctx, sk, ct_h)
    t2 = time.perf_counter()
    up, down = sum(n_in), sum(n_out)
    b_ct = words * 4
    enc_bytes = up * (b_ct + 4 * N)          # read the messages, write the ciphertexts
    dec_bytes = down * (b_ct + 4 * N)        # read the ciphertexts, write the messages
    with_client = step_ms + t_enc + t_dec
    log(f"client: encrypt {up} ct {t_enc:.3f} ms, decrypt {down} ct {t_dec:.3f} ms")
    return {"workload": f"inputs and outputs of the same {len(layers)} VGG-16 layers, {n_img} images",
            "ciphertexts_up": up, "ciphertexts_down": down,
            "bytes_up": up * b_ct, "bytes_down": down * b_ct,
            "encrypt_ms": t_enc, "decrypt_ms": t_dec,
            "encrypt_ct_per_s": up / (t_enc * 1e-3), "decrypt_ct_per_s": down / (t_dec * 1e-3),
            "encrypt_GBs": enc_bytes / (t_enc * 1e-3) / 1e9, "decrypt_GBs": dec_bytes / (t_dec * 1e-3) / 1e9,
            "algorithmic_bytes": {"encrypt": enc_bytes, "decrypt": dec_bytes},
            "step_ms": step_ms, "step_with_client_ms": with_client,
            "layers_per_s_with_client": n_layer_runs / (with_client * 1e-3),
            "roundtrip_checked_ciphertexts": up,
            "host_library": {"sample_ciphertexts": k, "threads": min(16, os.cpu_count() or 1),
                             "encrypt_ct_per_s": k / (t1 - t0), "decrypt_ct_per_s": k / (t2 - t1)}}


def simd_kernels(hy, torch):
    """Supplementary figure: the kernels of the paper's own SIMD setting at its
    parameters (n = 2048, a 60-bit q as two primes below 2^30, p = 307201):
    hoisted HRot of 2048 ciphertexts by the nine rotations of a 3x3 kernel over
    a 32-wide slot row, for three decomposition bases (more digits: more work,
    less noise), batch encoding and decoding, PMult by the [k, -k] plaintext and
    one automorphism, each the best of 3 runs (HIP events). Check: sampled
    rotated ciphertexts decrypt to the automorphism of their messages."""
    N, L, p, n_ct = 2048, 2, 307201, 2048
    log("supplementary run: SIMD-setting kernels (n = 2048) ...")
    dev = torch.device("cuda:0")
    ctx = hy.hyena_create(N, L, flags=hy.HYENA_PRIMES_30BIT | hy.HYENA_ALLOW_INSECURE)
    pctx = hy.hyena_create(N, 1, primes=[p], flags=hy.HYENA_PLAINTEXT_PRIME)
    LN = L * N
    sk = hy.hyena_keygen(ctx, 11)
    t = 1 << 20
    rng = np.random.default_rng(5)
    msg = rng.integers(-t // 2 + 1, t // 2 + 1, size=(n_ct, N)).astype(np.int32)
    d_sk = torch.from_numpy(sk).to(dev)
    d_s = torch.empty(LN, dtype=torch.int32, device=dev)
    hy.hyena_secret_prepare(ctx, d_sk, d_s)
    d_msg = torch.from_numpy(msg).to(dev)
    d_ct = torch.empty(n_ct * 2 * LN, dtype=torch.int32, device=dev)
    tmp = torch.empty(n_ct * LN, dtype=torch.int32, device=dev)
    hy.hyena_encrypt_device(ctx, d_s, d_msg, 3, tmp, d_ct)
    offs = [(di - 1) * 32 + (dj - 1) for di in range(3) for dj in range(3)]
    gs = [pow(3, o % (N // 2), 2 * N) for o in offs]

    def best(fn, reps=3):
        b = 1e30
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            b = min(b, e0.elapsed_time(e1))
        return b

    res = {"workload": f"n=2048, q = 2 primes < 2^30, p = {p}, {n_ct} ciphertexts x 9 rotations", "hrot": {}}
    d_out = torch.empty(n_ct * len(gs) * 2 * LN, dtype=torch.int32, device=dev)
    for b in (8, 11, 16):
        D = hy.n_digits(b)
        keys = np.stack([hy.hyena_galois_keygen(ctx, sk, g, b, 100 + g) for g in gs])
        d_k = torch.from_numpy(keys.view(np.int32)).to(dev)
        hy.hyena_ksk_prepare(ctx, d_k)
        work = torch.empty(n_ct * (L * D + 1) * LN, dtype=torch.int32, device=dev)
        ms = best(lambda: hy.hyena_hrot_hoisted(ctx, d_ct, gs, b, d_k, work, d_out))
        # semantic check on sampled outputs (host decryption)
        outv = d_out.view(n_ct, len(gs), 2, L, N)
        for m, r in [(0, 0), (n_ct - 1, 8), (777, 4)]:
            got = hy.hyena_decrypt(ctx, sk, outv[m, r].cpu().numpy().view(np.uint32)[None])[0]
            a = msg[m].astype(np.int64) % t
            want = np.zeros(N, dtype=np.int64)
            g = gs[r]
            for j in range(N):
                e = j * g % (2 * N)
                if e < N:
                    want[e] = (want[e] + a[j]) % t
                else:
                    want[e - N] = (want[e - N] - a[j]) % t
            want = np.where(want > t // 2, want - t, want)
            if not np.array_equal(got, want):
                raise SystemExit(f"hoisted HRot (b={b}) output ({m}, {r}) does not decrypt to m(X^g)")
        # HBM floor: read the work array once, write the rotations, read the keys once
        alg = n_ct * (L * D + 1) * LN * 4 + n_ct * len(gs) * 2 * LN * 4 + keys.nbytes
        res["hrot"][f"b={b}"] = {"digits_per_limb": D, "ms": ms, "rotations_per_s": n_ct * len(gs) / (ms * 1e-3),
                                 "noise_bound_bits": math.log2(L * D * N * ((1 << b) - 1) * 32),
                                 "algorithmic_GBs": alg / (ms * 1e-3) / 1e9}
        del d_k, work
    # batch encoding / decoding over Z_p
    slots = torch.from_numpy(rng.integers(0, p, size=(n_ct, N)).astype(np.int32)).to(dev)
    coef = torch.empty_like(slots)
    back = torch.empty_like(slots)
    res["encode_ms"] = best(lambda: hy.hyena_simd_encode(pctx, slots, coef))
    res["decode_ms"] = best(lambda: (hy.hyena_simd_encode(pctx, slots, coef), hy.hyena_simd_decode(pctx, coef, back)))
    res["decode_ms"] -= res["encode_ms"]
    if not torch.equal(back, slots):
        raise SystemExit("SIMD decode(encode(v)) != v")
    _, k, kh = hy.hyena_simd_params(N, p, 61)
    # PMult by the [k, -k] plaintext and one automorphism over the rotated ciphertexts
    d_o = torch.empty_like(d_out)
    pm = best(lambda: hy.hyena_pmult_sparse(ctx, d_out, [N // 4, 3 * N // 4], [kh, kh], d_o))
    au = best(lambda: hy.hyena_automorphism(ctx, d_out, 3, d_o))
    nbytes = 2 * d_out.numel() * 4
    res["pmult_pm_k"] = {"k": k, "kh": kh, "bytes": nbytes, "ms": pm, "GBs": nbytes / (pm * 1e-3) / 1e9}
    res["automorphism"] = {"bytes": nbytes, "ms": au, "GBs": nbytes / (au * 1e-3) / 1e9}
    res["encode_polys_per_s"] = n_ct / (res["encode_ms"] * 1e-3)
    del d_o, d_out
    hy.hyena_destroy(pctx)
    hy.hyena_destroy(ctx)
    res["conv_layer"] = simd_conv_layer(hy, torch, best, k, kh)
    log(f"simd: hrot b=16 {res['hrot']['b=16']['ms']:.3f} ms for {n_ct}x9, encode {res['encode_ms']:.3f} ms")
    return res


def simd_conv_layer(hy, torch, best, k, kh):
    """One convolution layer in the paper's SIMD setting with c_n = 2: 30x30
    images (32x32 frames, one channel per slot row), 64 -> 64 channels, 3x3,
    n = 2048, three primes below 2^30 (a 90-bit q: the noise of 288 scaled
    rotations plus the [k, -k] PMult needs more than the paper's 60 bits with
    this key switching), decomposition base 2^8. Steps: hoisted HRot of the
    32 input ciphertexts by the nine offsets; CMult-accumulate of the A and B
    Walsh components of every output channel over the 288 rotations; PMult of
    B by the [k, -k] plaintext; A + PMult(B); row-swap HRot; HAdd. Inputs are
    random valid residues (the time does not depend on them; parity of the
    same composition is a GPU test). The coefficient-encoded path (NTT, MAC,
    inverse NTT) of the same layer at the same n and q is timed beside it."""
    N, L, b, Ci, Co, fw = 2048, 3, 8, 64, 64, 32
    dev = torch.device("cuda:0")
    ctx = hy.hyena_create(N, L, flags=hy.HYENA_PRIMES_30BIT | hy.HYENA_ALLOW_INSECURE)
    LN, D, n_in = L * N, hy.n_digits(b), Ci // 2
    i32 = dict(dtype=torch.int32, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    ct = torch.empty((n_in, 2, L, N), **i32)
    for i, q in enumerate(ctx.primes):
        ct[:, :, i, :] = torch.randint(0, q, ct[:, :, i, :].shape, generator=g, device=dev, dtype=torch.int64).to(torch.int32)
    ct = ct.view(-1)
    sk = hy.hyena_keygen(ctx, 5)
    gs = [pow(3, ((di - 1) * fw + (dj - 1)) % (N // 2), 2 * N) for di in range(3) for dj in range(3)]
    keys = torch.from_numpy(np.stack([hy.hyena_galois_keygen(ctx, sk, gg, b, 10 + i) for i, gg in enumerate(gs)]).view(np.int32)).to(dev)
    skey = torch.from_numpy(hy.hyena_galois_keygen(ctx, sk, 2 * N - 1, b, 99).view(np.int32)).to(dev)
    hy.hyena_ksk_prepare(ctx, keys)
    hy.hyena_ksk_prepare(ctx, skey)
    rng = np.random.default_rng(9)
    wa, wb = hy.hyena_simd_conv_weights(rng.integers(-8, 8, size=(Co, Ci, 3, 3)).astype(np.int8), k)
    d_wa, d_wb = torch.from_numpy(wa).to(dev), torch.from_numpy(wb).to(dev)
    work = torch.empty(hy.hyena_simd_conv_workspace(ctx, n_in, Co, b), **i32)
    out = torch.empty(Co * 2 * LN, **i32)
    ms = best(lambda: hy.hyena_simd_conv_cn2(ctx, ct, fw, d_wa, d_wb, kh, b, keys, skey, work, out))
    res = {"workload": "30x30, 64 -> 64 channels, 3x3, n=2048, 3 primes < 2^30, base 2^8, c_n = 2",
           "ms": ms, "input_ciphertexts": n_in, "rotations": n_in * 9 + Co, "output_ciphertexts": Co,
           "call": "hyena_simd_conv_cn2"}
    # the same layer with output channel packing: two output channels per output ciphertext
    pa, pb = hy.hyena_simd_conv_weights_packed(rng.integers(-8, 8, size=(Co, Ci, 3, 3)).astype(np.int8), k)
    d_pa, d_pb = torch.from_numpy(pa).to(dev), torch.from_numpy(pb).to(dev)
    pwork = torch.empty(hy.hyena_simd_conv_packed_workspace(ctx, n_in, Co, b), **i32)
    pout = torch.empty(Co // 2 * 2 * LN, **i32)
    del work
    res["output_packed"] = {"ms": best(lambda: hy.hyena_simd_conv_packed(ctx, ct, fw, d_pa, d_pb, kh, b, keys, skey,
                                                                          pwork, pout)),
                            "rotations": n_in * 10, "output_ciphertexts": Co // 2,
                            "output_bytes": Co // 2 * 2 * LN * 4, "call": "hyena_simd_conv_packed"}
    del pwork
    # the coefficient-encoded path of the same layer at the same n and q
    d = hy.hyena_conv_plan(ctx, 30, 30, Ci, Co, 3, c_n=1, flags=hy.HYENA_FUSE_WHT)
    wt = torch.from_numpy(rng.integers(-8, 8, size=(Co, Ci, 3, 3)).astype(np.int8)).to(dev)
    wn = torch.empty(hy.wntt_words(ctx, d), **i32)
    hy.hyena_encode_weights(ctx, d, wt, wn)
    cin = torch.empty(d.n_in * 2 * LN, **i32)
    cin.copy_(ct[:cin.numel()].repeat(cin.numel() // ct.numel() + 1)[:cin.numel()])
    cout = torch.empty(d.n_out * 2 * LN, **i32)

    def coeff():
        hy.hyena_ntt(ctx, cin)
        hy.hyena_conv(ctx, d, cin, wn, cout)
        hy.hyena_intt(ctx, cout)

    res["coefficient_path"] = {"ms": best(coeff), "input_ciphertexts": d.n_in, "output_ciphertexts": d.n_out,
                               "channels_per_ciphertext": d.ci}
    # the decomposition base from the worst-case noise budget, with the [k, -k]
    # plaintext and with the [1, -1] one, and the layer at the chosen base
    h = hy.hyena_simd_params(N, 307201, 61)[0]
    bk, mk = hy.hyena_simd_conv_choose_base(ctx, 307201, kh, wa, wb)
    wa1, wb1 = hy.hyena_simd_conv_weights(rng.integers(-8, 8, size=(Co, Ci, 3, 3)).astype(np.int8), 1)
    b1, m1 = hy.hyena_simd_conv_choose_base(ctx, 307201, h, wa1, wb1)
    keys_c = torch.from_numpy(np.stack([hy.hyena_galois_keygen(ctx, sk, gg, bk, 20 + i)
                                        for i, gg in enumerate(gs)]).view(np.int32)).to(dev)
    skey_c = torch.from_numpy(hy.hyena_galois_keygen(ctx, sk, 2 * N - 1, bk, 98).view(np.int32)).to(dev)
    hy.hyena_ksk_prepare(ctx, keys_c)
    hy.hyena_ksk_prepare(ctx, skey_c)
    work_c = torch.empty(hy.hyena_simd_conv_workspace(ctx, n_in, Co, bk), **i32)
    res["noise_chosen_base"] = {
        "log2_base_k_plaintext": bk, "margin_bits": mk, "digits_per_limb": hy.n_digits(bk),
        "log2_base_pm1_plaintext": b1, "digits_per_limb_pm1": hy.n_digits(b1),
        "ms": best(lambda: hy.hyena_simd_conv_cn2(ctx, ct, fw, d_wa, d_wb, kh, bk, keys_c, skey_c, work_c, out))}
    hy.hyena_destroy(ctx)
    log(f"simd conv layer {ms:.3f} ms at base 2^{b}, {res['noise_chosen_base']['ms']:.3f} ms at the chosen 2^{bk}, "
        f"output-packed {res['output_packed']['ms']:.3f} ms "
        f"(coefficient path {res['coefficient_path']['ms']:.3f} ms)")
    return res


def walsh_layers(args, hy, wl, torch):
    """Supplementary figure: the ImageNet ResNet-shaped layers with the
    paper's Walsh-Hadamard output-channel packing and lazy reduction
    (56x56x64 -> 64 at c_n = 4, 14x14x256 -> 256 at c_n = 64; N = 16384, four
    primes below 2^31; one image each, as the workload states). Each layer is
    timed as forward NTT of its inputs, multiply-accumulate over the Walsh
    weights with the butterflies (fused into the MAC's epilogue where c_n
    divides the register tile's outputs, else the separate butterfly pass
    that hyena_conv launches), and inverse NTT; beside it the same layer
    with c_n = 1 (no Walsh step) and with the butterflies always unfused
    (hyena_conv without HYENA_FUSE_WHT, then hyena_wht_pack). Every variant
    gives the same output ciphertexts: two per layer and variant are copied to
    the host for the cpu_baseline leg to check against the oracle."""
    N, L = 16384, 4
    log("supplementary run: ResNet layers with Walsh-Hadamard packing (N = 16384, L = 4) ...")
    ctx = hy.hyena_create(N, L)
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    wk = wl.WORKLOADS[3]
    rows, parity = [], []
    for li, (lay, cn) in enumerate(zip(wk.layers, wk.c_n)):
        seed = wl.layer_seed(3, li)
        w_host = wl.weights(seed, lay)
        w = torch.from_numpy(w_host).to(dev)
        variants = [("walsh", cn, True), ("walsh_unfused", cn, False), ("no_walsh", 1, True)]
        d0 = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, c_n=1, flags=hy.HYENA_FUSE_WHT)
        ct0 = torch.empty(d0.n_in * 2 * L * N, dtype=torch.int32, device=dev)
        v = ct0.view(-1, L, N)
        gen.manual_seed(seed)
        for i, q in enumerate(ctx.primes):
            v[:, i, :] = torch.randint(0, q, v[:, i, :].shape, generator=gen, device=dev,
                                       dtype=torch.int64).to(torch.int32)
        ct = torch.empty_like(ct0)
        out = torch.empty(d0.n_out * 2 * L * N, dtype=torch.int32, device=dev)
        row = {"layer": f"{lay.H}x{lay.W}x{lay.Ci}->{lay.Co} 3x3", "c_n": cn, "input_ciphertexts": d0.n_in,
               "output_ciphertexts": d0.n_out, "channels_per_ciphertext": d0.ci}
        macs = d0.n_groups * lay.Co * d0.tiles * 2 * L * N
        sel = [(0, 0), (d0.tiles - 1, lay.Co - 1)]
        samples = {}
        for name, c, fuse in variants:
            d = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, c_n=c,
                                   flags=hy.HYENA_FUSE_WHT if fuse else 0)
            wn = torch.empty(hy.wntt_words(ctx, d), dtype=torch.int32, device=dev)
            hy.hyena_encode_weights(ctx, d, w, wn)
            G = d.n_out // c

            def run(ev=None):
                ct.copy_(ct0)
                if ev:
                    ev[0].record()
                hy.hyena_ntt(ctx, ct)
                if ev:
                    ev[1].record()
                hy.hyena_conv(ctx, d, ct, wn, out)
                if not fuse and c > 1:
                    hy.hyena_wht_pack(ctx, c, out, out, G)
                if ev:
                    ev[2].record()
                hy.hyena_intt(ctx, out)
                if ev:
                    ev[3].record()

            out.fill_(0)
            run()
            torch.cuda.synchronize()
            o5 = out.view(d0.tiles, lay.Co, 2, L, N)
            samples[name] = [o5[t, oc].cpu().numpy().view(np.uint32).copy() for t, oc in sel]
            best = None
            for _ in range(max(3, args.steps)):
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
                run(ev)
                torch.cuda.synchronize()
                t = (ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3]))
                if best is None or sum(t) < sum(best):
                    best = t
            w_bytes = wn.numel() * 4
            io_bytes = (d.n_in + d.n_out) * 2 * L * N * 4
            mac_gbs = (w_bytes + io_bytes) / (best[1] * 1e-3) / 1e9
            row[name] = {"c_n": c, "butterflies": ("HYENA_FUSE_WHT" if fuse else "hyena_wht_pack") if c > 1 else None,
                         "ms": sum(best), "ntt_ms": best[0], "mac_ms": best[1], "intt_ms": best[2],
                         "coeff_macs_per_s": macs / (sum(best) * 1e-3),
                         "mac_coeff_macs_per_s": macs / (best[1] * 1e-3),
                         "mac_GBs": mac_gbs, "mac_hbm_frac": mac_gbs / HBM_PEAK_GBS,
                         "mac_algorithmic_bytes": w_bytes + io_bytes}
            del wn
        row["coeff_macs"] = macs
        rows.append(row)
        parity.append((lay, ct0.cpu().numpy().view(np.uint32).reshape(d0.tiles, d0.n_groups, 2, L, N).copy(),
                       w_host, sel, samples))
        log(f"  {row['layer']} c_n={cn}: {row['walsh']['ms']:.3f} ms (unfused {row['walsh_unfused']['ms']:.3f}, "
            f"c_n=1 {row['no_walsh']['ms']:.3f}); MAC {row['walsh']['mac_GBs']:.0f} GB/s")
        del ct0, ct, out
    primes = list(ctx.primes)
    hy.hyena_destroy(ctx)
    res = {"workload": "ImageNet ResNet layers 56x56x64->64 (c_n=4) and 14x14x256->256 (c_n=64), 3x3 pad 1, "
                       "1 image, N=16384, 4 primes < 2^31, lazy reduction",
           "layers": rows, "parity_checked_outputs": 0,
           "ms_walsh": sum(r["walsh"]["ms"] for r in rows),
           "ms_no_walsh": sum(r["no_walsh"]["ms"] for r in rows)}
    return res, (N, primes, parity)


def check_walsh_layers(orc, c3):
    """The oracle's products for the sampled outputs of walsh_layers; every
    variant must equal them on every coefficient."""
    N, primes, parity = c3
    checked = 0
    for lay, ct, w, sel, samples in parity:
        pl = orc.plan(N, lay.H, lay.W, lay.Ci, lay.Co, lay.k)
        want = orc.conv_products(pl, ct, w, primes, outputs=sel)
        for name, got in samples.items():
            for u, (tau, oc) in enumerate(sel):
                if not np.array_equal(got[u], want[u]):
                    raise SystemExit(f"parity failure: ResNet layer {lay.name} variant {name} output {(tau, oc)}")
                checked += 1
    log(f"parity ok: {checked} sampled output ciphertexts of the Walsh-packed ResNet layers")
    return checked


class PickedLayer:
    pass


def run_picks(hy, wl, torch, picks, n_img, steps, warmup, batched, sample=False):
    """MobileNetV1's 27 layers for n_img images, each computed with its picked
    parameters (ring degree, limbs, channels per ciphertext, Walsh group, path).
    batched: NTT-path layers sharing (N, L) run as one tuned batch object
    (persistent multiply-accumulate, hipGraph), direct-path layers as one
    hyena_conv_direct launch over all images; otherwise every image and layer
    is launched on its own (ntt, conv, intt). Returns the time per step and,
    with `sample`, the host copies the parity check needs."""
    from paper_2311_12519_amd import costmodel as cm
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    ctxs, items = {}, []
    for li, (lay, c) in enumerate(zip(wl.mobilenet_v1_layers(), picks)):
        if (c.N, c.L) not in ctxs:
            ctxs[(c.N, c.L)] = hy.hyena_create(c.N, c.L)
        ctx = ctxs[(c.N, c.L)]
        o = PickedLayer()
        o.lay, o.c, o.ctx = lay, c, ctx
        mk = dict(depthwise=lay.depthwise, c_n=c.c_n, ci_req=c.ci, flags=hy.HYENA_FUSE_WHT)
        o.d_b = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, batch=n_img, **mk)
        o.d_1 = hy.hyena_conv_plan(ctx, lay.H, lay.W, lay.Ci, lay.Co, lay.k, batch=1, **mk)
        LN = c.L * c.N
        o.in_w, o.out_w = o.d_1.n_in * 2 * LN, o.d_1.n_out * 2 * LN
        seed = wl.layer_seed(5, li)
        o.w_host = wl.weights(seed, lay)
        o.w = torch.from_numpy(o.w_host).to(dev)
        o.ct0 = torch.empty((n_img, o.in_w), dtype=torch.int32, device=dev)
        v = o.ct0.view(-1, c.L, c.N)
        gen.manual_seed(seed)
        for i, q in enumerate(ctx.primes):
            v[:, i, :] = torch.randint(0, q, v[:, i, :].shape, generator=gen, device=dev,
                                       dtype=torch.int64).to(torch.int32)
        o.ct = o.ct0.clone()
        o.out = torch.empty((n_img, o.out_w), dtype=torch.int32, device=dev)
        if not c.direct:
            o.wn = torch.empty(hy.wntt_words(ctx, o.d_b), dtype=torch.int32, device=dev)
            hy.hyena_encode_weights(ctx, o.d_b, o.w, o.wn)
        items.append(o)
    del cm
    batches = []
    if batched:
        flags = hy.HYENA_BATCH_TUNE | hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH
        for key, ctx in ctxs.items():
            group = [o for o in items if not o.c.direct and (o.c.N, o.c.L) == key]
            if group:
                batches.append(hy.hyena_batch_create(ctx, [(o.d_b, o.ct, o.wn, o.out) for o in group], flags))

    def step():
        if batched:
            for b in batches:
                hy.hyena_batch_run(b)
            for o in items:
                if o.c.direct:
                    hy.hyena_conv_direct(o.ctx, o.d_b, o.ct, o.w, o.out)
        else:
            for o in items:
                for b in range(n_img):
                    if o.c.direct:
                        hy.hyena_conv_direct(o.ctx, o.d_1, o.ct[b], o.w, o.out[b])
                    else:
                        hy.hyena_ntt(o.ctx, o.ct[b])
                        hy.hyena_conv(o.ctx, o.d_1, o.ct[b], o.wn, o.out[b])
                        hy.hyena_intt(o.ctx, o.out[b])

    samples = None
    if sample:
        for o in items:
            o.ct.copy_(o.ct0)
        torch.cuda.synchronize()
        step()
        torch.cuda.synchronize()
        samples = []
        for o in items:
            c, d = o.c, o.d_1
            o5 = o.out[0].view(d.tiles, o.lay.Co, 2, c.L, c.N)
            sel = [(0, 0), (d.tiles - 1, o.lay.Co - 1)]
            samples.append((o.lay, c, list(o.ctx.primes),
                            o.ct0[0].cpu().numpy().view(np.uint32).reshape(d.tiles, d.n_groups, 2, c.L, c.N).copy(),
                            o.w_host, sel, [o5[t, oc].cpu().numpy().view(np.uint32).copy() for t, oc in sel]))
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    for b in batches:
        hy.hyena_batch_destroy(b)
    for o in items:
        o.ct = o.ct0 = o.out = o.w = None
        o.wn = None
    for ctx in ctxs.values():
        hy.hyena_destroy(ctx)
    torch.cuda.empty_cache()
    return ms, samples


def mobilenet_costmodel(args, hy, wl, torch):
    """Supplementary figure: the learned cost model on MobileNetV1 (27 layers
    at 224x224). The model (FP32 MLP 8-64-64-1, trained on the GPU by the
    library's own kernels) is trained on timed samples of random layer shapes
    (never MobileNetV1's), then picks (N, L, c_i, c_n, path) for every layer
    among the secure, decryptable candidates; exhaustive timing of every
    candidate judges its regret, and the default parameters (N = 8192, fewest
    limbs, widest channel partition, c_n = 1, NTT path) its gain. End to end,
    8 images of the whole network run with the default parameters launched per
    image and layer (the plain path), and batched with the model's and with
    the exhaustive search's picks."""
    from paper_2311_12519_amd import costmodel as cm
    log(f"supplementary run: learned cost model on MobileNetV1 ({args.cm_shapes} training shapes) ...")
    t0 = time.perf_counter()
    rep = cm.run(train_shapes=args.cm_shapes, per_shape=4, steps=4000, seed=0, log=log)
    t_cm = time.perf_counter() - t0
    rows = rep["layers"]
    log(f"  {rep['train_samples']} samples, regret {rep['regret']:.4f}, gain over default "
        f"{rep['gain_over_default']:.3f} ({t_cm:.1f} s)")
    picks = {"model": [cm.Cand(**r["model"]) for r in rows],
             "exhaustive": [cm.Cand(**r["best"]) for r in rows],
             "default": [cm.Cand(**r["default"]) for r in rows]}
    n_img, steps = args.images, max(2, min(args.steps, 5))
    e2e = {"images": n_img, "layers": len(rows)}
    samples = {}
    for name, which, batched in [("default_plain", "default", False), ("default_batched", "default", True),
                                 ("model_batched", "model", True), ("exhaustive_batched", "exhaustive", True)]:
        want = name in ("default_plain", "model_batched") and not args.no_check
        ms, smp = run_picks(hy, wl, torch, picks[which], n_img, steps, 1, batched, sample=want)
        e2e[f"{name}_ms"] = ms
        if smp is not None:
            samples[name] = smp
        log(f"  MobileNetV1 x {n_img}: {name} {ms:.2f} ms")
    e2e["speedup_model_batched_vs_plain"] = e2e["default_plain_ms"] / e2e["model_batched_ms"]
    e2e["speedup_model_batched_vs_default_batched"] = e2e["default_batched_ms"] / e2e["model_batched_ms"]
    e2e["layers_per_s_model_batched"] = n_img * len(rows) / (e2e["model_batched_ms"] * 1e-3)
    e2e["parity_checked_outputs"] = 0
    res = {"workload": f"MobileNetV1 27 layers at 224x224; search N in {{4096, 8192, 16384}} x limbs meeting "
                       f"128-bit security x channel partitions x c_n in {{1, 2, 4}} x NTT/direct path",
           "mlp": rep["mlp"], "train_samples": rep["train_samples"], "train_shapes": rep["train_shapes"],
           "candidates": rep["candidates"], "regret": rep["regret"], "gain_over_default": rep["gain_over_default"],
           "total_best_ms": rep["total_best_ms"], "total_model_ms": rep["total_model_ms"],
           "total_default_ms": rep["total_default_ms"], "collect_s": rep["collect_s"], "train_s": rep["train_s"],
           "exhaustive_search_s": rep["exhaustive_search_s"], "model_search_s": rep["model_search_s"],
           "wall_s": t_cm, "end_to_end": e2e,
           "picks": [{"layer": lay.name, "model": r["model"], "exhaustive": r["best"], "model_ms": r["model_ms"],
                      "best_ms": r["best_ms"], "default_ms": r["default_ms"]}
                     for lay, r in zip(wl.mobilenet_v1_layers(), rows)]}
    return res, samples


def check_mobilenet(orc, samples):
    """The oracle's products for the sampled outputs of the MobileNetV1 runs
    (default parameters per image, the model's picks batched)."""
    checked = 0
    for name, smp in samples.items():
        for lay, c, primes, ct, w, sel, got in smp:
            pl = orc.plan(c.N, lay.H, lay.W, lay.Ci, lay.Co, lay.k, lay.depthwise, c.ci)
            want = orc.conv_products(pl, ct, w, primes, outputs=sel)
            for u, (tau, oc) in enumerate(sel):
                if not np.array_equal(got[u], want[u]):
                    raise SystemExit(f"parity failure: MobileNetV1 {name} layer {lay.name} output {(tau, oc)}")
                checked += 1
    log(f"parity ok: {checked} sampled MobileNetV1 output ciphertexts")
    return checked


def alt_primes(args, hy, wl, torch, layers31, n_img, total_macs):
    """Supplementary figure: the same workload and tuned path with three primes
    below 2^30 (Harvey's lazy NTT butterflies, 15 products per fold); the
    headline stays on the largest primes below 2^31. Returns the figure and the
    parity set for the cpu_baseline leg."""
    import argparse
    for o in layers31:   # release the first run's buffers
        o.ct = o.ct0 = o.out = o.d_wn = o.d_w = o.d_taps = None
    torch.cuda.empty_cache()
    a = argparse.Namespace(**vars(args))
    a.primes = 30
    log("supplementary run: primes below 2^30 ...")
    ctx, layers = setup(a, hy, wl, torch)
    flags = hy.HYENA_BATCH_TUNE | hy.HYENA_BATCH_PERSISTENT | hy.HYENA_BATCH_GRAPH | hy.HYENA_BATCH_TIMING
    batch = hy.hyena_batch_create(ctx, [(o.desc_b, o.ct, o.d_wn, o.out) for o in layers], flags)
    parity = []
    if not args.no_check:
        parity.append((sampled_inputs(ctx, layers, n_img), ctx.primes,
                       {"tuned": sample_outputs(ctx, layers, torch, n_img, lambda: hy.hyena_batch_run(batch))}))
    for _ in range(args.warmup):
        hy.hyena_batch_run(batch)
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        hy.hyena_batch_run(batch)
        phases.append(hy.hyena_batch_phase_ms(batch))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ph = np.array(phases).mean(axis=0)
    log(f"primes < 2^30: {dt * 1e3:.2f} ms/step")
    return ({"ms_per_step": dt * 1e3, "coeff_macs_per_s": total_macs / dt, "primes": ctx.primes,
             "kernels_ms": {"ntt": float(ph[0]), "mac": float(ph[1]), "intt": float(ph[2])},
             "parity_checked_outputs": 0, "schedules": hy.hyena_batch_info(batch)}, parity)


if __name__ == "__main__":
    main()
