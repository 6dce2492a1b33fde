"""Seeded synthetic inputs for the Hyena homomorphic-convolution path.

This module only draws data and lists layer shapes. It holds none of the
method's arithmetic (no encoding, no modular arithmetic, no transforms), so
both the oracle and the GPU-side tests and benchmark can use it without
sharing any computation.

Value recipe. Activations and weights are uniform signed 4-bit integers in
[-8, 7], drawn with ``numpy.random.default_rng(seed)``. The paper evaluates on
trained ImageNet CNNs (VGG-16, ResNet, MobileNetV1; the "Evaluation
Setup" section); neither the dataset nor trained weights are available here, so the
layer *shapes* of those networks are used with synthetic values of the small
integer width the paper's kernels carry (kernel elements below 8 bits,
the "Optimal Parameter Selection" section).

Seeds. ``seed = 1000 * workload_id + layer_index``; image ``b`` of a batch uses
``seed + 100 * b``; key generation and encryption use ``seed ^ 0x5EED``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

VMIN, VMAX = -8, 7  # signed 4-bit


@dataclass(frozen=True)
class Layer:
    """One convolution layer: square H x W input, Ci -> Co, k x k kernel.

    ``stride`` is the CNN's stride; the encrypted computation is always the
    stride-1 convolution, subsampled after decryption. ``depthwise`` layers
    have Co == Ci and one k x k filter per channel.
    """
    name: str
    H: int
    W: int
    Ci: int
    Co: int
    k: int = 3
    stride: int = 1
    depthwise: bool = False


@dataclass(frozen=True)
class Workload:
    wid: int
    name: str
    N: int
    L: int
    prime_bits: int
    layers: tuple
    images: int = 1
    c_n: tuple = field(default_factory=tuple)  # per-layer Walsh group size (empty: 1)


def activations(seed: int, C: int, H: int, W: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(VMIN, VMAX + 1, size=(C, H, W), dtype=np.int64).astype(np.int8)


def weights(seed: int, layer: Layer) -> np.ndarray:
    """int8 [Co][Ci][k][k], or [C][1][k][k] for depthwise layers."""
    rng = np.random.default_rng(seed ^ 0x3EA7)
    cin = 1 if layer.depthwise else layer.Ci
    return rng.integers(VMIN, VMAX + 1, size=(layer.Co, cin, layer.k, layer.k),
                        dtype=np.int64).astype(np.int8)


def layer_seed(wid: int, layer_idx: int, image: int = 0) -> int:
    return 1000 * wid + layer_idx + 100 * image


def crypto_seed(seed: int) -> int:
    return seed ^ 0x5EED


def random_residues(seed: int, shape, primes) -> np.ndarray:
    """Uniform residues in [0, q_i) along axis -2 (limb axis) for raw-throughput
    inputs whose values need not be encryptions (timing samples)."""
    rng = np.random.default_rng(seed)
    shape = tuple(shape)
    out = np.empty(shape, dtype=np.uint32)
    for i, q in enumerate(primes):
        out[..., i, :] = rng.integers(0, q, size=shape[:-2] + (shape[-1],), dtype=np.uint64)
    return out


# ---------------------------------------------------------------------------
# Layer tables (standard published architectures; shapes only)
# ---------------------------------------------------------------------------

def vgg16_layers(res: int = 224):
    widths = [(64, 2), (128, 2), (256, 3), (512, 3), (512, 3)]
    out, cin, h = [], 3, res
    for stage, (w, n) in enumerate(widths):
        for j in range(n):
            out.append(Layer(f"conv{stage + 1}_{j + 1}", h, h, cin, w, 3))
            cin = w
        h //= 2
    return tuple(out)


def mobilenet_v1_layers(res: int = 224):
    out = [Layer("conv0", res, res, 3, 32, 3, stride=2)]
    h, c = res // 2, 32
    plan = [(64, 1), (128, 2), (128, 1), (256, 2), (256, 1), (512, 2),
            (512, 1), (512, 1), (512, 1), (512, 1), (512, 1), (1024, 2), (1024, 1)]
    for i, (co, s) in enumerate(plan):
        out.append(Layer(f"dw{i + 1}", h, h, c, c, 3, stride=s, depthwise=True))
        h = h // s
        out.append(Layer(f"pw{i + 1}", h, h, c, co, 1))
        c = co
    return tuple(out)


WORKLOADS = {
    1: Workload(1, "single 16x16x16->16 3x3 layer", 4096, 2, 30,
                (Layer("l16", 16, 16, 16, 16, 3),)),
    2: Workload(2, "ResNet-20 CIFAR layer 32x32x16->32", 8192, 3, 31,
                (Layer("res32", 32, 32, 16, 32, 3),)),
    3: Workload(3, "ImageNet ResNet layers", 16384, 4, 31,
                (Layer("res56", 56, 56, 64, 64, 3), Layer("res14", 14, 14, 256, 256, 3)),
                c_n=(4, 64)),
    4: Workload(4, "VGG-16 13 conv layers at 224, 8 images", 8192, 3, 31,
                vgg16_layers(), images=8),
    5: Workload(5, "MobileNetV1 27 layers at 224", 8192, 3, 31, mobilenet_v1_layers()),
}
