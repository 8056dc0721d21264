"""Seeded parameter sets for the guess network (host side, float64).

Tensor names and shapes (torch-style conv layout [out, in, ky, kx]):

    conv1.w [C, 2, 3, 3]   conv1.b [C]
    conv2.w [C, C, 3, 3]   conv2.b [C]
    spec.w1 [C, C]         spec.b  [C]      (1x1 skip path of the spectral layer)
    spec.wk [M, M, C, C]                    (per-mode channel mixing, [ky, kx, out, in])
    conv4.w [C, C, 3, 3]   conv4.b [C]
    conv5.w [C, C, 3, 3]   conv5.b [C]
    conv6.w [1, C, 3, 3]   conv6.b [1]
    band.w  [K, K]                          (per-mode weights of the band path; absent for K = 0)

Weights are uniform in +-sqrt(6 / fan_in) (He-uniform); biases are drawn in
+-0.1 when ``random_bias`` is set (tests) and are zero otherwise; the band
weights are uniform in [0, 1).  With ``zero_last`` the output layer and the
band weights start at zero, so the untrained network returns the previous
solution unchanged.
"""
from __future__ import annotations

import numpy as np

PARAM_ORDER = ("conv1.w", "conv1.b", "conv2.w", "conv2.b", "spec.w1", "spec.b",
               "spec.wk", "conv4.w", "conv4.b", "conv5.w", "conv5.b",
               "conv6.w", "conv6.b", "band.w")


def param_shapes(channels: int = 32, modes: int = 16, skip_modes: int | None = None) -> dict:
    C, M = channels, modes
    K = M if skip_modes is None else skip_modes
    return {
        "conv1.w": (C, 2, 3, 3), "conv1.b": (C,),
        "conv2.w": (C, C, 3, 3), "conv2.b": (C,),
        "spec.w1": (C, C), "spec.b": (C,),
        "spec.wk": (M, M, C, C),
        "conv4.w": (C, C, 3, 3), "conv4.b": (C,),
        "conv5.w": (C, C, 3, 3), "conv5.b": (C,),
        "conv6.w": (1, C, 3, 3), "conv6.b": (1,),
        "band.w": (K, K),
    }


def guess_net_params(seed: int, channels: int = 32, modes: int = 16,
                     zero_last: bool = False, random_bias: bool = True,
                     skip_modes: int | None = None) -> dict:
    rng = np.random.default_rng(seed)
    out = {}
    for name in PARAM_ORDER:
        shape = param_shapes(channels, modes, skip_modes)[name]
        if name == "band.w" and shape[0] == 0:
            continue
        if name.endswith(".b"):
            out[name] = (rng.uniform(-0.1, 0.1, size=shape) if random_bias
                         else np.zeros(shape))
            continue
        if name == "band.w":
            out[name] = rng.uniform(0.0, 1.0, size=shape)
            continue
        if name == "spec.wk":
            fan_in = 2 * shape[3]
        elif name == "spec.w1":
            fan_in = 2 * shape[1]
        else:
            fan_in = shape[1] * shape[2] * shape[3]
        bound = np.sqrt(6.0 / fan_in)
        out[name] = rng.uniform(-bound, bound, size=shape)
    if zero_last:
        out["conv6.w"] = np.zeros_like(out["conv6.w"])
        out["conv6.b"] = np.zeros_like(out["conv6.b"])
        if "band.w" in out:
            out["band.w"] = np.zeros_like(out["band.w"])
    return out


def fluid_net_params(seed: int, channels: int = 32, levels: int = 4, max_blocks: int = 2,
                     random_bias: bool = True, zero_last: bool = False,
                     zero_block_out: bool = True) -> dict:
    """Seeded parameters of the multi-scale (pooling pyramid) guess network, in
    its tensor order: per level conv1.w [C, 2, 3, 3], conv1.b, conv2.w
    [C, C, 3, 3], conv2.b; per residual block a.w, a.b, b.w, b.b ([C, C, 3, 3],
    [C]); head.conv1.w [C, C, 3, 3], head.conv1.b, head.conv2.w [1, C, 3, 3],
    head.conv2.b [1].  He-uniform weights, biases in +-0.1 when
    ``random_bias``; with ``zero_block_out`` every block's second convolution
    (weights and bias) is zero, with ``zero_last`` the output layer is."""
    rng = np.random.default_rng(seed)
    C = channels
    out = {}
    for l in range(levels):
        out[f"lvl{l}.conv1.w"], out[f"lvl{l}.conv1.b"] = _conv(rng, C, 2, random_bias)
        out[f"lvl{l}.conv2.w"], out[f"lvl{l}.conv2.b"] = _conv(rng, C, C, random_bias)
    for i in range(max_blocks):
        out[f"blk{i}.a.w"], out[f"blk{i}.a.b"] = _conv(rng, C, C, random_bias)
        out[f"blk{i}.b.w"], out[f"blk{i}.b.b"] = _conv(rng, C, C, random_bias)
        if zero_block_out:
            out[f"blk{i}.b.w"] = np.zeros_like(out[f"blk{i}.b.w"])
            out[f"blk{i}.b.b"] = np.zeros_like(out[f"blk{i}.b.b"])
    out["head.conv1.w"], out["head.conv1.b"] = _conv(rng, C, C, random_bias)
    out["head.conv2.w"], out["head.conv2.b"] = _conv(rng, 1, C, random_bias)
    if zero_last:
        out["head.conv2.w"] = np.zeros_like(out["head.conv2.w"])
        out["head.conv2.b"] = np.zeros_like(out["head.conv2.b"])
    return out


def _conv(rng, cout: int, cin: int, random_bias: bool):
    bound = np.sqrt(6.0 / (9 * cin))
    w = rng.uniform(-bound, bound, size=(cout, cin, 3, 3))
    b = rng.uniform(-0.1, 0.1, size=(cout,)) if random_bias else np.zeros(cout)
    return w, b
