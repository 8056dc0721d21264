"""NumPy FP64 oracle for the multi-scale guess network (test infrastructure only).

Section 2.1 of the paper describes its best network as a variant of the
FluidNet pressure model: the input is average-pooled 2^d-wise several times
(the number of poolings set by the problem), the original and every pooled
field pass through their own convolution layers in parallel, all are upsampled
back to the full resolution and summed, and the sum goes through output
convolutions; residual blocks are stacked before the output layer, appended
one at a time while training runs (a shallow model first, deeper when its
progress stagnates).  The paper gives no layer sizes; the network built here
(readings listed in the design notes):

  inputs   (r / s_r, f / s_f), the same normalised pair as the spectral
           network (r = f - A u_prev in FP64; `oracle.net.normalise`)
  pyramid  X_0 = input, X_l = avgpool2(X_{l-1}), l = 1 .. L-1
  branch l a_l = ReLU(conv3x3_{2->C}(X_l)); y_l = ReLU(conv3x3_{C->C}(a_l))
  sum      S_0 = sum_l up_l(y_l), up_l the nearest-neighbour 2^l x 2^l upsampling
  block i  h_i = ReLU(conv3x3(S_{i-1})); S_i = S_{i-1} + conv3x3(h_i), i = 1 .. R
  head     o = ReLU(conv3x3(S_R)); out = conv3x3_{C->1}(o)
  guess    u_prev + (s_r / c_u) out
The second convolution of a block starts at zero, so a new block is the
identity and appending it leaves the output unchanged.  Everything is
float64, NCHW, with `oracle.net.conv3x3` (zero padding, [out, in, ky, kx]).
"""
from __future__ import annotations

import numpy as np

from .net import C_U, conv3x3, conv3x3_backward, normalise, target


def tensor_names(levels: int, max_blocks: int) -> list:
    """Tensor order of a parameter set (the GPU layout uses the same order)."""
    names = []
    for l in range(levels):
        names += [f"lvl{l}.conv1.w", f"lvl{l}.conv1.b", f"lvl{l}.conv2.w", f"lvl{l}.conv2.b"]
    for i in range(max_blocks):
        names += [f"blk{i}.a.w", f"blk{i}.a.b", f"blk{i}.b.w", f"blk{i}.b.b"]
    names += ["head.conv1.w", "head.conv1.b", "head.conv2.w", "head.conv2.b"]
    return names


def tensor_shapes(channels: int, levels: int, max_blocks: int) -> dict:
    C = channels
    out = {}
    for name in tensor_names(levels, max_blocks):
        if name.endswith(".b"):
            out[name] = (1,) if name == "head.conv2.b" else (C,)
        elif name.endswith("conv1.w") and name.startswith("lvl"):
            out[name] = (C, 2, 3, 3)
        elif name == "head.conv2.w":
            out[name] = (1, C, 3, 3)
        else:
            out[name] = (C, C, 3, 3)
    return out


def avgpool2(x: np.ndarray) -> np.ndarray:
    """[B, C, H, W] -> [B, C, H/2, W/2]: the mean of each 2 x 2 block."""
    B, C, H, W = x.shape
    return x.reshape(B, C, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def upsample(y: np.ndarray, k: int) -> np.ndarray:
    """Nearest-neighbour upsampling by k along both axes: out[i, j] = y[i // k, j // k]."""
    return np.repeat(np.repeat(y, k, axis=2), k, axis=3)


def upsample_adjoint(z: np.ndarray, k: int) -> np.ndarray:
    """The adjoint of `upsample`: the sum of each k x k block."""
    B, C, H, W = z.shape
    return z.reshape(B, C, H // k, k, W // k, k).sum(axis=(3, 5))


def relu(x):
    return np.maximum(x, 0.0)


def forward(params: dict, f: np.ndarray, u_prev: np.ndarray, levels: int, blocks: int,
            keep: bool = False):
    """f, u_prev: [B, H, W] float64 (H, W divisible by 2^(levels-1)); `blocks`
    active residual blocks.  Returns (guess, out, s_in[, cache])."""
    x0, s_r, s = normalise(f, u_prev)
    X = [x0]
    for _ in range(1, levels):
        X.append(avgpool2(X[-1]))
    A, Y = [], []
    S = np.zeros((x0.shape[0], params["lvl0.conv2.w"].shape[0]) + x0.shape[2:])
    for l in range(levels):
        a = relu(conv3x3(X[l], params[f"lvl{l}.conv1.w"], params[f"lvl{l}.conv1.b"]))
        y = relu(conv3x3(a, params[f"lvl{l}.conv2.w"], params[f"lvl{l}.conv2.b"]))
        A.append(a)
        Y.append(y)
        S = S + upsample(y, 2 ** l)
    Ss, H = [S], []
    for i in range(blocks):
        h = relu(conv3x3(Ss[-1], params[f"blk{i}.a.w"], params[f"blk{i}.a.b"]))
        H.append(h)
        Ss.append(Ss[-1] + conv3x3(h, params[f"blk{i}.b.w"], params[f"blk{i}.b.b"]))
    o = relu(conv3x3(Ss[-1], params["head.conv1.w"], params["head.conv1.b"]))
    out = conv3x3(o, params["head.conv2.w"], params["head.conv2.b"])[:, 0]
    guess = u_prev + (s_r / C_U)[:, None, None] * out
    if keep:
        return guess, out, s, {"X": X, "A": A, "Y": Y, "S": Ss, "H": H, "o": o}
    return guess, out, s


def loss_and_grads(params: dict, f, u_prev, u_target, levels: int, blocks: int):
    """L = (1/B) sum_b |out_b - t_b|_2^2 (t: the solution in output units) and
    its gradient for every parameter of the active part of the network."""
    B = f.shape[0]
    _, out, s, c = forward(params, f, u_prev, levels, blocks, keep=True)
    diff = out - target(u_target, u_prev, s)
    loss = float(np.sum(diff ** 2) / B)
    g = {}
    d = (2.0 / B) * diff[:, None]
    do, g["head.conv2.w"], g["head.conv2.b"] = conv3x3_backward(c["o"], params["head.conv2.w"], d)
    do = do * (c["o"] > 0.0)
    dS, g["head.conv1.w"], g["head.conv1.b"] = conv3x3_backward(c["S"][-1], params["head.conv1.w"], do)
    for i in reversed(range(blocks)):
        dh, g[f"blk{i}.b.w"], g[f"blk{i}.b.b"] = conv3x3_backward(c["H"][i], params[f"blk{i}.b.w"], dS)
        dh = dh * (c["H"][i] > 0.0)
        dprev, g[f"blk{i}.a.w"], g[f"blk{i}.a.b"] = conv3x3_backward(c["S"][i], params[f"blk{i}.a.w"], dh)
        dS = dS + dprev
    for l in range(levels):
        dy = upsample_adjoint(dS, 2 ** l) * (c["Y"][l] > 0.0)
        da, g[f"lvl{l}.conv2.w"], g[f"lvl{l}.conv2.b"] = conv3x3_backward(
            c["A"][l], params[f"lvl{l}.conv2.w"], dy)
        da = da * (c["A"][l] > 0.0)
        _, g[f"lvl{l}.conv1.w"], g[f"lvl{l}.conv1.b"] = conv3x3_backward(
            c["X"][l], params[f"lvl{l}.conv1.w"], da)
    return loss, g
