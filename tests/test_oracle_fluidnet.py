"""Pins of the multi-scale (pooling pyramid) guess network oracle.

Checked against: torch's CPU float64 avg_pool2d / interpolate(nearest) /
conv2d with autograd (forward values and every gradient), central finite
differences, the adjoint identity of nearest upsampling and block summation,
the mean of a constant, and the identity start of a residual block whose
second convolution is zero (the property block growth relies on)."""
import numpy as np
import pytest
import torch

from oracle import fluidnet as fn
from oracle import net
from synthetic import fluid_net_params


def small(C=4, L=3, R=2, seed=0, **kw):
    return fluid_net_params(seed, channels=C, levels=L, max_blocks=R, **kw)


def inputs(B, H, W, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((B, H, W))
    u = rng.standard_normal((B, H, W)) * 0.05
    ut = u + rng.standard_normal((B, H, W)) * 0.05
    return f, u, ut


def test_pool_and_upsample_pins():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 8, 12))
    assert np.allclose(fn.avgpool2(np.full((1, 2, 6, 4), 2.5)), 2.5, rtol=0, atol=0)
    ref = torch.nn.functional.avg_pool2d(torch.from_numpy(x), 2).numpy()
    assert np.allclose(fn.avgpool2(x), ref, rtol=1e-15, atol=1e-15)
    y = rng.standard_normal((2, 3, 2, 3))
    up = torch.nn.functional.interpolate(torch.from_numpy(y), scale_factor=4, mode="nearest").numpy()
    assert np.array_equal(fn.upsample(y, 4), up)
    z = rng.standard_normal((2, 3, 8, 12))
    # <up(y), z> = <y, up^T(z)>
    assert np.isclose(np.sum(fn.upsample(y, 4) * z), np.sum(y * fn.upsample_adjoint(z, 4)), rtol=1e-13)


def torch_forward(p, f, u, levels, blocks):
    """The same network from torch's library routines (float64, autograd)."""
    F = torch.nn.functional
    x0, s_r, s = net.normalise(f, u)
    T = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    x = torch.tensor(x0)
    S = 0.0
    xl = x
    for l in range(levels):
        if l:
            xl = F.avg_pool2d(xl, 2)
        a = F.relu(F.conv2d(xl, T[f"lvl{l}.conv1.w"], T[f"lvl{l}.conv1.b"], padding=1))
        y = F.relu(F.conv2d(a, T[f"lvl{l}.conv2.w"], T[f"lvl{l}.conv2.b"], padding=1))
        S = S + (F.interpolate(y, scale_factor=2 ** l, mode="nearest") if l else y)
    for i in range(blocks):
        h = F.relu(F.conv2d(S, T[f"blk{i}.a.w"], T[f"blk{i}.a.b"], padding=1))
        S = S + F.conv2d(h, T[f"blk{i}.b.w"], T[f"blk{i}.b.b"], padding=1)
    o = F.relu(F.conv2d(S, T["head.conv1.w"], T["head.conv1.b"], padding=1))
    out = F.conv2d(o, T["head.conv2.w"], T["head.conv2.b"], padding=1)[:, 0]
    return T, out, s


@pytest.mark.parametrize("levels,blocks", [(1, 0), (3, 2), (2, 1)])
def test_forward_and_gradients_match_torch(levels, blocks):
    p = small(L=3, R=2, seed=levels + blocks, zero_block_out=False)
    f, u, ut = inputs(2, 8, 12, seed=5)
    _, out, s = fn.forward(p, f, u, levels, blocks)
    T, tout, ts = torch_forward(p, f, u, levels, blocks)
    assert np.allclose(out, tout.detach().numpy(), rtol=1e-12, atol=1e-12)
    t = torch.tensor(net.target(ut, u, s))
    loss = torch.sum((tout - t) ** 2) / f.shape[0]
    loss.backward()
    L, g = fn.loss_and_grads(p, f, u, ut, levels, blocks)
    assert abs(L - float(loss.detach())) <= 1e-12 * L
    for name in g:
        assert np.allclose(g[name], T[name].grad.numpy(), rtol=1e-10, atol=1e-12 * np.abs(g[name]).max()), name
    # inactive levels' and blocks' tensors get no gradient
    active = set(g)
    for name in p:
        if name not in active:
            assert T[name].grad is None or float(T[name].grad.abs().max()) == 0.0, name


def test_gradients_match_finite_differences():
    p = small(C=3, L=2, R=1, seed=3, zero_block_out=False)
    f, u, ut = inputs(2, 4, 6, seed=9)
    rng = np.random.default_rng(4)
    L, g = fn.loss_and_grads(p, f, u, ut, 2, 1)
    eps = 1e-6
    for name in g:
        d = rng.standard_normal(p[name].shape)
        pp = {k: v.copy() for k, v in p.items()}
        pm = {k: v.copy() for k, v in p.items()}
        pp[name] = p[name] + eps * d
        pm[name] = p[name] - eps * d
        fd = (fn.loss_and_grads(pp, f, u, ut, 2, 1)[0] - fn.loss_and_grads(pm, f, u, ut, 2, 1)[0]) / (2 * eps)
        an = float(np.sum(g[name] * d))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * abs(L)), name


def test_new_block_starts_as_identity():
    """A block whose second convolution is zero adds nothing: growing the
    network by one block leaves its output unchanged, and the new block's
    second convolution is the only block tensor with a gradient."""
    p = small(L=3, R=2, seed=7)
    f, u, ut = inputs(1, 8, 8, seed=2)
    o0 = fn.forward(p, f, u, 3, 0)[1]
    o1 = fn.forward(p, f, u, 3, 1)[1]
    o2 = fn.forward(p, f, u, 3, 2)[1]
    assert np.array_equal(o0, o1) and np.array_equal(o0, o2)
    _, g = fn.loss_and_grads(p, f, u, ut, 3, 1)
    assert np.abs(g["blk0.b.w"]).max() > 0
    assert np.abs(g["blk0.a.w"]).max() == 0


def test_untrained_output_layer_returns_previous_solution():
    p = small(seed=8, zero_last=True)
    f, u, _ = inputs(2, 8, 8, seed=3)
    guess, out, _ = fn.forward(p, f, u, 3, 2)
    assert np.array_equal(out, np.zeros_like(out)) and np.array_equal(guess, u)


def test_single_level_is_a_plain_cnn():
    """L = 1, no blocks: conv-ReLU-conv-ReLU-conv-ReLU-conv, written out with
    a direct sum for the 3x3 correlation."""
    p = small(C=2, L=1, R=0, seed=11)
    f, u, _ = inputs(1, 5, 4, seed=6)
    x0, _, _ = net.normalise(f, u)

    def conv(x, w, b):
        Ci, H, W = x.shape
        y = np.zeros((w.shape[0], H, W))
        for d in range(w.shape[0]):
            for i in range(H):
                for j in range(W):
                    acc = b[d]
                    for c in range(Ci):
                        for pp in range(3):
                            for q in range(3):
                                ii, jj = i + pp - 1, j + q - 1
                                if 0 <= ii < H and 0 <= jj < W:
                                    acc += w[d, c, pp, q] * x[c, ii, jj]
                    y[d, i, j] = acc
        return y
    a = np.maximum(conv(x0[0], p["lvl0.conv1.w"], p["lvl0.conv1.b"]), 0)
    y = np.maximum(conv(a, p["lvl0.conv2.w"], p["lvl0.conv2.b"]), 0)
    o = np.maximum(conv(y, p["head.conv1.w"], p["head.conv1.b"]), 0)
    ref = conv(o, p["head.conv2.w"], p["head.conv2.b"])[0]
    assert np.allclose(fn.forward(p, f, u, 1, 0)[1][0], ref, rtol=1e-13, atol=1e-13)
