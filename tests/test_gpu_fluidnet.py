"""GPU parity of the multi-scale guess network (forward, gradients, Adam,
block growth) against the NumPy FP64 oracle.

BF16 weights and activations with FP32 accumulation against FP64 on the same
BF16-rounded weights.  Bars, from BF16's unit roundoff 2^-8 compounded over
the layers a value passes (pyramid level, two branch convolutions, the sum,
two per block, two in the head; at most 9 here): (1 + 2^-8)^9 - 1 = 3.6e-2 on
the network correction relative to its norm; gradients within 5e-2 relative
L2 with cosine >= 0.998 per tensor; loss within 2e-2.  Blocks beyond the
active count have exactly zero gradient and do not move; a block whose second
convolution is zero leaves the output bitwise unchanged.
"""
import numpy as np
import pytest
import torch

from oracle import fluidnet as ofn
from oracle import gmres as og
from synthetic import DriftingGaussians, RandomDipoles, fluid_net_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlg():
    import paper_2103_10975_amd as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return m


def bf16_round(p):
    return {k: torch.as_tensor(v).to(torch.bfloat16).to(torch.float64).numpy() for k, v in p.items()}


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_params(mlg, cfg, p):
    buf = torch.zeros(mlg.fluid_net_param_bytes(cfg), dtype=torch.uint8, device="cuda")
    mlg.net_views(cfg, buf)["master"].copy_(mlg.fluid_pack(cfg, p).cuda())
    mlg.fluid_net_refresh(cfg, buf)
    torch.cuda.synchronize()
    return buf


def inputs(shape, B, seed):
    g = RandomDipoles(shape, seed=seed)
    f = np.stack([g.field(t + 1) for t in range(B)])
    u = np.stack([og.gmres(g.field(t), m=20, rtol=1e-6)[0] for t in range(B)])
    ut = np.stack([og.gmres(g.field(t + 1), m=20, rtol=1e-8)[0] for t in range(B)])
    return f, u, ut


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("shape,L,R,blocks,B", [((64, 64), 4, 2, 2, 2), ((40, 72), 3, 2, 1, 1),
                                                ((96, 136), 4, 1, 0, 3), ((256, 256), 6, 1, 1, 1)])
def test_forward_parity(mlg, shape, L, R, blocks, B):
    print("fluid forward", shape, L, R, blocks, B, flush=True)
    cfg = mlg.FluidCfg(levels=L, max_blocks=R)
    p = bf16_round(fluid_net_params(3 + L, channels=32, levels=L, max_blocks=R, zero_block_out=False))
    buf = make_params(mlg, cfg, p)
    f, u, _ = inputs(shape, B, 40 + L)
    guess = torch.empty_like(dev(f))
    ws = mlg.workspace(mlg.fluid_net_workspace_bytes(cfg, mlg.grid_of(shape), B, False))
    mlg.fluid_net_infer(cfg, buf, blocks, dev(f), dev(u), guess, ws)
    torch.cuda.synchronize()
    go, _, _ = ofn.forward(p, f, u, L, blocks)
    err = rel(guess.cpu().numpy() - u, go - u)
    print(f"  correction rel. error {err:.2e}")
    assert err <= 3.6e-2


@pytest.mark.parametrize("shape,L,R,blocks,B", [((32, 64), 3, 2, 2, 2), ((48, 40), 4, 2, 1, 1)])
def test_train_step_gradients_and_adam(mlg, shape, L, R, blocks, B):
    print("fluid train", shape, L, R, blocks, B, flush=True)
    cfg = mlg.FluidCfg(levels=L, max_blocks=R, lr=1e-3)
    p = bf16_round(fluid_net_params(11 + L, channels=32, levels=L, max_blocks=R,
                                    zero_block_out=False))
    buf = make_params(mlg, cfg, p)
    views = mlg.net_views(cfg, buf)
    master0 = views["master"].clone()
    f, u, ut = inputs(shape, B, 70 + L)
    ws = mlg.workspace(mlg.fluid_net_workspace_bytes(cfg, mlg.grid_of(shape), B, True))
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    mlg.fluid_net_train_step(cfg, buf, blocks, list(dev(f)), list(dev(u)), list(dev(ut)), ws, loss)
    torch.cuda.synchronize()
    Lo, go = ofn.loss_and_grads(p, f, u, ut, L, blocks)
    print(f"  loss gpu {loss.item():.6e} oracle {Lo:.6e}")
    assert abs(loss.item() - Lo) <= 2e-2 * Lo
    gg = mlg.fluid_unpack(cfg, views["grad"])
    for k in mlg.fluid_tensor_names(cfg):
        a = gg[k].numpy().ravel()
        if k not in go:                       # an inactive block
            assert np.all(a == 0), k
            continue
        b = go[k].ravel()
        e = rel(a, b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
        print(f"  grad {k:14s} rel {e:.2e} cos {cos:.5f}")
        assert e <= 5e-2 and cos >= 0.998, k
    g32 = views["grad"]
    expect = master0 - cfg.lr * g32 / (g32.abs() + cfg.eps)
    assert torch.allclose(views["master"], expect, rtol=1e-6, atol=1e-9)
    assert int(views["step"].item()) == 1
    assert torch.equal(views["bf16"], views["master"].to(torch.bfloat16))


def test_init_and_block_growth_start_as_identity(mlg):
    """The initialised network returns u_prev; after training, appending a
    block (zero second convolution) leaves the guess bitwise unchanged."""
    print("fluid init and growth", flush=True)
    cfg = mlg.FluidCfg(levels=3, max_blocks=2, seed=99)
    buf = torch.zeros(mlg.fluid_net_param_bytes(cfg), dtype=torch.uint8, device="cuda")
    mlg.fluid_net_init(cfg, buf)
    buf2 = torch.zeros_like(buf)
    mlg.fluid_net_init(cfg, buf2)
    torch.cuda.synchronize()
    assert torch.equal(buf, buf2)
    t = mlg.fluid_unpack(cfg, mlg.net_views(cfg, buf)["master"])
    for k, v in t.items():
        zero = k.endswith(".b") or ".b.w" in k or k == "head.conv2.w"
        if zero:
            assert torch.all(v == 0), k
        else:
            fan = 9 * v.shape[1]
            bound = np.sqrt(6.0 / fan)
            assert v.abs().max() <= bound and v.std() > 0.3 * bound, k
    shape = (48, 48)
    f, u, ut = inputs(shape, 2, 5)
    fd, ud, td = dev(f), dev(u), dev(ut)
    ws_i = mlg.workspace(mlg.fluid_net_workspace_bytes(cfg, mlg.grid_of(shape), 2, False))
    g0 = torch.empty_like(fd)
    mlg.fluid_net_infer(cfg, buf, 0, fd, ud, g0, ws_i)
    torch.cuda.synchronize()
    assert torch.equal(g0, ud)
    ws_t = mlg.workspace(mlg.fluid_net_workspace_bytes(cfg, mlg.grid_of(shape), 2, True))
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for _ in range(60):
        mlg.fluid_net_train_step(cfg, buf, 0, list(fd), list(ud), list(td), ws_t, loss)
        hist.append(loss.item())
    print("  loss", hist[0], hist[-1])
    assert hist[-1] < 0.5 * hist[0]
    g1, g2 = torch.empty_like(fd), torch.empty_like(fd)
    mlg.fluid_net_infer(cfg, buf, 0, fd, ud, g1, ws_i)
    mlg.fluid_net_infer(cfg, buf, 1, fd, ud, g2, ws_i)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and not torch.equal(g1, ud)
    # a step with the new block active moves its second convolution only as
    # far as Adam's first step allows, and keeps the second block untouched
    v = mlg.net_views(cfg, buf)
    before = mlg.fluid_unpack(cfg, v["master"])
    mlg.fluid_net_train_step(cfg, buf, 1, list(fd), list(ud), list(td), ws_t, loss)
    torch.cuda.synchronize()
    after = mlg.fluid_unpack(cfg, v["master"])
    assert not torch.equal(before["blk0.b.w"], after["blk0.b.w"])
    assert torch.equal(before["blk1.a.w"], after["blk1.a.w"])
    assert torch.equal(before["blk1.b.w"], after["blk1.b.w"])


def test_argument_errors(mlg):
    cfg = mlg.FluidCfg(levels=4, max_blocks=1)
    with pytest.raises(mlg.MlgError):
        mlg.fluid_net_workspace_bytes(cfg, mlg.grid_of((60, 64)), 1, False)   # 60 % 8 != 0
    buf = torch.zeros(mlg.fluid_net_param_bytes(cfg), dtype=torch.uint8, device="cuda")
    f = torch.zeros((1, 64, 64), dtype=torch.float64, device="cuda")
    ws = mlg.workspace(mlg.fluid_net_workspace_bytes(cfg, mlg.grid_of((64, 64)), 1, False))
    with pytest.raises(mlg.MlgError):
        mlg.fluid_net_infer(cfg, buf, 2, f, f, f.clone(), ws)                 # blocks > max
