"""The autotuner: its choice is valid, recorded, and solves that use it
(tile 0, schedule 0) match the explicit tile/schedule bitwise and the oracle;
the two launch modes (graph replay, direct launches) give the same bits."""
import numpy as np
import pytest
import torch

from oracle import gmres as og
from synthetic import DriftingGaussians

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlg():
    import paper_2103_10975_amd as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return m


def solve(mlg, b, **kw):
    grid = mlg.grid_of(b.shape)
    opts = mlg.Opts(**kw)
    ws = mlg.workspace(mlg.gmres_workspace_bytes(grid, opts))
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    st = mlg.gmres_solve(grid, bd, xd, opts, ws)
    return xd.cpu().numpy(), st


@pytest.mark.parametrize("shape,m,precision", [((200, 150), 20, 0), ((96, 96), 12, 1),
                                                ((24, 20, 28), 16, 0)])
def test_autotune_choice_is_used(mlg, shape, m, precision):
    print("autotune", shape, m, precision, flush=True)
    grid = mlg.grid_of(shape)
    tune = mlg.Opts(restart_m=m, precision=precision)
    tile, fused, split, launch = mlg.mlg_autotune(grid, tune)
    print(f"  tile {tile} fused mask {fused:#x} split mask {split:#x} launch {launch}")
    assert 1 <= tile <= mlg.mlg_tile_count(len(shape))
    assert launch in (1, 2)
    assert fused < (1 << m) and split & ~fused == 0
    if len(shape) == 3:
        assert fused == 0                       # no fused sweep in 3D
    b = DriftingGaussians(shape, 3, 0.06, seed=42).field(0)
    tol = 1e-9
    xa, sa = solve(mlg, b, restart_m=m, rtol=tol, precision=precision)
    # the same tile with the tuned mask forced through an explicit schedule
    # (both forms of the fused sweep give the same bits)
    sched = 2 if fused == (1 << m) - 1 else (1 if fused == 0 else None)
    if sched is not None:
        xe, se = solve(mlg, b, restart_m=m, rtol=tol, precision=precision, tile=tile,
                       schedule=sched)
        assert np.array_equal(xa, xe) and sa.iters == se.iters
    rn, bn = og.residual_norm(b, xa)
    assert sa.status == 0 and rn <= tol * bn
    xo, so = og.gmres(b, m=m, rtol=tol)
    if precision == 0:
        assert abs(sa.iters - so.iters) <= 1
        assert np.linalg.norm(xa - xo) <= 1e-8 * np.linalg.norm(xo)


def test_autotune_errors(mlg):
    grid = mlg.grid_of((64, 64))
    opts = mlg.Opts(restart_m=10)
    need = mlg.mlg_autotune_workspace_bytes(grid, opts)
    with pytest.raises(mlg.MlgError) as e:
        mlg.mlg_autotune(grid, opts, mlg.workspace(need // 2))
    assert e.value.code == mlg.MLG_ERR_WORKSPACE
    with pytest.raises(mlg.MlgError):
        mlg.mlg_autotune(grid, mlg.Opts(restart_m=0))


@pytest.mark.parametrize("shape,m,precision,schedule,poll",
                         [((200, 150), 20, 0, 3, 1), ((96, 96), 12, 1, 1, 2),
                          ((24, 20, 28), 16, 0, 1, 1), ((130, 70), 9, 1, 2, 3)])
def test_launch_modes_give_the_same_bits(mlg, shape, m, precision, schedule, poll):
    """Graph replay and direct launches enqueue the same kernels in the same
    order: solutions and statistics agree bitwise, over many restart cycles
    and several host poll intervals."""
    print("launch modes", shape, m, precision, schedule, poll, flush=True)
    b = DriftingGaussians(shape, 3, 0.06, seed=7).field(0)
    runs = [solve(mlg, b, restart_m=m, rtol=1e-9, precision=precision, schedule=schedule,
                  poll_cycles=poll, launch=launch) for launch in (1, 2)]
    (xg, sg), (xd, sd) = runs
    assert sg.status == 0 and sd.status == 0 and sg.cycles > 3
    assert np.array_equal(xg, xd)
    for f in ("iters", "cycles", "relres_init", "relres_first_cycle", "relres_est",
              "relres_true", "relres_iter5"):
        assert getattr(sg, f) == getattr(sd, f), f


def test_launch_modes_batched(mlg):
    """A batched solve of a 2D and a 3D system (several right-hand sides each)
    gives the same bits with graph replay and direct launches."""
    print("launch modes batched", flush=True)
    shapes = [(90, 110), (20, 18, 22)]
    rhs = [np.stack([DriftingGaussians(sh, 3, 0.08, seed=30 + i).field(t) for t in range(3)])
           for i, sh in enumerate(shapes)]
    out = []
    for launch in (1, 2):
        bs = [torch.from_numpy(r).cuda() for r in rhs]
        xs = [torch.zeros_like(b) for b in bs]
        systems = [mlg.make_system(b, x, 1) for b, x in zip(bs, xs)]
        opts = mlg.Opts(restart_m=14, rtol=1e-9, precision=1, launch=launch)
        ws = mlg.workspace(mlg.gmres_batched_workspace_bytes(systems, opts))
        stats = mlg.gmres_solve_batched(systems, opts, ws)
        torch.cuda.synchronize()
        out.append(([x.cpu().numpy() for x in xs], [(s.status, s.iters, s.relres_true)
                                                     for s in stats]))
    (xg, sg), (xd, sd) = out
    assert all(s[0] == 0 for s in sg)
    assert sg == sd
    assert all(np.array_equal(a, c) for a, c in zip(xg, xd))



@pytest.mark.parametrize("precision,launch", [(0, 1), (1, 1), (1, 2)])
def test_split_cycles_give_the_same_bits(mlg, precision, launch):
    """A single right-hand side whose workspace has solved before splits each
    restart cycle after the steps the previous solve took there (the rest of
    the cycle launched only when needed).  The kernels and their order are
    those of whole cycles: solves after a shorter one (cycles longer than the
    split) and after a longer one (cycles that stop inside the first part)
    give the bits of the static entry point, which always runs whole cycles."""
    print("split cycles", precision, launch, flush=True)
    shape, m, tol = (200, 150), 20, 1e-9
    grid = mlg.grid_of(shape)
    opts = mlg.Opts(restart_m=m, rtol=tol, precision=precision, launch=launch)
    f = [torch.from_numpy(DriftingGaussians(shape, 3, 0.06, seed=11).field(t)).cuda()
         for t in range(3)]
    ws = mlg.workspace(mlg.gmres_workspace_bytes(grid, opts))
    zero = torch.zeros_like(f[0])
    x = zero.clone()
    mlg.gmres_solve(grid, f[0], x, opts, ws)
    close = x.clone()
    # from a close guess (short cycles), from zero (cycles longer than that
    # history), from a close guess again (stops inside the first part)
    for b, x0 in [(f[1], close), (f[2], zero), (f[1], close), (f[1], close)]:
        xs = x0.clone()
        ss = mlg.gmres_solve(grid, b, xs, opts, ws)
        xw = x0.clone()
        sw = mlg.gmres_solve_static(grid, b, xw, opts)
        torch.cuda.synchronize()
        assert ss.status == 0 and sw.status == 0
        assert ss.iters == sw.iters and ss.cycles == sw.cycles
        assert ss.relres_true == sw.relres_true and ss.relres_first_cycle == sw.relres_first_cycle
        assert torch.equal(xs, xw)
