"""The autotuner: its choice is valid, recorded, and solves that use it
(tile 0, schedule 0) match the explicit tile/schedule bitwise and the oracle."""
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
    tile, fused, split = mlg.mlg_autotune(grid, tune)
    print(f"  tile {tile} fused mask {fused:#x} split mask {split:#x}")
    assert 1 <= tile <= mlg.mlg_tile_count(len(shape))
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
