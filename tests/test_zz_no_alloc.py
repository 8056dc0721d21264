"""gmres_solve_static (the entry point that allocates nothing: its workspace
is the library's static per-device scratch) against gmres_solve with a
caller workspace, through the C-ABI.  Same plan, same kernels: the solutions
and the statistics agree bit for bit, on consecutive calls whose second one
is smaller (the scratch keeps the first call's contents), and a problem that
does not fit the scratch is rejected before anything runs.
"""
import numpy as np
import pytest
import torch

from synthetic import DriftingGaussians

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlg():
    import paper_2103_10975_amd as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return m


def rhs(shape, seed):
    return torch.from_numpy(DriftingGaussians(shape, 3, 0.05, seed=seed).field(0)).to("cuda")


def both(mlg, b, x0, opts):
    grid = mlg.grid_of(b.shape)
    ws = mlg.workspace(mlg.gmres_workspace_bytes(grid, opts))
    assert mlg.gmres_workspace_bytes(grid, opts) <= mlg.MLG_STATIC_SCRATCH_BYTES
    xw, xs = x0.clone(), x0.clone()
    sw = mlg.gmres_solve(grid, b, xw, opts, ws)
    ss = mlg.gmres_solve_static(grid, b, xs, opts)
    torch.cuda.synchronize()
    return xw, sw, xs, ss


def same(xw, sw, xs, ss):
    assert torch.equal(xw, xs), float((xw - xs).abs().max())
    assert (ss.status, ss.cycles, ss.iters) == (sw.status, sw.cycles, sw.iters)
    for f in ("relres_init", "relres_first_cycle", "relres_est", "relres_true", "relres_iter5"):
        assert getattr(ss, f) == getattr(sw, f), f


@pytest.mark.parametrize("prec", [0, 1])
def test_static_matches_workspace_solve_on_consecutive_calls(mlg, prec):
    # first call: 256 x 256, zero guess
    print("static solve 256x256 prec", prec, flush=True)
    b = rhs((256, 256), 11)
    opts = mlg.Opts(restart_m=30, rtol=1e-10, precision=prec)
    xw, sw, xs, ss = both(mlg, b, torch.zeros_like(b), opts)
    same(xw, sw, xs, ss)
    assert ss.status == 0 and ss.relres_true <= 1e-10
    # second call, smaller: 100 x 90 from a nonzero guess, another restart length
    print("static solve 100x90 prec", prec, flush=True)
    b2 = rhs((100, 90), 12)
    x0 = 0.5 * rhs((100, 90), 13)
    opts2 = mlg.Opts(restart_m=16, rtol=1e-9, precision=prec)
    xw, sw, xs, ss = both(mlg, b2, x0, opts2)
    same(xw, sw, xs, ss)
    assert ss.status == 0 and ss.relres_true <= 1e-9
    # third, smaller still and 3D
    print("static solve 20x24x28 prec", prec, flush=True)
    b3 = rhs((20, 24, 28), 14)
    xw, sw, xs, ss = both(mlg, b3, torch.zeros_like(b3), mlg.Opts(restart_m=20, rtol=1e-10,
                                                                   precision=prec))
    same(xw, sw, xs, ss)
    assert ss.status == 0


def test_static_rejects_a_problem_larger_than_the_scratch(mlg):
    print("static solve too large", flush=True)
    shape = (1024, 1024)
    opts = mlg.Opts(restart_m=30, rtol=1e-10, precision=0)
    grid = mlg.grid_of(shape)
    assert mlg.gmres_workspace_bytes(grid, opts) > mlg.MLG_STATIC_SCRATCH_BYTES
    b = torch.ones(shape, dtype=torch.float64, device="cuda")
    x = torch.full(shape, 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(mlg.MlgError) as e:
        mlg.gmres_solve_static(grid, b, x, opts)
    assert e.value.code == -2 and "static scratch" in str(e.value)
    assert bool((x == 3.0).all())
    # a fitting call afterwards still works
    b2 = rhs((64, 64), 15)
    xw, sw, xs, ss = both(mlg, b2, torch.zeros_like(b2), mlg.Opts(restart_m=20, rtol=1e-10))
    same(xw, sw, xs, ss)
