"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "mlgmres.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_library_exports_every_declared_symbol():
    import paper_2103_10975_amd as mlg
    declared = header_functions()
    assert len(declared) >= 17
    assert sorted(mlg.EXPORTS) == declared
    raw = ctypes.CDLL(mlg.LIB_PATH)
    for name in declared:
        assert hasattr(raw, name), name


def test_argument_validation_without_device_work():
    import paper_2103_10975_amd as mlg
    g = mlg.grid_of((64, 64))
    assert mlg.gmres_workspace_bytes(g, mlg.Opts(restart_m=20)) > 0
    for bad in (mlg.Opts(restart_m=0), mlg.Opts(restart_m=65), mlg.Opts(precision=7),
                mlg.Opts(rtol=-1.0), mlg.Opts(tile=99), mlg.Opts(schedule=4),
                mlg.Opts(launch=3), mlg.Opts(launch=-1)):
        with pytest.raises(mlg.MlgError):
            mlg.gmres_workspace_bytes(g, bad)
    with pytest.raises(mlg.MlgError):
        mlg.gmres_workspace_bytes(mlg.Grid(4, 8, 8, 8), mlg.Opts())
    with pytest.raises(mlg.MlgError):
        mlg.gmres_workspace_bytes(mlg.Grid(2, 0, 8, 1), mlg.Opts())
    assert "restart_m" in mlg.mlg_last_error() or "dim" in mlg.mlg_last_error() or mlg.mlg_last_error()


def test_workspace_grows_with_problem_and_precision():
    import paper_2103_10975_amd as mlg
    g = mlg.grid_of((512, 512))
    w64 = mlg.gmres_workspace_bytes(g, mlg.Opts(restart_m=30, precision=0))
    w32 = mlg.gmres_workspace_bytes(g, mlg.Opts(restart_m=30, precision=1))
    n = 512 * 512
    assert w64 >= 31 * n * 8 and w32 >= 31 * n * 4 and w32 < w64
    assert mlg.gmres_workspace_bytes(g, mlg.Opts(restart_m=40)) > w64


def test_tile_table():
    import paper_2103_10975_amd as mlg
    for dim in (2, 3):
        cnt = mlg.mlg_tile_count(dim)
        assert cnt >= 3
        for i in range(cnt):
            tx, ty, tz = mlg.mlg_tile_shape(dim, i)
            assert (tx * ty * tz) % 256 == 0 and (dim == 3 or tz == 1)
    assert mlg.mlg_tile_count(5) == 0


def test_binding_rejects_mismatched_shapes():
    """The binding checks shapes and buffer sizes before any library call
    (CPU tensors would be rejected later; the shape checks come first)."""
    import pytest
    import torch
    import paper_2103_10975_amd as mlg
    g = mlg.grid_of((8, 8))
    with pytest.raises(ValueError):
        mlg.gmres_solve(g, torch.zeros(8, 9, dtype=torch.float64), torch.zeros(8, 9, dtype=torch.float64),
                        mlg.Opts(), torch.zeros(16, dtype=torch.uint8))
    with pytest.raises(ValueError):
        mlg.gmres_solve(g, torch.zeros(8, 8, dtype=torch.float64), torch.zeros(8, 7, dtype=torch.float64),
                        mlg.Opts(), torch.zeros(16, dtype=torch.uint8))
    cfg = mlg.NetCfg(skip_modes=4, modes=4)
    f = torch.zeros(1, 8, 8, dtype=torch.float64)
    with pytest.raises(ValueError):
        mlg.guess_net_infer(cfg, torch.zeros(16, dtype=torch.uint8), f, torch.zeros(1, 8, 9), f,
                            torch.zeros(16, dtype=torch.uint8))
    with pytest.raises(ValueError):
        mlg.guess_net_infer(cfg, torch.zeros(16, dtype=torch.uint8), f, f, f,
                            torch.zeros(16, dtype=torch.uint8))          # parameters too small
    with pytest.raises(ValueError):
        mlg.guess_net_train_step(cfg, torch.zeros(16, dtype=torch.uint8), [f[0]], [f[0], f[0]], [f[0]],
                                 torch.zeros(16, dtype=torch.uint8))
    with pytest.raises(ValueError):
        mlg.make_system(torch.zeros(2, 8, 8, dtype=torch.float64), torch.zeros(2, 8, 7, dtype=torch.float64))
