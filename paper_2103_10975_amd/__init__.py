"""MI355X-native MLGMRES: Python binding of the C ABI in include/mlgmres.h.

Argument marshalling only: every step of the solver and of the guess network
runs in the HIP kernels of ``libmlgmres.so`` (built in-tree by ``build.py``).
Device buffers are torch tensors on a ROCm device; their ``data_ptr()`` and
torch's current HIP stream are handed to the library.  There is no CPU
fallback: if the library is missing or fails to load, importing this package
raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "Grid", "Opts", "Stats", "System", "NetCfg", "MLG_FP64", "MLG_FP32_IR",
    "grid_of", "lib", "gmres_workspace_bytes", "gmres_solve", "gmres_solve_static",
    "MLG_STATIC_SCRATCH_BYTES", "gmres_batched_workspace_bytes", "gmres_solve_batched", "mlg_apply_operator", "mlg_kernel_bench_scratch_bytes",
    "mlg_kernel_bench", "mlg_tile_count", "mlg_tile_shape", "mlg_autotune_workspace_bytes",
    "mlg_autotune", "guess_net_param_count", "guess_net_param_offset", "guess_net_param_bytes",
    "guess_net_workspace_bytes", "guess_net_init", "guess_net_refresh", "guess_net_infer",
    "guess_net_train_step", "FluidCfg", "fluid_net_param_count", "fluid_net_param_offset",
    "fluid_net_param_bytes", "fluid_net_workspace_bytes", "fluid_net_init", "fluid_net_refresh",
    "fluid_net_infer", "fluid_net_train_step", "linear_guess_param_bytes",
    "linear_guess_workspace_bytes", "linear_guess_init", "linear_guess_infer",
    "linear_guess_train_step", "mlg_last_error", "mlg_shutdown", "MlgError", "EXPORTS",
    "net_views", "net_pack", "net_unpack", "net_band_weights", "net_set_band", "net_output_gain",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlgmres.so")

MLG_OK, MLG_NOT_CONVERGED = 0, 1
MLG_ERR_ARG, MLG_ERR_WORKSPACE, MLG_ERR_HIP, MLG_ERR_NONFINITE = -1, -2, -3, -4
MLG_FP64, MLG_FP32_IR = 0, 1
MLG_STATIC_SCRATCH_BYTES = 64 << 20

# every symbol the header declares
EXPORTS = (
    "gmres_workspace_bytes", "gmres_solve", "gmres_solve_static", "gmres_batched_workspace_bytes",
    "gmres_solve_batched", "mlg_apply_operator", "mlg_kernel_bench_scratch_bytes",
    "mlg_kernel_bench", "mlg_tile_count", "mlg_tile_shape", "mlg_autotune_workspace_bytes",
    "mlg_autotune", "guess_net_param_count", "guess_net_param_offset", "guess_net_param_bytes",
    "guess_net_workspace_bytes", "guess_net_init", "guess_net_refresh", "guess_net_infer",
    "guess_net_train_step", "fluid_net_param_count", "fluid_net_param_offset",
    "fluid_net_param_bytes", "fluid_net_workspace_bytes", "fluid_net_init", "fluid_net_refresh",
    "fluid_net_infer", "fluid_net_train_step", "linear_guess_param_bytes",
    "linear_guess_workspace_bytes", "linear_guess_init", "linear_guess_infer",
    "linear_guess_train_step", "mlg_last_error", "mlg_shutdown",
)


class MlgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mlgmres error {code}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("restart_m", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("max_iters", ctypes.c_int64),
                ("fixed_iters", ctypes.c_int64), ("tile", ctypes.c_int32),
                ("poll_cycles", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("launch", ctypes.c_int32)]

    def __init__(self, restart_m=30, precision=MLG_FP64, rtol=1e-8, max_iters=0,
                 fixed_iters=0, tile=0, poll_cycles=1, schedule=0, launch=0):
        super().__init__(restart_m, precision, rtol, max_iters, fixed_iters, tile, poll_cycles,
                         schedule, launch)


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("cycles", ctypes.c_int32), ("iters", ctypes.c_int64),
                ("relres_init", ctypes.c_double), ("relres_first_cycle", ctypes.c_double),
                ("relres_est", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("seconds", ctypes.c_double), ("relres_iter5", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class System(ctypes.Structure):
    _fields_ = [("grid", Grid), ("nrhs", ctypes.c_int32), ("guess", ctypes.c_int32),
                ("b", ctypes.c_void_p), ("x", ctypes.c_void_p)]


class NetCfg(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32), ("modes", ctypes.c_int32),
                ("skip_modes", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]

    def __init__(self, channels=32, modes=16, skip_modes=64, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, seed=0):
        super().__init__(channels, modes, skip_modes, lr, beta1, beta2, eps, seed)


class FluidCfg(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("max_blocks", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]

    def __init__(self, channels=32, levels=4, max_blocks=4, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, seed=0):
        super().__init__(channels, levels, max_blocks, lr, beta1, beta2, eps, seed)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2103_10975_amd/build.py "
                          "(or __graft_entry__.build()) first; there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    sig = {
        "gmres_workspace_bytes": (sz, [P(Grid), P(Opts)]),
        "gmres_solve": (ctypes.c_int, [P(Grid), vp, vp, P(Opts), vp, sz, P(Stats), vp]),
        "gmres_solve_static": (ctypes.c_int, [P(Grid), vp, vp, P(Opts), P(Stats), vp]),
        "gmres_batched_workspace_bytes": (sz, [i32, P(System), P(Opts)]),
        "gmres_solve_batched": (ctypes.c_int, [i32, P(System), P(Opts), vp, sz, P(Stats), vp]),
        "mlg_apply_operator": (ctypes.c_int, [P(Grid), vp, vp, vp]),
        "mlg_kernel_bench_scratch_bytes": (sz, [i32]),
        "mlg_kernel_bench": (ctypes.c_int, [P(Grid), P(Opts), vp, sz, vp, sz, i32, i32, i32,
                                            P(ctypes.c_double), vp]),
        "mlg_tile_count": (i32, [i32]),
        "mlg_tile_shape": (ctypes.c_int, [i32, i32, P(i32), P(i32), P(i32)]),
        "mlg_autotune_workspace_bytes": (sz, [P(Grid), P(Opts)]),
        "mlg_autotune": (ctypes.c_int, [P(Grid), P(Opts), vp, sz, P(i32), P(ctypes.c_uint64),
                                        P(ctypes.c_uint64), P(i32), vp]),
        "guess_net_param_count": (i64, [P(NetCfg)]),
        "guess_net_param_offset": (i64, [P(NetCfg), i32]),
        "guess_net_param_bytes": (sz, [P(NetCfg)]),
        "guess_net_workspace_bytes": (sz, [P(NetCfg), P(Grid), i32, i32]),
        "guess_net_init": (ctypes.c_int, [P(NetCfg), vp, vp]),
        "guess_net_refresh": (ctypes.c_int, [P(NetCfg), vp, vp]),
        "guess_net_infer": (ctypes.c_int, [P(NetCfg), vp, P(Grid), i32, vp, vp, vp, vp, sz, vp]),
        "guess_net_train_step": (ctypes.c_int, [P(NetCfg), vp, P(Grid), i32, P(vp), P(vp), P(vp),
                                                vp, sz, vp, vp]),
        "fluid_net_param_count": (i64, [P(FluidCfg)]),
        "fluid_net_param_offset": (i64, [P(FluidCfg), i32]),
        "fluid_net_param_bytes": (sz, [P(FluidCfg)]),
        "fluid_net_workspace_bytes": (sz, [P(FluidCfg), P(Grid), i32, i32]),
        "fluid_net_init": (ctypes.c_int, [P(FluidCfg), vp, vp]),
        "fluid_net_refresh": (ctypes.c_int, [P(FluidCfg), vp, vp]),
        "fluid_net_infer": (ctypes.c_int, [P(FluidCfg), vp, i32, P(Grid), i32, vp, vp, vp, vp, sz,
                                           vp]),
        "fluid_net_train_step": (ctypes.c_int, [P(FluidCfg), vp, i32, P(Grid), i32, P(vp), P(vp),
                                                P(vp), vp, sz, vp, vp]),
        "linear_guess_param_bytes": (sz, [P(Grid)]),
        "linear_guess_workspace_bytes": (sz, [P(Grid), i32]),
        "linear_guess_init": (ctypes.c_int, [P(Grid), vp, vp]),
        "linear_guess_infer": (ctypes.c_int, [P(Grid), vp, i32, vp, vp, vp]),
        "linear_guess_train_step": (ctypes.c_int, [P(Grid), vp, ctypes.c_float, i32, P(vp), P(vp),
                                                   vp, sz, vp, vp]),
        "mlg_last_error": (ctypes.c_char_p, []),
        "mlg_shutdown": (None, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


# ------------------------------------------------------------------ helpers
def mlg_last_error() -> str:
    return lib.mlg_last_error().decode(errors="replace")


def mlg_shutdown() -> None:
    lib.mlg_shutdown()


def _check(rc: int, allow_not_converged: bool = False) -> int:
    if rc < 0 or (rc == MLG_NOT_CONVERGED and not allow_not_converged):
        raise MlgError(rc, mlg_last_error())
    return rc


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t: torch.Tensor | None, dtype=torch.float64):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _points(grid: Grid) -> int:
    return grid.nx * grid.ny * (grid.nz if grid.dim == 3 else 1)


def _need(cond: bool, msg: str) -> None:
    if not cond:
        raise ValueError(msg)


def _same_fields(ts, shape, what: str) -> None:
    for t in ts:
        if t.shape != shape:                              # the message only on failure
            raise ValueError(f"{what}: every field must have shape {tuple(shape)}, "
                             f"got {tuple(t.shape)}")


def _params_ok(params: torch.Tensor, nbytes: int) -> None:
    if params.numel() < nbytes:
        raise ValueError(f"parameter buffer holds {params.numel()} bytes, "
                         f"the configuration needs {nbytes}")


def grid_of(shape) -> Grid:
    """Grid for a field of numpy/torch shape (ny, nx) or (nz, ny, nx)."""
    shape = tuple(int(s) for s in shape)
    if len(shape) == 2:
        return Grid(2, shape[1], shape[0], 1)
    if len(shape) == 3:
        return Grid(3, shape[2], shape[1], shape[0])
    raise ValueError("fields are 2D or 3D")


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """Device byte buffer (torch's allocator aligns to >= 256 B)."""
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device or "cuda")


# ------------------------------------------------------------------ solver
def gmres_workspace_bytes(grid: Grid, opts: Opts) -> int:
    n = lib.gmres_workspace_bytes(ctypes.byref(grid), ctypes.byref(opts))
    if n == 0:
        raise MlgError(MLG_ERR_ARG, mlg_last_error())
    return n


def gmres_solve(grid: Grid, b: torch.Tensor, x: torch.Tensor, opts: Opts, ws: torch.Tensor,
                stream=None, allow_not_converged: bool = False) -> Stats:
    """Solve A x = b in place in x (x holds the initial guess on entry)."""
    _need(b.numel() == _points(grid), f"b has {b.numel()} elements, the grid {_points(grid)}")
    _need(x.shape == b.shape, f"x has shape {tuple(x.shape)}, b {tuple(b.shape)}")
    st = Stats()
    rc = lib.gmres_solve(ctypes.byref(grid), _ptr(b), _ptr(x), ctypes.byref(opts),
                         _ptr(ws, torch.uint8), ws.numel(), ctypes.byref(st), _stream(stream))
    _check(rc, allow_not_converged)
    return st


def gmres_solve_static(grid: Grid, b: torch.Tensor, x: torch.Tensor, opts: Opts,
                       stream=None, allow_not_converged: bool = False) -> Stats:
    """gmres_solve without a workspace argument: the library's static
    per-device scratch (MLG_STATIC_SCRATCH_BYTES) holds the workspace, and the
    call allocates nothing."""
    _need(b.numel() == _points(grid), f"b has {b.numel()} elements, the grid {_points(grid)}")
    _need(x.shape == b.shape, f"x has shape {tuple(x.shape)}, b {tuple(b.shape)}")
    st = Stats()
    rc = lib.gmres_solve_static(ctypes.byref(grid), _ptr(b), _ptr(x), ctypes.byref(opts),
                                ctypes.byref(st), _stream(stream))
    _check(rc, allow_not_converged)
    return st


def gmres_batched_workspace_bytes(systems, opts: Opts) -> int:
    arr = (System * len(systems))(*systems)
    n = lib.gmres_batched_workspace_bytes(len(systems), arr, ctypes.byref(opts))
    if n == 0:
        raise MlgError(MLG_ERR_ARG, mlg_last_error())
    return n


def make_system(b: torch.Tensor, x: torch.Tensor, guess: int = 0) -> System:
    """b, x: [nrhs, ...field shape] device float64 tensors."""
    _need(b.dim() in (3, 4), "b must be [nrhs, ny, nx] or [nrhs, nz, ny, nx]")
    _need(x.shape == b.shape, f"x has shape {tuple(x.shape)}, b {tuple(b.shape)}")
    return System(grid_of(b.shape[1:]), b.shape[0], guess, _ptr(b), _ptr(x))


def gmres_solve_batched(systems, opts: Opts, ws: torch.Tensor, stream=None,
                        allow_not_converged: bool = False):
    arr = (System * len(systems))(*systems)
    total = sum(s.nrhs for s in systems)
    stats = (Stats * total)()
    rc = lib.gmres_solve_batched(len(systems), arr, ctypes.byref(opts), _ptr(ws, torch.uint8),
                                 ws.numel(), stats, _stream(stream))
    _check(rc, allow_not_converged)
    return list(stats)


def mlg_apply_operator(u: torch.Tensor, y: torch.Tensor, stream=None) -> None:
    g = grid_of(u.shape)
    _need(y.shape == u.shape, f"y has shape {tuple(y.shape)}, u {tuple(u.shape)}")
    _check(lib.mlg_apply_operator(ctypes.byref(g), _ptr(u), _ptr(y), _stream(stream)))


(MLG_K_DOTS, MLG_K_COEF, MLG_K_EXTEND, MLG_K_UPDATE, MLG_K_RESIDUAL, MLG_K_STEP, MLG_K_SUMS,
 MLG_K_STEPC) = range(8)
# kernel symbol of each kind (MLG_K_STEPC is the split-form instance of k_step)
KERNEL_NAMES = {MLG_K_DOTS: "k_dots", MLG_K_COEF: "k_coef", MLG_K_EXTEND: "k_extend",
                MLG_K_UPDATE: "k_update", MLG_K_RESIDUAL: "k_resid", MLG_K_STEP: "k_step",
                MLG_K_SUMS: "k_sums", MLG_K_STEPC: "k_step"}


def mlg_kernel_bench_scratch_bytes(reps: int) -> int:
    return lib.mlg_kernel_bench_scratch_bytes(reps)


def mlg_kernel_bench(grid: Grid, opts: Opts, ws: torch.Tensor, scratch: torch.Tensor, kind: int,
                     step: int, reps: int, stream=None) -> float:
    """Average duration (us) of `reps` launches of one solver kernel, timed with
    HIP events on the stream (ws: workspace of a finished gmres_solve)."""
    out = ctypes.c_double()
    _check(lib.mlg_kernel_bench(ctypes.byref(grid), ctypes.byref(opts), _ptr(ws, torch.uint8),
                                ws.numel(), _ptr(scratch, torch.uint8), scratch.numel(), kind, step,
                                reps, ctypes.byref(out), _stream(stream)))
    return out.value


def mlg_autotune_workspace_bytes(grid: Grid, opts: Opts) -> int:
    n = lib.mlg_autotune_workspace_bytes(ctypes.byref(grid), ctypes.byref(opts))
    if n == 0:
        raise MlgError(MLG_ERR_ARG, mlg_last_error())
    return n


def mlg_autotune(grid: Grid, opts: Opts, ws: torch.Tensor | None = None, stream=None):
    """Time every tile, per-step sweep schedule and launch mode for (grid,
    opts) and record the fastest for later solves with tile=0, schedule=0,
    launch=0.  Returns (tile, fused-step bit mask, split-form bit mask, launch
    mode: 1 graph replay, 2 direct launches).  ws: scratch of
    mlg_autotune_workspace_bytes bytes (allocated here when None)."""
    if ws is None:
        ws = workspace(mlg_autotune_workspace_bytes(grid, opts))
    tile, fused, split = ctypes.c_int32(), ctypes.c_uint64(), ctypes.c_uint64()
    launch = ctypes.c_int32()
    _check(lib.mlg_autotune(ctypes.byref(grid), ctypes.byref(opts), _ptr(ws, torch.uint8),
                            ws.numel(), ctypes.byref(tile), ctypes.byref(fused),
                            ctypes.byref(split), ctypes.byref(launch), _stream(stream)))
    return tile.value, fused.value, split.value, launch.value


def mlg_tile_count(dim: int) -> int:
    return lib.mlg_tile_count(dim)


def mlg_tile_shape(dim: int, index: int):
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib.mlg_tile_shape(dim, index, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


# ------------------------------------------------------------------ network
def guess_net_param_count(cfg: NetCfg) -> int:
    return lib.guess_net_param_count(ctypes.byref(cfg))


def guess_net_param_offset(cfg: NetCfg, index: int) -> int:
    return lib.guess_net_param_offset(ctypes.byref(cfg), index)


def guess_net_param_bytes(cfg: NetCfg) -> int:
    return lib.guess_net_param_bytes(ctypes.byref(cfg))


def guess_net_workspace_bytes(cfg: NetCfg, grid: Grid, batch: int, train: bool) -> int:
    n = lib.guess_net_workspace_bytes(ctypes.byref(cfg), ctypes.byref(grid), batch, int(train))
    if n == 0:
        raise MlgError(MLG_ERR_ARG, mlg_last_error())
    return n


def guess_net_init(cfg: NetCfg, params: torch.Tensor, stream=None) -> None:
    _check(lib.guess_net_init(ctypes.byref(cfg), _ptr(params, torch.uint8), _stream(stream)))


def guess_net_refresh(cfg: NetCfg, params: torch.Tensor, stream=None) -> None:
    _check(lib.guess_net_refresh(ctypes.byref(cfg), _ptr(params, torch.uint8), _stream(stream)))


def guess_net_infer(cfg: NetCfg, params: torch.Tensor, f: torch.Tensor, u_prev: torch.Tensor,
                    guess: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    """f, u_prev, guess: [batch, ny, nx] (or [ny, nx]) float64 device tensors."""
    _need(f.dim() in (2, 3), "f must be [ny, nx] or [batch, ny, nx]")
    _same_fields([u_prev, guess], f.shape, "u_prev and guess")
    shape = f.shape[-2:]
    batch = 1 if f.dim() == 2 else f.shape[0]
    g = grid_of(shape)
    _params_ok(params, guess_net_param_bytes(cfg))
    _check(lib.guess_net_infer(ctypes.byref(cfg), _ptr(params, torch.uint8), ctypes.byref(g), batch,
                               _ptr(f), _ptr(u_prev), _ptr(guess), _ptr(ws, torch.uint8),
                               ws.numel(), _stream(stream)))


def guess_net_train_step(cfg: NetCfg, params: torch.Tensor, fs, u_prevs, u_targets,
                         ws: torch.Tensor, loss: torch.Tensor | None = None, stream=None) -> None:
    """fs, u_prevs, u_targets: lists of [ny, nx] float64 device tensors (one per sample)."""
    batch = len(fs)
    _need(batch >= 1 and len(u_prevs) == batch and len(u_targets) == batch,
          "fs, u_prevs and u_targets must be equally long, non-empty lists")
    _need(fs[0].dim() == 2, "samples are [ny, nx] fields")
    _same_fields(list(fs) + list(u_prevs) + list(u_targets), fs[0].shape, "samples")
    g = grid_of(fs[0].shape)
    _params_ok(params, guess_net_param_bytes(cfg))
    arr = lambda ts: (ctypes.c_void_p * batch)(*[_ptr(t) for t in ts])  # noqa: E731
    lp = _ptr(loss, torch.float32) if loss is not None else None
    _check(lib.guess_net_train_step(ctypes.byref(cfg), _ptr(params, torch.uint8), ctypes.byref(g),
                                    batch, arr(fs), arr(u_prevs), arr(u_targets),
                                    _ptr(ws, torch.uint8), ws.numel(), lp, _stream(stream)))


# ------------------------------------------------------------------ parameter layout
# Tensor order and shapes of the parameter arrays (see include/mlgmres.h).
NET_TENSORS = ("conv1.w", "conv1.b", "conv2.w", "conv2.b", "spec.w1", "spec.b", "spec.wk",
               "conv4.w", "conv4.b", "conv5.w", "conv5.b", "conv6.w", "conv6.b")


def net_tensor_shapes(cfg: NetCfg) -> dict:
    C, M = cfg.channels, cfg.modes
    return {"conv1.w": (C, 2, 3, 3), "conv1.b": (C,), "conv2.w": (C, C, 3, 3), "conv2.b": (C,),
            "spec.w1": (C, C), "spec.b": (C,), "spec.wk": (M, M, C, C),
            "conv4.w": (C, C, 3, 3), "conv4.b": (C,), "conv5.w": (C, C, 3, 3), "conv5.b": (C,),
            "conv6.w": (1, C, 3, 3), "conv6.b": (1,)}


def _align(v: int, a: int = 256) -> int:
    return (v + a - 1) // a * a


def net_views(cfg, params: torch.Tensor) -> dict:
    """Views of the regions of a parameter buffer (uint8 device tensor) of
    either network (NetCfg or FluidCfg).  For the guess network, "band" is
    the band path's least-squares state, float64 [2, K, K] (sums of X T, then
    of X^2)."""
    fluid = isinstance(cfg, FluidCfg)
    P = fluid_net_param_count(cfg) if fluid else guess_net_param_count(cfg)
    f = _align(P * 4)
    step = 4 * f + _align(P * 2)
    out = {"master": params[0:P * 4].view(torch.float32),
           "grad": params[f:f + P * 4].view(torch.float32),
           "adam_m": params[2 * f:2 * f + P * 4].view(torch.float32),
           "adam_v": params[3 * f:3 * f + P * 4].view(torch.float32),
           "bf16": params[4 * f:4 * f + P * 2].view(torch.bfloat16),
           "step": params[step:step + 8].view(torch.int64)}
    if not fluid:
        K = cfg.skip_modes
        band = step + 256
        out["band"] = params[band:band + 16 * K * K].view(torch.float64).view(2, K, K)
        gate = band + _align(16 * K * K)
        out["gate"] = params[gate:gate + 16].view(torch.float64)
    return out


def net_output_gain(cfg: NetCfg, params: torch.Tensor) -> float:
    """The convolutional branch's output gain applied at inference (1 before
    any training batch)."""
    g = net_views(cfg, params)["gate"].cpu()
    return float(g[0] / g[1]) if g[1] > 0 else 1.0


def net_band_weights(cfg: NetCfg, params: torch.Tensor) -> torch.Tensor:
    """The band path's current weights w = sxt / sxx (0 where sxx = 0), [K, K]
    float64 (device)."""
    b = net_views(cfg, params)["band"]
    return torch.where(b[1] > 0, b[0] / torch.where(b[1] > 0, b[1], 1.0), torch.zeros_like(b[0]))


def net_set_band(cfg: NetCfg, params: torch.Tensor, w) -> None:
    """Impose band weights w [K, K] (sxt = w, sxx = 1); later train steps add
    their sums to this state."""
    b = net_views(cfg, params)["band"]
    b[0].copy_(torch.as_tensor(w, dtype=torch.float64))
    b[1].fill_(1.0)


def net_pack(cfg: NetCfg, tensors: dict) -> torch.Tensor:
    """Host float32 [P] array from a dict of tensors (names and shapes above)."""
    P = guess_net_param_count(cfg)
    out = torch.zeros(P, dtype=torch.float32)
    shapes = net_tensor_shapes(cfg)
    for i, name in enumerate(NET_TENSORS):
        off = guess_net_param_offset(cfg, i)
        t = torch.as_tensor(tensors[name], dtype=torch.float32).reshape(-1)
        if t.numel() != int(torch.tensor(shapes[name]).prod()):
            raise ValueError(f"{name}: expected shape {shapes[name]}")
        out[off:off + t.numel()] = t
    return out


def net_unpack(cfg: NetCfg, flat: torch.Tensor) -> dict:
    """Dict of host float64 tensors from a float32 [P] array (inverse of net_pack)."""
    flat = flat.detach().to("cpu", torch.float64)
    shapes = net_tensor_shapes(cfg)
    out = {}
    for i, name in enumerate(NET_TENSORS):
        off = guess_net_param_offset(cfg, i)
        n = int(torch.tensor(shapes[name]).prod())
        out[name] = flat[off:off + n].reshape(shapes[name]).clone()
    return out


# ------------------------------------------------------------------ multi-scale network
def fluid_net_param_count(cfg: FluidCfg) -> int:
    return lib.fluid_net_param_count(ctypes.byref(cfg))


def fluid_net_param_offset(cfg: FluidCfg, index: int) -> int:
    return lib.fluid_net_param_offset(ctypes.byref(cfg), index)


def fluid_net_param_bytes(cfg: FluidCfg) -> int:
    return lib.fluid_net_param_bytes(ctypes.byref(cfg))


def fluid_net_workspace_bytes(cfg: FluidCfg, grid: Grid, batch: int, train: bool) -> int:
    n = lib.fluid_net_workspace_bytes(ctypes.byref(cfg), ctypes.byref(grid), batch, int(train))
    if n == 0:
        raise MlgError(MLG_ERR_ARG, mlg_last_error())
    return n


def fluid_net_init(cfg: FluidCfg, params: torch.Tensor, stream=None) -> None:
    _check(lib.fluid_net_init(ctypes.byref(cfg), _ptr(params, torch.uint8), _stream(stream)))


def fluid_net_refresh(cfg: FluidCfg, params: torch.Tensor, stream=None) -> None:
    _check(lib.fluid_net_refresh(ctypes.byref(cfg), _ptr(params, torch.uint8), _stream(stream)))


def fluid_net_infer(cfg: FluidCfg, params: torch.Tensor, blocks: int, f: torch.Tensor,
                    u_prev: torch.Tensor, guess: torch.Tensor, ws: torch.Tensor,
                    stream=None) -> None:
    """f, u_prev, guess: [batch, ny, nx] (or [ny, nx]) float64 device tensors."""
    _need(f.dim() in (2, 3), "f must be [ny, nx] or [batch, ny, nx]")
    _same_fields([u_prev, guess], f.shape, "u_prev and guess")
    batch = 1 if f.dim() == 2 else f.shape[0]
    g = grid_of(f.shape[-2:])
    _params_ok(params, fluid_net_param_bytes(cfg))
    _check(lib.fluid_net_infer(ctypes.byref(cfg), _ptr(params, torch.uint8), blocks,
                               ctypes.byref(g), batch, _ptr(f), _ptr(u_prev), _ptr(guess),
                               _ptr(ws, torch.uint8), ws.numel(), _stream(stream)))


def fluid_net_train_step(cfg: FluidCfg, params: torch.Tensor, blocks: int, fs, u_prevs, u_targets,
                         ws: torch.Tensor, loss: torch.Tensor | None = None, stream=None) -> None:
    """fs, u_prevs, u_targets: lists of [ny, nx] float64 device tensors."""
    batch = len(fs)
    _need(batch >= 1 and len(u_prevs) == batch and len(u_targets) == batch,
          "fs, u_prevs and u_targets must be equally long, non-empty lists")
    _need(fs[0].dim() == 2, "samples are [ny, nx] fields")
    _same_fields(list(fs) + list(u_prevs) + list(u_targets), fs[0].shape, "samples")
    g = grid_of(fs[0].shape)
    _params_ok(params, fluid_net_param_bytes(cfg))
    arr = lambda ts: (ctypes.c_void_p * batch)(*[_ptr(t) for t in ts])  # noqa: E731
    lp = _ptr(loss, torch.float32) if loss is not None else None
    _check(lib.fluid_net_train_step(ctypes.byref(cfg), _ptr(params, torch.uint8), blocks,
                                    ctypes.byref(g), batch, arr(fs), arr(u_prevs), arr(u_targets),
                                    _ptr(ws, torch.uint8), ws.numel(), lp, _stream(stream)))


def fluid_tensor_names(cfg: FluidCfg) -> list:
    """Tensor order of the multi-scale network's parameter arrays."""
    names = []
    for l in range(cfg.levels):
        names += [f"lvl{l}.conv1.w", f"lvl{l}.conv1.b", f"lvl{l}.conv2.w", f"lvl{l}.conv2.b"]
    for i in range(cfg.max_blocks):
        names += [f"blk{i}.a.w", f"blk{i}.a.b", f"blk{i}.b.w", f"blk{i}.b.b"]
    return names + ["head.conv1.w", "head.conv1.b", "head.conv2.w", "head.conv2.b"]


def fluid_tensor_shapes(cfg: FluidCfg) -> dict:
    C = cfg.channels
    out = {}
    for name in fluid_tensor_names(cfg):
        if name == "head.conv2.b":
            out[name] = (1,)
        elif name.endswith(".b"):
            out[name] = (C,)
        elif name == "head.conv2.w":
            out[name] = (1, C, 3, 3)
        elif name.startswith("lvl") and ".conv1." in name:
            out[name] = (C, 2, 3, 3)
        else:
            out[name] = (C, C, 3, 3)
    return out


def fluid_pack(cfg: FluidCfg, tensors: dict) -> torch.Tensor:
    """Host float32 [P] array from a dict of tensors (names and shapes above)."""
    out = torch.zeros(fluid_net_param_count(cfg), dtype=torch.float32)
    shapes = fluid_tensor_shapes(cfg)
    for i, name in enumerate(fluid_tensor_names(cfg)):
        off = fluid_net_param_offset(cfg, i)
        t = torch.as_tensor(tensors[name], dtype=torch.float32).reshape(-1)
        if t.numel() != int(torch.tensor(shapes[name]).prod()):
            raise ValueError(f"{name}: expected shape {shapes[name]}")
        out[off:off + t.numel()] = t
    return out


def fluid_unpack(cfg: FluidCfg, flat: torch.Tensor) -> dict:
    """Dict of host float64 tensors from a float32 [P] array (inverse of fluid_pack)."""
    flat = flat.detach().to("cpu", torch.float64)
    shapes = fluid_tensor_shapes(cfg)
    out = {}
    for i, name in enumerate(fluid_tensor_names(cfg)):
        off = fluid_net_param_offset(cfg, i)
        n = int(torch.tensor(shapes[name]).prod())
        out[name] = flat[off:off + n].reshape(shapes[name]).clone()
    return out


# ------------------------------------------------------------------ linear model
def linear_guess_param_bytes(grid: Grid) -> int:
    n = lib.linear_guess_param_bytes(ctypes.byref(grid))
    if n == 0:
        raise MlgError(MLG_ERR_ARG, mlg_last_error())
    return n


def linear_guess_workspace_bytes(grid: Grid, batch: int) -> int:
    n = lib.linear_guess_workspace_bytes(ctypes.byref(grid), batch)
    if n == 0:
        raise MlgError(MLG_ERR_ARG, mlg_last_error())
    return n


def linear_guess_init(grid: Grid, params: torch.Tensor, stream=None) -> None:
    _check(lib.linear_guess_init(ctypes.byref(grid), _ptr(params, torch.uint8), _stream(stream)))


def linear_guess_infer(grid: Grid, params: torch.Tensor, b: torch.Tensor, x0: torch.Tensor,
                       stream=None) -> None:
    """b, x0: float64 device tensors holding `batch` contiguous fields of the
    grid's n points ([batch, n], [n] or grid-shaped with a leading batch axis)."""
    n = _points(grid)
    if b.numel() % n or x0.numel() != b.numel():
        raise ValueError("b and x0 must hold the same whole number of grid fields")
    _params_ok(params, linear_guess_param_bytes(grid))
    batch = b.numel() // n
    _check(lib.linear_guess_infer(ctypes.byref(grid), _ptr(params, torch.uint8), batch, _ptr(b),
                                  _ptr(x0), _stream(stream)))


def linear_guess_train_step(grid: Grid, params: torch.Tensor, lr: float, bs, xs, ws: torch.Tensor,
                            loss: torch.Tensor | None = None, stream=None) -> None:
    """bs, xs: lists of float64 device tensors of the grid's n points."""
    batch = len(bs)
    _need(batch >= 1 and len(xs) == batch, "bs and xs must be equally long, non-empty lists")
    _need(all(t.numel() == _points(grid) for t in list(bs) + list(xs)),
          "every sample must hold the grid's points")
    _params_ok(params, linear_guess_param_bytes(grid))
    arr = lambda ts: (ctypes.c_void_p * batch)(*[_ptr(t) for t in ts])  # noqa: E731
    lp = _ptr(loss, torch.float32) if loss is not None else None
    _check(lib.linear_guess_train_step(ctypes.byref(grid), _ptr(params, torch.uint8), lr, batch,
                                       arr(bs), arr(xs), _ptr(ws, torch.uint8), ws.numel(), lp,
                                       _stream(stream)))


def linear_views(grid: Grid, params: torch.Tensor) -> dict:
    """T and its last gradient as [n, n] float32 views of a parameter buffer."""
    half = linear_guess_param_bytes(grid) // 2
    n = grid.nx * grid.ny * (grid.nz if grid.dim == 3 else 1)
    return {"T": params[:n * n * 4].view(torch.float32).view(n, n),
            "grad": params[half:half + n * n * 4].view(torch.float32).view(n, n)}
