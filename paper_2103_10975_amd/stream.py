"""In-situ learned-guess loop over a time series of Poisson problems.

This is the control flow of the paper's Fig. 2 / Section 2: for every time
step, ask the network for the initial guess x0 = N(b), solve with GMRES(k),
record the solver metrics (E_k, TOS of Section 2.2), keep the (RHS, solution)
pair and train the network on pairs the solver produced (Section 2.3).  The
reading used here (the paper leaves batch sizes, schedules and the replay
policy open):
  - the network sees (f_t, u_{t-1}) and predicts a correction to u_{t-1};
  - one training step per solved pair, on a batch of the newest pair plus
    randomly drawn older ones from a FIFO replay buffer (recent data is always
    used, older data guards against forgetting, as Section 2.3 asks);
  - a pair needs a previous solution, so the first right-hand side of the
    stream gives none (with u_prev = 0 its input would be the whole field,
    not an increment, and its outsized gradients would stall Adam's steps on
    the slowest modes for as long as its second moment remembers them);
  - during the first `warmup` steps the guess is the previous solution;
  - a guess that GMRES rejects as non-finite falls back to the previous
    solution (the solver, not the network, decides the answer).
Every computation runs in the HIP library; this module only sequences calls.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import (MLG_ERR_NONFINITE, MLG_FP32_IR, MlgError, NetCfg, Opts, grid_of, gmres_solve,
               mlg_autotune,
               gmres_workspace_bytes, guess_net_infer, guess_net_init, guess_net_param_bytes,
               guess_net_train_step, guess_net_workspace_bytes, workspace)


class ReplayBuffer:
    """FIFO of (f, u_prev, u) device tensors; sample = newest + uniform others."""

    def __init__(self, capacity: int, seed: int):
        self.items = deque(maxlen=capacity)
        self.rng = np.random.default_rng(seed)

    def push(self, f, u_prev, u):
        self.items.append((f, u_prev, u))

    def __len__(self):
        return len(self.items)

    def sample_indices(self, batch: int):
        n = len(self.items)
        k = min(batch, n)
        others = self.rng.choice(n - 1, size=k - 1, replace=False) if k > 1 else []
        return [n - 1] + [int(i) for i in others]

    def sample(self, batch: int):
        idx = self.sample_indices(batch)
        return [self.items[i] for i in idx]


@dataclass
class StepRecord:
    t: int
    guess: str
    iters: int
    cycles: int
    relres_init: float
    relres_first_cycle: float
    relres_true: float
    tos: float
    train_s: float = 0.0
    loss: float = float("nan")
    extra: dict = field(default_factory=dict)


class StreamSolver:
    """Solve a stream of right-hand sides on one grid with a chosen guess policy.

    guess: "zero", "prev" (u_{t-1}) or "learned" (network, trained in situ).
    """

    def __init__(self, shape, guess: str = "learned", restart_m: int = 30, rtol: float = 1e-8,
                 precision: int = MLG_FP32_IR, warmup: int = 16, replay: int = 64, batch: int = 8,
                 net_cfg: NetCfg | None = None, seed: int = 0, train: bool = True,
                 time_train: bool = True, autotune: bool = True, tile: int = 0):
        if guess not in ("zero", "prev", "learned"):
            raise ValueError("guess must be zero, prev or learned")
        self.shape = tuple(shape)
        self.grid = grid_of(self.shape)
        self.guess_kind = guess
        self.opts = Opts(restart_m=restart_m, precision=precision, rtol=rtol)
        # tile shape and per-step sweep schedule for this grid, timed once per
        # process (solves with tile 0 / schedule 0 then use the recorded choice;
        # an explicit tile keeps the tuned schedule of that tile)
        self.tuned = mlg_autotune(self.grid, self.opts) if autotune else None
        if tile:
            self.opts.tile = tile
        self.ws = workspace(gmres_workspace_bytes(self.grid, self.opts))
        self.warmup, self.batch = warmup, batch
        self.train_enabled = train and guess == "learned"
        self.time_train = time_train
        self.t = 0
        self.u_prev = torch.zeros(self.shape, dtype=torch.float64, device="cuda")
        self.x = torch.empty_like(self.u_prev)
        self.records: list[StepRecord] = []
        if guess == "learned":
            if len(self.shape) != 2:
                raise ValueError("the learned guess is defined on 2D grids")
            # the skip band may not exceed the grid
            self.net_cfg = net_cfg or NetCfg(seed=seed, skip_modes=min(64, *self.shape))
            self.params = torch.zeros(guess_net_param_bytes(self.net_cfg), dtype=torch.uint8,
                                      device="cuda")
            guess_net_init(self.net_cfg, self.params)
            self.ws_infer = workspace(guess_net_workspace_bytes(self.net_cfg, self.grid, 1, False))
            self.ws_train = workspace(guess_net_workspace_bytes(self.net_cfg, self.grid, batch, True))
            self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            self.replay = ReplayBuffer(replay, seed)

    # ------------------------------------------------------------------
    def _guess(self, f: torch.Tensor) -> str:
        if self.guess_kind == "zero" or self.t == 0:
            self.x.zero_()
            return "zero"
        if self.guess_kind == "prev" or self.t < self.warmup:
            self.x.copy_(self.u_prev)
            return "prev"
        guess_net_infer(self.net_cfg, self.params, f.view(1, *self.shape),
                        self.u_prev.view(1, *self.shape), self.x.view(1, *self.shape),
                        self.ws_infer)
        return "learned"

    def step(self, f: torch.Tensor) -> StepRecord:
        """Solve A u_t = f_t; returns the step's record (u_t in self.u_prev after)."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kind = self._guess(f)
        try:
            st = gmres_solve(self.grid, f, self.x, self.opts, self.ws)
        except MlgError as e:
            if e.code != MLG_ERR_NONFINITE or kind != "learned":
                raise
            kind = "learned->prev"
            self.x.copy_(self.u_prev)
            st = gmres_solve(self.grid, f, self.x, self.opts, self.ws)
        tos = time.perf_counter() - t0
        rec = StepRecord(self.t, kind, st.iters, st.cycles, st.relres_init, st.relres_first_cycle,
                         st.relres_true, tos)
        if self.train_enabled and self.t > 0:
            self.replay.push(f.clone(), self.u_prev.clone(), self.x.clone())
            t1 = time.perf_counter()
            self.train_step()
            if self.time_train:
                torch.cuda.synchronize()
                rec.train_s = time.perf_counter() - t1
                rec.loss = float(self.loss.item())
        self.u_prev.copy_(self.x)
        self.records.append(rec)
        self.t += 1
        return rec

    def train_step(self) -> None:
        batch = self.replay.sample(self.batch)
        guess_net_train_step(self.net_cfg, self.params, [b[0] for b in batch],
                             [b[1] for b in batch], [b[2] for b in batch], self.ws_train,
                             self.loss)
