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

import json
import time
from collections import deque
from dataclasses import asdict, dataclass, field

import numpy as np
import torch

from . import (MLG_ERR_NONFINITE, MLG_FP32_IR, FluidCfg, MlgError, NetCfg, Opts, grid_of,
               gmres_solve, mlg_autotune,
               fluid_net_infer, fluid_net_init, fluid_net_param_bytes, fluid_net_train_step,
               fluid_net_workspace_bytes,
               gmres_workspace_bytes, guess_net_infer, guess_net_init, guess_net_param_bytes,
               guess_net_train_step, guess_net_workspace_bytes, linear_guess_infer,
               linear_guess_init, linear_guess_param_bytes, linear_guess_train_step,
               linear_guess_workspace_bytes, workspace)


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


def moving_average(values, p: int) -> float:
    """M_p of Section 2.2: the unweighted mean of the last p values (the
    current one included; fewer than p values: all of them).  The printed
    formula sums p + 1 terms and divides by p; read as the mean of p."""
    w = list(values)[-p:]
    return sum(w) / len(w)


def cosine(a, b) -> float:
    """|<a, b>| / (|a| |b|) for two device or host arrays (0 if either is 0)."""
    if isinstance(a, torch.Tensor):
        na, nb = float(torch.linalg.norm(a)), float(torch.linalg.norm(b))
        dot = float(torch.sum(a * b))
    else:
        na, nb = float(np.linalg.norm(a)), float(np.linalg.norm(b))
        dot = float(np.sum(np.asarray(a) * np.asarray(b)))
    return abs(dot) / (na * nb) if na > 0 and nb > 0 else 0.0


class SelectiveCollector:
    """Algorithm 1 of the paper (Section 2.2, "collecting data after the model
    has been trained"): a solved step whose first-restart residual E_k and
    time to solution are both below their moving averages M_p (current value
    included) passes; otherwise the network under-performed on it, its pair is
    added to the candidate set C_t if its solution is sufficiently orthogonal
    to every candidate's solution (|cos| <= cos_max), and the failure counts
    towards f_r.  After f_r failures the caller retrains on C_t (mixed with
    the training set) and drains it.  Readings: the test uses the current
    guess x_n^0 (the listing writes x_i^0); the spread d(.,.) is measured on
    the solutions, as the text says (the listing applies it to the RHS);
    p, f_r and the threshold are not given."""

    def __init__(self, p: int = 10, f_r: int = 8, cos_max: float = 0.999, similarity=cosine):
        self.p, self.f_r, self.cos_max, self.similarity = p, f_r, cos_max, similarity
        self.E: list[float] = []
        self.T: list[float] = []
        self.candidates: list = []
        self.cand_x: list = []
        self.failures = 0
        self.seen = 0
        self.retained = 0

    def passes(self, e_k: float, tos: float) -> bool:
        self.E.append(e_k)
        self.T.append(tos)
        return e_k < moving_average(self.E, self.p) and tos < moving_average(self.T, self.p)

    def observe(self, e_k: float, tos: float, pair, x) -> bool:
        """Record one solved step; True when f_r under-performing steps have
        been seen since the last retraining (time to retrain)."""
        self.seen += 1
        if self.passes(e_k, tos):
            return False
        if all(self.similarity(x, c) <= self.cos_max for c in self.cand_x):
            self.candidates.append(pair)
            self.cand_x.append(x)
            self.retained += 1
        self.failures += 1
        return self.failures >= self.f_r

    def drain(self) -> list:
        out = self.candidates
        self.candidates, self.cand_x, self.failures = [], [], 0
        return out


class BlockGrowth:
    """When to append a residual block to the multi-scale network (Section
    2.1: blocks are added before the output layer as the network's progress
    stagnates).  Training losses are averaged over windows of `window` steps;
    when a window's mean is not at least `min_gain` (relative) below the
    previous window's, the network grows by one block (up to `max_blocks`) and
    the comparison restarts.  The paper gives no rule; this one is ours."""

    def __init__(self, window: int = 50, min_gain: float = 0.05, max_blocks: int = 4):
        self.window, self.min_gain, self.max_blocks = window, min_gain, max_blocks
        self.blocks = 0
        self.cur: list[float] = []
        self.prev_mean: float | None = None
        self.events: list[tuple[int, int]] = []     # (training step, blocks after)
        self.steps = 0

    def observe(self, loss: float) -> bool:
        """Record one training loss; True when a block was just appended."""
        self.steps += 1
        self.cur.append(loss)
        if len(self.cur) < self.window:
            return False
        mean = sum(self.cur) / len(self.cur)
        self.cur = []
        prev, self.prev_mean = self.prev_mean, mean
        if prev is None or self.blocks >= self.max_blocks or mean < (1.0 - self.min_gain) * prev:
            return False
        self.blocks += 1
        self.prev_mean = None
        self.events.append((self.steps, self.blocks))
        return True


def fluid_levels(shape, coarsest: int = 8, most: int = 6) -> int:
    """Pyramid levels for a grid: the most (<= `most`) for which both sides
    divide by 2^(levels-1) and the coarsest level keeps >= `coarsest` points
    per side."""
    L = 1
    while L < most and all(n % (1 << L) == 0 and n >> L >= coarsest for n in shape):
        L += 1
    return L


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
    relres_iter5: float = float("nan")
    train_s: float = 0.0
    loss: float = float("nan")
    extra: dict = field(default_factory=dict)


def record_json(rec: StepRecord) -> str:
    """One step's record as a JSON object (NaN written as null)."""
    def clean(v):
        if isinstance(v, float) and v != v:
            return None
        if isinstance(v, dict):
            return {k: clean(x) for k, x in v.items()}
        return v
    return json.dumps({k: clean(v) for k, v in asdict(rec).items()}, sort_keys=True)


class StreamSolver:
    """Solve a stream of right-hand sides on one grid with a chosen guess policy.

    guess: "zero", "prev" (u_{t-1}), "learned" (network, trained in situ) or
    "linear" (the single-layer model x0 = T f_t of Section 3, one
    gradient-descent step of rate `lin_lr` per solved pair on the replay
    buffer).
    network (learned guess): "spectral" (the guess_net network) or "fluid"
    (the multi-scale pooling-pyramid network, growing residual blocks by
    BlockGrowth up to `max_blocks`).
    policy (learned guess): "replay" -- one training step per solved pair on
    the replay buffer (above); "algorithm1" -- the paper's schedule: every
    pair of the first `collect` steps goes to the training set, which then
    trains the network for `init_steps` steps; afterwards SelectiveCollector
    decides which pairs become candidates and when to retrain
    (`retrain_steps` steps on batches of the candidates plus samples of the
    training set, after which the candidates join the training set).
    """

    def __init__(self, shape, guess: str = "learned", restart_m: int = 30, rtol: float = 1e-8,
                 precision: int = MLG_FP32_IR, warmup: int = 16, replay: int = 64, batch: int = 8,
                 net_cfg: NetCfg | None = None, seed: int = 0, train: bool = True,
                 time_train: bool = True, autotune: bool = True, tile: int = 0,
                 policy: str = "replay", collect: int = 50, init_steps: int = 300,
                 retrain_steps: int = 32, p: int = 10, f_r: int = 8, cos_max: float = 0.999,
                 train_set: int = 512, network: str = "spectral", fluid_cfg: FluidCfg | None = None,
                 max_blocks: int = 4, grow_window: int = 50, grow_min_gain: float = 0.05,
                 lin_lr: float = 0.1, shadow_cfgs=(), log_path: str | None = None):
        if guess not in ("zero", "prev", "learned", "linear"):
            raise ValueError("guess must be zero, prev, learned or linear")
        self.lin_lr = lin_lr
        if policy not in ("replay", "algorithm1"):
            raise ValueError("policy must be replay or algorithm1")
        if network not in ("spectral", "fluid"):
            raise ValueError("network must be spectral or fluid")
        self.network = network
        self.policy = policy
        self.collect, self.init_steps, self.retrain_steps = collect, init_steps, retrain_steps
        if policy == "algorithm1":
            warmup = collect                      # the collection phase guesses u_{t-1}
            replay = train_set                    # the training set X_t
            self.collector = SelectiveCollector(p, f_r, cos_max)
            self.rng = np.random.default_rng(seed + 1)
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
        self.train_enabled = train and guess in ("learned", "linear")
        self.time_train = time_train
        self.t = 0
        self.u_prev = torch.zeros(self.shape, dtype=torch.float64, device="cuda")
        self.x = torch.empty_like(self.u_prev)
        # batch-of-one views of the two fixed fields (the guess call's arguments)
        self._u1 = self.u_prev.view(1, *self.shape)
        self._x1 = self.x.view(1, *self.shape)
        self.records: list[StepRecord] = []
        # one JSON object per right-hand side (the step's record), appended to
        # log_path as the stream runs
        self.log = open(log_path, "a") if log_path else None
        if guess == "linear":
            self.warmup = 1
            self.params = torch.zeros(linear_guess_param_bytes(self.grid), dtype=torch.uint8,
                                      device="cuda")
            linear_guess_init(self.grid, self.params)
            self.ws_train = workspace(linear_guess_workspace_bytes(self.grid, batch))
            self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            self.replay = ReplayBuffer(replay, seed)
        if guess == "learned":
            if len(self.shape) != 2:
                raise ValueError("the learned guess is defined on 2D grids")
            if network == "fluid":
                self.net_cfg = fluid_cfg or FluidCfg(seed=seed, levels=fluid_levels(self.shape),
                                                     max_blocks=max_blocks)
                self.growth = BlockGrowth(grow_window, grow_min_gain, self.net_cfg.max_blocks)
                self.params = torch.zeros(fluid_net_param_bytes(self.net_cfg), dtype=torch.uint8,
                                          device="cuda")
                fluid_net_init(self.net_cfg, self.params)
                nbytes = lambda b, tr: fluid_net_workspace_bytes(self.net_cfg, self.grid, b, tr)  # noqa: E731
            else:
                # the skip band may not exceed the grid
                self.net_cfg = net_cfg or NetCfg(seed=seed, skip_modes=min(64, *self.shape))
                self.params = torch.zeros(guess_net_param_bytes(self.net_cfg), dtype=torch.uint8,
                                          device="cuda")
                guess_net_init(self.net_cfg, self.params)
                nbytes = lambda b, tr: guess_net_workspace_bytes(self.net_cfg, self.grid, b, tr)  # noqa: E731
            self.ws_infer = workspace(nbytes(1, False))
            self.ws_train = workspace(nbytes(batch, True))
            self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            self.replay = ReplayBuffer(replay, seed)
        # shadow networks (guess_net configurations) trained on exactly the
        # batches of this stream while train_shadows is set, whose guesses the
        # solver never uses: they measure other networks on the same pairs
        self.shadows = []
        self.train_shadows = True
        for cfg in shadow_cfgs:
            prm = torch.zeros(guess_net_param_bytes(cfg), dtype=torch.uint8, device="cuda")
            guess_net_init(cfg, prm)
            self.shadows.append({
                "cfg": cfg, "params": prm,
                "ws_infer": workspace(guess_net_workspace_bytes(cfg, self.grid, 1, False)),
                "ws_train": workspace(guess_net_workspace_bytes(cfg, self.grid, batch, True))})

    # ------------------------------------------------------------------
    def state_dict(self) -> dict:
        """What the stream carries from one step to the next, in host memory:
        the step count, u_{t-1}, the network's parameter buffer (weights, Adam
        moments and step, the band's least-squares sums, the output gain), the
        replay buffer's pairs and its generator state, and the shadow networks.
        Resuming from it continues the stream as if it had not stopped (the
        kernels are deterministic).  Covers the replay policy with the spectral
        network or the linear model."""
        if self.policy != "replay" or (self.guess_kind == "learned" and self.network != "spectral"):
            raise NotImplementedError("checkpoints cover the replay policy with the spectral "
                                      "network or the linear model")
        st = {"t": self.t, "u_prev": self.u_prev.cpu(),
              "shadows": [sh["params"].cpu() for sh in self.shadows]}
        if hasattr(self, "params"):
            st["params"] = self.params.cpu()
        if hasattr(self, "replay"):
            st["replay"] = [torch.stack([a.cpu() for a in item]) for item in self.replay.items]
            st["replay_rng"] = self.replay.rng.bit_generator.state
        return st

    def load_state_dict(self, st: dict) -> None:
        """Resume from state_dict() of a stream with the same configuration."""
        if self.policy != "replay" or (self.guess_kind == "learned" and self.network != "spectral"):
            raise NotImplementedError("checkpoints cover the replay policy with the spectral "
                                      "network or the linear model")
        if tuple(st["u_prev"].shape) != self.shape:
            raise ValueError(f"checkpoint grid {tuple(st['u_prev'].shape)}, stream {self.shape}")
        if ("params" in st) != hasattr(self, "params") or len(st["shadows"]) != len(self.shadows):
            raise ValueError("checkpoint of a stream with another guess or other shadow networks")
        if "params" in st:
            if st["params"].numel() != self.params.numel():
                raise ValueError("checkpoint of another network configuration")
            self.params.copy_(st["params"].to(self.params.device))
        for sh, prm in zip(self.shadows, st["shadows"]):
            if prm.numel() != sh["params"].numel():
                raise ValueError("checkpoint of another shadow network configuration")
            sh["params"].copy_(prm.to(sh["params"].device))
        self.t = int(st["t"])
        self.u_prev.copy_(st["u_prev"].to(self.u_prev.device))
        if hasattr(self, "replay"):
            self.replay.items.clear()
            for item in st.get("replay", []):
                self.replay.push(*(x.cuda() for x in item.unbind(0)))
            self.replay.rng.bit_generator.state = st["replay_rng"]

    def save(self, path) -> None:
        torch.save(self.state_dict(), path)

    def load(self, path) -> None:
        """Resume from a file written by save() (read with the loader that
        executes nothing from the file)."""
        self.load_state_dict(torch.load(path, weights_only=True))

    # ------------------------------------------------------------------
    def _guess(self, f: torch.Tensor) -> str:
        if self.guess_kind == "zero" or self.t == 0:
            self.x.zero_()
            return "zero"
        if self.guess_kind == "prev" or self.t < self.warmup:
            self.x.copy_(self.u_prev)
            return "prev"
        if self.guess_kind == "linear":
            linear_guess_infer(self.grid, self.params, f.reshape(1, -1), self.x.view(1, -1))
            return "linear"
        args = (f.view(1, *self.shape), self._u1, self._x1, self.ws_infer)
        if self.network == "fluid":
            fluid_net_infer(self.net_cfg, self.params, self.growth.blocks, *args)
        else:
            guess_net_infer(self.net_cfg, self.params, *args)
        return "learned"

    def step(self, f: torch.Tensor) -> StepRecord:
        """Solve A u_t = f_t; returns the step's record (u_t in self.u_prev after)."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kind = self._guess(f)
        try:
            st = gmres_solve(self.grid, f, self.x, self.opts, self.ws)
        except MlgError as e:
            if e.code != MLG_ERR_NONFINITE or kind not in ("learned", "linear"):
                raise
            kind = kind + "->prev"
            self.x.copy_(self.u_prev)
            st = gmres_solve(self.grid, f, self.x, self.opts, self.ws)
        tos = time.perf_counter() - t0
        rec = StepRecord(self.t, kind, st.iters, st.cycles, st.relres_init, st.relres_first_cycle,
                         st.relres_true, tos, st.relres_iter5)
        if self.train_enabled and self.t > 0:
            t1 = time.perf_counter()
            steps = self._train_after(f, rec)
            if self.time_train and steps:
                torch.cuda.synchronize()
                rec.train_s = time.perf_counter() - t1
                rec.loss = float(self.loss.item())
            rec.extra["train_steps"] = steps
        self.u_prev.copy_(self.x)
        self.records.append(rec)
        if self.log:
            self.log.write(record_json(rec) + "\n")
            self.log.flush()
        self.t += 1
        return rec

    def _train_after(self, f: torch.Tensor, rec: StepRecord) -> int:
        """Training after the solve of step t >= 1; returns the steps taken."""
        pair = (f.clone(), self.u_prev.clone(), self.x.clone())
        if self.policy == "replay":
            self.replay.push(*pair)
            self.train_step()
            return 1
        if self.t < self.collect:                       # collection phase
            self.replay.push(*pair)
            if self.t == self.collect - 1:
                for _ in range(self.init_steps):
                    self.train_step()
                return self.init_steps
            return 0
        retrain = self.collector.observe(rec.relres_first_cycle, rec.tos, pair, pair[2])
        rec.extra["candidates"] = len(self.collector.candidates)
        if not retrain:
            return 0
        cands = self.collector.drain()
        for _ in range(self.retrain_steps):
            k = min(len(cands), self.batch)
            chosen = [cands[i] for i in self.rng.choice(len(cands), size=k, replace=False)]
            fill = self.batch - k
            if fill > 0 and len(self.replay) > 0:
                idx = self.rng.choice(len(self.replay), size=min(fill, len(self.replay)),
                                      replace=False)
                chosen += [self.replay.items[i] for i in idx]
            self._train_on(chosen)
        for c in cands:
            self.replay.push(*c)
        return self.retrain_steps

    def _train_on(self, batch) -> None:
        if self.guess_kind == "linear":
            linear_guess_train_step(self.grid, self.params, self.lin_lr,
                                    [b[0].reshape(-1) for b in batch],
                                    [b[2].reshape(-1) for b in batch], self.ws_train, self.loss)
            return
        args = ([b[0] for b in batch], [b[1] for b in batch], [b[2] for b in batch],
                self.ws_train, self.loss)
        if self.train_shadows:
            for sh in self.shadows:
                guess_net_train_step(sh["cfg"], sh["params"], *args[:3], sh["ws_train"])
        if self.network == "fluid":
            fluid_net_train_step(self.net_cfg, self.params, self.growth.blocks, *args)
            self.growth.observe(float(self.loss.item()))
        else:
            guess_net_train_step(self.net_cfg, self.params, *args)

    def train_step(self) -> None:
        self._train_on(self.replay.sample(self.batch))

    def shadow_guess(self, i: int, f: torch.Tensor, u_prev: torch.Tensor, out: torch.Tensor):
        """Guess of shadow network i from (f, u_prev) into out (fields of the grid)."""
        sh = self.shadows[i]
        guess_net_infer(sh["cfg"], sh["params"], f.view(1, *self.shape),
                        u_prev.view(1, *self.shape), out.view(1, *self.shape), sh["ws_infer"])
