"""What the in-situ trained network gains over the method without it.

The same drifting-Gaussian stream (256 x 256, 4 sources, sigma 0.03) is solved
three times with FP32-basis GMRES(30) to 1e-8: from a zero guess, from the
previous solution u_{t-1}, and from the learned guess (network trained one step
per solved pair on the replay buffer).  Measured over steps [100, 200):

* the previous solution beats the zero guess in iterations, and the learned
  guess needs well under the previous solution's count (measured 10 vs
  5352: the band path's least-squares weights on exact training pairs are
  right after the first batches);
* the trained network removes nearly all of the slow-mode error of u_{t-1}
  (its projection on the 16 x 16 slowest sine modes of the Dirichlet
  Laplacian -- the error restarted GMRES converges slowest on): measured
  5e9x.

The paper prints no iteration counts for this network or workload, so the
sizes of these gains are measured and printed, not pinned.
"""
import math
import statistics

import pytest
import torch

from synthetic import DriftingGaussians

pytestmark = pytest.mark.gpu

N, T, W0 = 256, 200, 100


@pytest.fixture(scope="module")
def mlg():
    import paper_2103_10975_amd as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return m


def slow_part(S, e):
    return S.T @ (S @ e @ S.T) @ S


def test_learned_guess_gain(mlg):
    from paper_2103_10975_amd.stream import StreamSolver
    print("stream gain", flush=True)
    gen = DriftingGaussians((N, N), 4, 0.03, seed=4000)
    fields = [torch.from_numpy(gen.field(t)).cuda() for t in range(T)]
    k = torch.arange(1, 17, dtype=torch.float64, device="cuda")[:, None]
    i = torch.arange(1, N + 1, dtype=torch.float64, device="cuda")[None, :]
    S = torch.sin(k * math.pi * i / (N + 1)) * math.sqrt(2.0 / (N + 1))
    iters = {}
    ratios = []
    for guess in ("zero", "prev", "learned"):
        sv = StreamSolver((N, N), guess=guess, restart_m=30, rtol=1e-8, seed=1, time_train=False)
        for t in range(T):
            probe = guess == "learned" and t >= W0 and t % 10 == 0
            if probe:                      # the guess this step will start from
                up = sv.u_prev.clone()
                g = torch.empty_like(up)
                mlg.guess_net_infer(sv.net_cfg, sv.params, fields[t].view(1, N, N),
                                    up.view(1, N, N), g.view(1, N, N), sv.ws_infer)
            sv.step(fields[t])
            if probe:
                u = sv.u_prev
                ratios.append(float(torch.linalg.norm(slow_part(S, u - up)) /
                                    torch.linalg.norm(slow_part(S, u - g))))
        iters[guess] = statistics.fmean(r.iters for r in sv.records[W0:])
        assert all(r.relres_true <= 1e-8 for r in sv.records)
    gain = statistics.fmean(ratios)
    print(f"  mean iterations over [{W0}, {T}): zero {iters['zero']:.0f}, "
          f"prev {iters['prev']:.0f}, learned {iters['learned']:.0f}; "
          f"slow-mode error of u_(t-1) / of the learned guess: {gain:.2f}")
    assert iters["prev"] < iters["zero"]
    assert iters["learned"] < 0.6 * iters["prev"]
    assert gain > 100.0


def test_algorithm1_schedule(mlg):
    """The paper's data-collection schedule (Algorithm 1): every pair of the
    first 50 steps trains the network, then only under-performing steps feed
    the candidate set and trigger retraining.  On the same stream the trained
    guess needs well under the previous solution's iterations (measured over
    [80, 140): 9 vs 5273), the candidate set takes a fraction of the judged
    steps (measured 30 of 90), and every retraining is counted."""
    from paper_2103_10975_amd.stream import StreamSolver
    print("stream algorithm1", flush=True)
    n, steps, w0 = 256, 140, 80
    gen = DriftingGaussians((n, n), 4, 0.03, seed=4000)
    fields = [torch.from_numpy(gen.field(t)).cuda() for t in range(steps)]
    iters = {}
    for guess, policy in (("prev", "replay"), ("learned", "algorithm1")):
        sv = StreamSolver((n, n), guess=guess, restart_m=30, rtol=1e-8, seed=1, time_train=False,
                          policy=policy, collect=50, init_steps=300)
        for t in range(steps):
            sv.step(fields[t])
        iters[guess] = statistics.fmean(r.iters for r in sv.records[w0:])
        assert all(r.relres_true <= 1e-8 for r in sv.records)
    c = sv.collector
    trained = [r.extra.get("train_steps", 0) for r in sv.records]
    print(f"  mean iterations over [{w0}, {steps}): prev {iters['prev']:.0f}, "
          f"learned (algorithm 1) {iters['learned']:.0f}; retained {c.retained} of {c.seen} "
          f"judged steps, {sum(trained)} training steps")
    assert iters["learned"] < 0.5 * iters["prev"]
    assert 0 < c.retained < c.seen == steps - 50
    assert trained[49] == 300 and sum(trained[1:49]) == 0
    assert sum(trained) == 300 + 32 * (sum(1 for k in trained[50:] if k))


def test_dipole_workload(mlg):
    """The multi-scale workload (Section 3, dipoles with two scales per pole,
    redrawn at every step): u_{t-1} is no better than a zero guess, and the
    network trained by the Algorithm 1 schedule cuts the iterations by far
    more than the order of magnitude the paper reports for its fifth-iteration
    error (measured at 256 x 256 over steps [80, 120): zero guess 7714
    Arnoldi steps per RHS, learned 315; median first-cycle residual 0.56 ->
    1.1e-7)."""
    from paper_2103_10975_amd.stream import StreamSolver
    from synthetic import RandomDipoles
    print("stream dipoles", flush=True)
    n, steps, w0 = 256, 120, 80
    gen = RandomDipoles((n, n), seed=6000)
    fields = [torch.from_numpy(gen.field(t)).cuda() for t in range(steps)]
    zero = StreamSolver((n, n), guess="zero", restart_m=30, rtol=1e-8, seed=6000, time_train=False)
    for t in range(w0, w0 + 8):
        zero.step(fields[t])
    sv = StreamSolver((n, n), guess="learned", restart_m=30, rtol=1e-8, seed=6000, time_train=False,
                      policy="algorithm1")
    for t in range(steps):
        sv.step(fields[t])
    assert all(r.relres_true <= 1e-8 for r in sv.records + zero.records)
    it_zero = statistics.fmean(r.iters for r in zero.records)
    it_learned = statistics.fmean(r.iters for r in sv.records[w0:])
    ek_zero = statistics.median(r.relres_first_cycle for r in zero.records)
    ek_learned = statistics.median(r.relres_first_cycle for r in sv.records[w0:])
    print(f"  Arnoldi steps per RHS: zero guess {it_zero:.0f}, learned {it_learned:.0f}; "
          f"first-cycle residual (median): {ek_zero:.2e} -> {ek_learned:.2e}")
    assert it_learned < 0.1 * it_zero
    assert ek_learned < 1e-3 * ek_zero


def test_multiscale_network_stream(mlg):
    """The multi-scale (pooling pyramid) network in the stream: guesses stay
    finite and every solve meets the tolerance while residual blocks are
    appended (a growth threshold that every window meets, so both blocks
    are added), and training runs at every step.  Its effect is measured,
    not asserted: at 128 x 128 on the dipole stream its first-cycle residual
    is 0.40 at steps 60-119 against 0.34 for the zero guess, and after 800
    steps its iterations are only ~6 % below the zero guess's, where the
    spectral network needs 70 against ~2000."""
    from paper_2103_10975_amd.stream import StreamSolver
    from synthetic import RandomDipoles
    print("stream multiscale network", flush=True)
    n, steps, w0 = 128, 120, 60
    gen = RandomDipoles((n, n), seed=6000)
    fields = [torch.from_numpy(gen.field(t)).cuda() for t in range(steps)]
    zero = StreamSolver((n, n), guess="zero", restart_m=30, rtol=1e-8, seed=6000, time_train=False)
    for t in range(w0, w0 + 10):
        zero.step(fields[t])
    sv = StreamSolver((n, n), guess="learned", network="fluid", restart_m=30, rtol=1e-8,
                      seed=6000, time_train=False, grow_window=20, grow_min_gain=0.9, max_blocks=2)
    for t in range(steps):
        sv.step(fields[t])
    assert all(r.relres_true <= 1e-8 for r in sv.records + zero.records)
    assert all(r.guess == "learned" for r in sv.records[sv.warmup:])
    assert sum(r.extra.get("train_steps", 0) for r in sv.records) == steps - 1
    ek_zero = statistics.median(r.relres_first_cycle for r in zero.records)
    ek = statistics.median(r.relres_first_cycle for r in sv.records[w0:])
    print(f"  blocks {sv.growth.blocks} (events {sv.growth.events}); first-cycle residual "
          f"zero guess {ek_zero:.3f}, multi-scale network {ek:.3f}")
    assert sv.growth.blocks == 2 and [e[1] for e in sv.growth.events] == [1, 2]
    assert math.isfinite(ek)


def test_stream_jsonl_log(mlg, tmp_path):
    """The per-RHS log: one JSON object per solved right-hand side, the same
    figures as the in-memory records (NaN written as null)."""
    import json
    from paper_2103_10975_amd.stream import StreamSolver
    print("stream log", flush=True)
    shape = (48, 40)
    g = DriftingGaussians(shape, 2, 0.1, seed=31)
    path = tmp_path / "stream.jsonl"
    sv = StreamSolver(shape, guess="prev", restart_m=12, rtol=1e-9, autotune=False,
                      log_path=str(path))
    for t in range(3):
        sv.step(torch.from_numpy(g.field(t)).cuda())
    sv.log.close()
    lines = path.read_text().splitlines()
    assert len(lines) == 3
    for line, rec in zip(lines, sv.records):
        d = json.loads(line)
        assert d["t"] == rec.t and d["guess"] == rec.guess and d["iters"] == rec.iters
        assert d["relres_true"] == rec.relres_true and d["relres_true"] <= 1e-9
        assert d["tos"] > 0 and d["loss"] is None


def test_stream_checkpoint_resume(mlg, tmp_path):
    """A stream saved after step 6 and resumed in a fresh solver (another
    workspace, another process's worth of state) continues bit for bit: the
    same guesses, Arnoldi steps and solutions as the uninterrupted stream."""
    from paper_2103_10975_amd.stream import StreamSolver
    print("stream checkpoint", flush=True)
    shape = (64, 64)
    g = DriftingGaussians(shape, 3, 0.05, seed=77)
    fields = [torch.from_numpy(g.field(t)).cuda() for t in range(12)]
    kw = dict(guess="learned", restart_m=20, rtol=1e-9, warmup=3, replay=16, batch=4, seed=5,
              autotune=False, shadow_cfgs=[mlg.NetCfg(skip_modes=0, seed=5)])
    a = StreamSolver(shape, **kw)
    for t in range(6):
        a.step(fields[t])
    path = tmp_path / "stream.pt"
    a.save(path)
    for t in range(6, 12):
        a.step(fields[t])
    b = StreamSolver(shape, **kw)
    b.load(path)
    assert b.t == 6
    for t in range(6, 12):
        rb = b.step(fields[t])
        ra = a.records[t]
        assert (rb.guess, rb.iters, rb.relres_true) == (ra.guess, ra.iters, ra.relres_true), t
    assert torch.equal(a.u_prev, b.u_prev)
    assert torch.equal(a.params, b.params)
