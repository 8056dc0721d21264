"""Benchmark: time-to-solution per right-hand side, learned guess vs plain GMRES.

Workload (one GPU): the 512 x 512 zero-Dirichlet Poisson stream with four
drifting Gaussian sources (sigma 0.03), GMRES(30), relative residual 1e-8.
One step = one time step of the in-situ method: network guess from
(f_t, u_{t-1}) -> GMRES(30) with the FP32 Krylov basis and FP64 refinement ->
one training step of the network on the replay buffer.  `--warmup` steps run
first (they also train the network in situ: its spectral skip gains reach the
exact inverse of A on their band after about 300 steps of the stream), then
exactly `--steps` steps are timed.  The same right-hand sides are then solved
by plain FP64 GMRES(30) from a zero guess (the comparison the metric names),
and by FP64 GMRES from the previous solution.  Beside the timed window, the
whole stream (learning phase included) is summarised: mean time to solution
and iterations per RHS, and the training time.

Printed: one JSON line with the metric, the roofline of the dominant kernel
(HIP-event timing of its launches in the solve's launch configuration) and
the CPU oracle timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-solution per RHS at rel. residual 1e-8: learned guess vs plain GMRES"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-baseline", action="store_true", help="skip the plain-GMRES legs")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-systems leg")
    ap.add_argument("--batched-cycles", type=int, default=3,
                    help="restart cycles per system in the batched leg")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--probe", default=None, metavar="KERNEL",
                    help="counter-collection run: a 256 MiB device copy (the byte-count "
                         "calibration) then every launch of KERNEL (step, dots, extend, update, "
                         "resid) in one restart cycle, in the learned-guess solve's launch "
                         "configuration")
    return ap.parse_args()


def kernel_roofline(mlg, shape, opts, b, tile, fused, split=0, reps=20, only=None):
    """Average launch duration of every solver kernel over one restart cycle,
    in the launch configuration of the solve (tuned tile and per-step sweep
    schedule; HIP events on the stream), with the algorithmic bytes of each
    launch."""
    grid = mlg.grid_of(shape)
    m = opts.restart_m
    fixed = mlg.Opts(restart_m=m, precision=opts.precision, rtol=opts.rtol, fixed_iters=m,
                     tile=tile)
    ws = mlg.workspace(mlg.gmres_workspace_bytes(grid, fixed))
    x = torch.zeros_like(b)
    mlg.gmres_solve(grid, b, x, fixed, ws)                 # fills the basis of one full cycle
    scratch = mlg.workspace(mlg.mlg_kernel_bench_scratch_bytes(reps))
    n = int(np.prod(shape))
    s = 8 if opts.precision == mlg.MLG_FP64 else 4
    # the launches of one cycle: (kind, step index, algorithmic bytes)
    launches = [(mlg.MLG_K_DOTS, 0, 1 * n * s)]           # w = A u_0 and |u_0|: read u_0
    for j in range(m):
        if (split >> j) & 1:
            # sums over workgroups; the sweep forms the coefficients itself
            launches.append((mlg.MLG_K_SUMS, j, 0))
            launches.append((mlg.MLG_K_STEPC, j, (j + 3) * n * s))
        elif (fused >> j) & 1:
            # read v_0..v_{j-1}, u_j; write v_j, u_{j+1}
            launches.append((mlg.MLG_K_COEF, j, 0))       # one-workgroup sums
            launches.append((mlg.MLG_K_STEP, j, (j + 3) * n * s))
        else:
            launches.append((mlg.MLG_K_COEF, j, 0))
            launches.append((mlg.MLG_K_EXTEND, j, (j + 3) * n * s))
            launches.append((mlg.MLG_K_DOTS, j + 1, (j + 2) * n * s))   # read v_0..v_j, u_{j+1}
    launches.append((mlg.MLG_K_COEF, m, 0))
    launches.append((mlg.MLG_K_UPDATE, m, m * n * s + 2 * n * 8))      # read V_m, read+write x
    launches.append((mlg.MLG_K_RESIDUAL, m, 3 * n * 8))                # read x, b; write r
    out = {}
    for kind, j, byts in launches:
        name = mlg.KERNEL_NAMES[kind]
        if only is not None and name != only:
            continue
        us = mlg.mlg_kernel_bench(grid, fixed, ws, scratch, kind, j, reps)
        d = out.setdefault(name, {"launches_per_cycle": 0, "us": [], "bytes": []})
        d["launches_per_cycle"] += 1
        d["us"].append(us)
        d["bytes"].append(byts)
    for d in out.values():
        d["avg_us"] = statistics.fmean(d["us"])
        d["avg_bytes"] = statistics.fmean(d["bytes"])
        d["cycle_us"] = sum(d["us"])
    del ws, scratch
    return out


def batched_leg(mlg, seed, cycles, m=30):
    """Many uneven systems in one graph-replayed launch sequence: 64 2D grids
    with sides drawn from {128, ..., 1024} and 8 3D grids of 64^3..128^3, one
    drifting-Gaussian right-hand side each, FP32-basis GMRES(30) run for a
    fixed number of restart cycles (the throughput of the batched engine, not a
    convergence race: the largest grids need tens of thousands of steps)."""
    from synthetic import DriftingGaussians
    rng = np.random.default_rng(seed)
    shapes = [(int(s), int(s)) for s in rng.choice([128, 192, 256, 384, 512, 768, 1024], 64)]
    shapes += [(int(s),) * 3 for s in rng.integers(64, 129, 8)]
    opts = mlg.Opts(restart_m=m, precision=mlg.MLG_FP32_IR, rtol=1e-8, fixed_iters=cycles * m)
    for dim in (2, 3):          # tune the largest system of each dimension
        big = max((sh for sh in shapes if len(sh) == dim), key=lambda sh: int(np.prod(sh)))
        mlg.mlg_autotune(mlg.grid_of(big), mlg.Opts(restart_m=m, precision=mlg.MLG_FP32_IR))
    bs, xs = [], []
    for i, sh in enumerate(shapes):
        g = DriftingGaussians(sh, 4, 0.03, seed=seed + i)
        bs.append(torch.from_numpy(g.field(0)[None]).cuda())
        xs.append(torch.zeros_like(bs[-1]))
    systems = [mlg.make_system(b, x, 0) for b, x in zip(bs, xs)]
    ws = mlg.workspace(mlg.gmres_batched_workspace_bytes(systems, opts))
    mlg.gmres_solve_batched(systems, opts, ws)                  # captures the cycle graph
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = mlg.gmres_solve_batched(systems, opts, ws)
    dt = time.perf_counter() - t0
    n = sum(int(np.prod(sh)) for sh in shapes)
    steps = cycles * m
    # algorithmic bytes of one cycle per point (FP32 basis): the steps' sweeps
    # (read j basis vectors and the direction, write two vectors) + update + residual
    per_point = 4 * sum(j + 3 for j in range(m)) + (4 * m + 16) + 24
    return {"systems": len(shapes), "points": n, "steps_per_system": steps,
            "seconds": dt, "us_per_step": 1e6 * dt / steps,
            "point_steps_per_s": n * steps / dt,
            "effective_GB/s": n * per_point * cycles / dt / 1e9,
            "iters_ok": all(st.iters == steps for st in stats)}


def counter_traffic(kernel, shape, precision_tag, m, tile):
    """HBM bytes per launch of `kernel` on tile shape `tile` (e.g. "64x16") from
    the committed FETCH_SIZE/WRITE_SIZE summary
    (profiles/<kernel>_<H>x<W>_traffic.md), or None when there is none for this
    workload or the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{shape[0]}x{shape[1]}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    if fields.get("workload_key") != f"{kernel} {shape[0]}x{shape[1]} {precision_tag} m{m}":
        return None
    h = hashlib.sha256()
    for src in fields.get("kernel_sources", "").split():
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != fields.get("kernel_source_sha256"):
        return None
    v = fields.get(f"traffic_bytes_per_launch tile={tile}")
    return float(v) if v else None


def cpu_baseline(shape, m, rtol, f0, plain_iters, budget_s):
    """The FP64 CPU oracle (single thread) on a bounded sample: a fixed number
    of Arnoldi steps on the first RHS, projected to the plain-GMRES iteration
    count of the same RHS."""
    from oracle import gmres as og
    t0 = time.perf_counter()
    og.gmres(f0, m=m, fixed_iters=m)                       # one cycle, to size the sample
    per_cycle = time.perf_counter() - t0
    cycles = max(1, int(budget_s / max(per_cycle, 1e-6)))
    k = cycles * m
    t0 = time.perf_counter()
    og.gmres(f0, m=m, fixed_iters=k)
    dt = time.perf_counter() - t0
    per_iter = dt / k
    return {"value": per_iter * plain_iters, "unit": "s/RHS", "cores": 1, "kind": "oracle",
            "sample": f"{k} FP64 CGS2 GMRES({m}) Arnoldi steps of RHS 0 on {shape[0]}x{shape[1]} "
                      f"({dt:.1f} s, {per_iter * 1e3:.2f} ms/step), projected to the "
                      f"{plain_iters:.0f} steps plain GMRES needs per RHS"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus N > 1 is not supported"}))
        sys.exit(2)
    import paper_2103_10975_amd as mlg
    from paper_2103_10975_amd.stream import StreamSolver
    from synthetic import DriftingGaussians

    torch.cuda.set_device(0)
    shape = (args.grid, args.grid)
    if args.probe:
        probe(mlg, shape, args)
        return
    gen = DriftingGaussians(shape, 4, 0.03, seed=args.seed)
    total = args.warmup + args.steps
    fields = [torch.from_numpy(gen.field(t)).cuda() for t in range(total)]

    learned = StreamSolver(shape, guess="learned", restart_m=args.restart, rtol=args.rtol,
                           precision=mlg.MLG_FP32_IR, seed=args.seed, time_train=False)
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    for t in range(args.warmup):
        learned.step(fields[t])
    torch.cuda.synchronize()
    stream_s = time.perf_counter() - ts0
    t0 = time.perf_counter()
    for t in range(args.warmup, total):
        learned.step(fields[t])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed = learned.records[args.warmup:]
    tos_learned = statistics.fmean(r.tos for r in timed)
    warm = learned.records[:args.warmup]
    gains = mlg.net_unpack(learned.net_cfg, mlg.net_views(learned.net_cfg, learned.params)["master"])
    # error of the trained skip gains against the exact inverse (rho g = 1):
    # over the 16 x 16 slowest modes (where the sources put their content) and
    # the median over the whole band (its fastest modes carry next to nothing
    # and barely move from their initial zero)
    gerr = (32.0 * gains["skip.g"] - 1.0).abs()
    gain_err = {"max_16x16": float(gerr[:16, :16].max()), "median_band": float(gerr.median())}

    result = {
        "metric": METRIC, "value": tos_learned, "unit": "s/RHS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (f32 Krylov basis) + bf16 network",
        "data": "synthetic",
        "config": {"workload": f"2D 5-point Poisson {shape[0]}x{shape[1]}, 4 drifting Gaussian "
                               f"sources (sigma 0.03), GMRES({args.restart}), rtol {args.rtol}, "
                               "learned guess + FP32-basis refinement vs plain FP64 GMRES",
                   "grid": list(shape), "restart_m": args.restart, "rtol": args.rtol,
                   "seed": args.seed},
        "learned": {"tos_mean": tos_learned, "tos_median": statistics.median(r.tos for r in timed),
                    "tos_p90": float(np.percentile([r.tos for r in timed], 90)),
                    "iters_mean": statistics.fmean(r.iters for r in timed),
                    "relres_init_mean": statistics.fmean(r.relres_init for r in timed),
                    "E_k_mean": statistics.fmean(r.relres_first_cycle for r in timed),
                    "guess_kinds": sorted(set(r.guess for r in timed)),
                    "skip_gain_error": gain_err},
        # the in-situ learning phase before the timed window: every step
        # solved (guess, GMRES) and trained once
        "stream": {"steps": args.warmup, "seconds": stream_s,
                   "tos_mean": statistics.fmean(r.tos for r in warm) if warm else None,
                   "iters_mean": statistics.fmean(r.iters for r in warm) if warm else None,
                   "train_s_per_step": ((stream_s - sum(r.tos for r in warm)) / len(warm)
                                        if warm else None)},
    }

    if not args.no_baseline:
        legs = {}
        for name, guess, prec in [("plain_fp64_zero", "zero", mlg.MLG_FP64),
                                  ("fp64_prev", "prev", mlg.MLG_FP64)]:
            sv = StreamSolver(shape, guess=guess, restart_m=args.restart, rtol=args.rtol,
                              precision=prec)
            if guess == "prev":
                sv.u_prev.copy_(_solution_before(fields, args, mlg))
                sv.t = 1
            for t in range(args.warmup, total):
                sv.step(fields[t])
            legs[name] = {"tos_mean": statistics.fmean(r.tos for r in sv.records),
                          "iters_mean": statistics.fmean(r.iters for r in sv.records)}
            del sv
        result["baselines"] = legs
        result["speedup_vs_plain"] = legs["plain_fp64_zero"]["tos_mean"] / tos_learned
        result["speedup_vs_prev_fp64"] = legs["fp64_prev"]["tos_mean"] / tos_learned

    # roofline of the dominant kernel of the learned-guess solve
    tile, fused, split = learned.tuned
    tshape = mlg.mlg_tile_shape(2, tile - 1)
    result["config"]["tile"] = list(tshape)
    result["config"]["fused_steps"] = bin(fused).count("1")
    result["config"]["split_steps"] = bin(split).count("1")
    kr = kernel_roofline(mlg, shape, learned.opts, fields[0], tile, fused, split)
    dom = max((k for k in kr if kr[k]["avg_bytes"] > 0), key=lambda k: kr[k]["cycle_us"])
    d = kr[dom]
    achieved = d["avg_bytes"] / (d["avg_us"] * 1e-6) / 1e9
    tag = "fp64" if learned.opts.precision == mlg.MLG_FP64 else "fp32"
    result["roofline"] = {"kernel": dom, "bound": "hbm", "achieved": achieved,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                          "traffic": counter_traffic(dom, shape, tag, args.restart,
                                                     f"{tshape[0]}x{tshape[1]}"),
                          "avg_us": d["avg_us"], "avg_bytes": d["avg_bytes"]}
    result["kernels"] = {k: {"avg_us": v["avg_us"], "per_cycle": v["launches_per_cycle"],
                             "GB/s": v["avg_bytes"] / v["avg_us"] / 1e3, "cycle_us": v["cycle_us"]}
                         for k, v in kr.items()}

    if not args.no_batched:
        result["batched"] = batched_leg(mlg, args.seed, args.batched_cycles)

    if not args.no_cpu:
        plain_iters = (result.get("baselines", {}).get("plain_fp64_zero", {}).get("iters_mean")
                       or result["learned"]["iters_mean"])
        result["cpu_baseline"] = cpu_baseline(shape, args.restart, args.rtol,
                                              fields[args.warmup].cpu().numpy(), plain_iters,
                                              args.cpu_seconds)
    line = json.dumps(result)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as fh:
            fh.write(line + "\n")


def probe(mlg, shape, args):
    """Launches for hardware-counter runs (no timing is reported): a 256 MiB
    device copy (the byte-count calibration), then for every tile shape one
    restart cycle's launches of the probed kernel in the learned-guess solve's
    configuration (fused steps in the split form for `step` and `sums`), each
    step index once."""
    from synthetic import DriftingGaussians
    names = {v.replace("k_", ""): v for v in mlg.KERNEL_NAMES.values()}
    if args.probe not in names:
        raise SystemExit(f"--probe takes one of {sorted(names)}")
    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")       # 256 MiB
    for _ in range(3):
        a.clone()
    torch.cuda.synchronize()
    f0 = torch.from_numpy(DriftingGaussians(shape, 4, 0.03, seed=args.seed).field(0)).cuda()
    opts = mlg.Opts(restart_m=args.restart, rtol=args.rtol, precision=mlg.MLG_FP32_IR)
    fused = (1 << args.restart) - 1 if args.probe in ("step", "sums") else 0
    out = {}
    for tile in range(1, mlg.mlg_tile_count(2) + 1):
        r = kernel_roofline(mlg, shape, opts, f0, tile, fused, fused, reps=1,
                            only=names[args.probe])
        out["x".join(map(str, mlg.mlg_tile_shape(2, tile - 1)[:2]))] = r[names[args.probe]]["avg_bytes"]
    torch.cuda.synchronize()
    print(json.dumps({"probe": args.probe, "copy_bytes": 2 * a.numel() * 4, "avg_bytes": out}),
          flush=True)


def _solution_before(fields, args, mlg):
    """u_{warmup-1} for the previous-solution leg: solved afresh in FP64."""
    grid = mlg.grid_of(fields[0].shape)
    opts = mlg.Opts(restart_m=args.restart, rtol=args.rtol)
    ws = mlg.workspace(mlg.gmres_workspace_bytes(grid, opts))
    x = torch.zeros_like(fields[0])
    mlg.gmres_solve(grid, fields[args.warmup - 1], x, opts, ws)
    return x


if __name__ == "__main__":
    main()
