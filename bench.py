"""Benchmark: time-to-solution per RHS, learned guess vs plain GMRES.

Workload (one GPU): the 512 x 512 zero-Dirichlet Poisson stream with four
drifting Gaussian sources (sigma 0.03), GMRES(30), relative residual 1e-8.
One step = one time step of the in-situ method: network guess from
(f_t, u_{t-1}) -> GMRES(30) with the FP32 Krylov basis and FP64 refinement ->
one training step of the network on the replay buffer (Fig. 2 of the paper).

Phases of the stream (all on the same right-hand sides):
  learn   `--learn` steps (default 400, whatever --warmup says): the in-situ
          method from an untrained network; a shadow network trains on the
          same batches (the configuration's network without a band path),
          its guesses unused;
  warmup  `--warmup` further untimed steps of the method;
  timed   exactly `--steps` steps of the method, bracketed by synchronisation
          (`value` = their mean time to solution per RHS; `ms_per_step` also
          counts the method's own training step).
The same timed right-hand sides are then solved from the same previous
solutions by the comparison legs: plain FP64 GMRES from zero (the metric's
baseline), FP64 and FP32-basis GMRES from u_{t-1}, the configuration's
network without a band path (trained in situ by Adam on the same pairs), the
learned network with its convolutional output switched off, and the band at
its analytic optimum c_u / lambda_kl with nothing trained (what learning
converges to).  Whole-stream totals (training included) are reported beside
the timed window.

Printed: one JSON line with the metric, the roofline of the dominant kernel
(HIP-event timing of its launches in the solve's launch configuration), the
same per-step rooflines at the large single-system sizes, and the CPU oracle
timed on a bounded sample on this host (one thread and all threads).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import subprocess
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
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--learn", type=int, default=400,
                    help="in-situ learning steps before the warm-up and the timed window")
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of each CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-baseline", action="store_true", help="skip the comparison legs")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-systems leg")
    ap.add_argument("--no-scale", action="store_true", help="skip the large-size rooflines")
    ap.add_argument("--batched-cycles", type=int, default=3,
                    help="restart cycles per system in the batched leg")
    ap.add_argument("--config2", type=int, default=0, metavar="N",
                    help="also solve N steps of the 1024^2 FP64 stream from zero and from the "
                         "previous solution (minutes per step; off by default)")
    ap.add_argument("--config5", type=int, default=0, metavar="N",
                    help="also solve the batched leg's 72 uneven systems to rel. residual 1e-8 "
                         "for N right-hand sides each (a sample of configuration 5's 20)")
    ap.add_argument("--no-config3", action="store_true",
                    help="skip the mixed-precision configuration's solves to 1e-10 (160^3, 2048^2)")
    ap.add_argument("--records", default=None, metavar="PATH",
                    help="write every right-hand side's record of the stream as a JSON line")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--schedule", type=int, default=0, choices=(0, 1, 2, 3),
                    help="step schedule of the learned stream's solves (mlg_opts.schedule; 0 = "
                         "autotuned): pins the tuned choice for profiled runs, whose timings "
                         "the profiler shifts")
    ap.add_argument("--log-jsonl", default=None, metavar="PATH",
                    help="append one JSON line per right-hand side of the learned stream "
                         "(guess, Arnoldi steps, initial, fifth-iteration and final residuals, "
                         "time to solution, training) to PATH")
    ap.add_argument("--probe", default=None, metavar="KERNEL",
                    help="counter-collection run: a 256 MiB device copy (the byte-count "
                         "calibration) then every launch of KERNEL (step, dots, extend, update, "
                         "resid) in one restart cycle, in the learned-guess solve's launch "
                         "configuration; `net`: three inference calls (batch 1) and three "
                         "training steps (batch 8) of the guess network instead")
    ap.add_argument("--probe-grid", default=None,
                    help="with --probe: another workload, e.g. 1024x1024:fp64:30, "
                         "2048x2048:fp32:40 or 160x160x160:fp32:40")
    ap.add_argument("--probe-tile", type=int, default=0,
                    help="with --probe-grid: this tile index (1-based) instead of the autotuned "
                         "one; every step fused in the split form for step/sums, none otherwise")
    return ap.parse_args()


def kernel_roofline(mlg, shape, opts, b, tile, fused, split=0, reps=20, only=None):
    """Average launch duration of every solver kernel over one restart cycle,
    in the launch configuration of the solve (tuned tile and per-step sweep
    schedule; HIP events on the stream), with two byte counts per launch:
    `bytes`, what the kernel itself must move (the fused sweep reads the basis
    once), and `bytes_cgs2`, the CGS2 step's algorithmic bytes
    (2(j+1) + 1) n s of step j -- two sweeps over v_0..v_j and one vector
    written -- credited to the launch that completes the step."""
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
    step = lambda j: (2 * (j + 1) + 1) * n * s             # noqa: E731
    # the launches of one cycle: (kind, step index, bytes, CGS2 bytes)
    launches = [(mlg.MLG_K_DOTS, 0, 1 * n * s, 0)]         # w = A u_0 and |u_0|: read u_0
    for j in range(m):
        if (split >> j) & 1:
            # sums over workgroups; the sweep forms the coefficients itself
            launches.append((mlg.MLG_K_SUMS, j, 0, 0))
            launches.append((mlg.MLG_K_STEPC, j, (j + 3) * n * s, step(j)))
        elif (fused >> j) & 1:
            # read v_0..v_{j-1}, u_j; write v_j, u_{j+1}
            launches.append((mlg.MLG_K_COEF, j, 0, 0))     # one-workgroup sums
            launches.append((mlg.MLG_K_STEP, j, (j + 3) * n * s, step(j)))
        else:
            # separate sweeps: half of the step's CGS2 bytes to each
            launches.append((mlg.MLG_K_COEF, j, 0, 0))
            launches.append((mlg.MLG_K_EXTEND, j, (j + 3) * n * s, step(j) / 2))
            launches.append((mlg.MLG_K_DOTS, j + 1, (j + 2) * n * s, step(j) / 2))  # read v_0..v_j, u_{j+1}
    launches.append((mlg.MLG_K_COEF, m, 0, 0))
    launches.append((mlg.MLG_K_UPDATE, m, m * n * s + 2 * n * 8, m * n * s + 2 * n * 8))
    launches.append((mlg.MLG_K_RESIDUAL, m, 3 * n * 8, 3 * n * 8))   # read x, b; write r
    out = {}
    for kind, j, byts, cg in launches:
        name = mlg.KERNEL_NAMES[kind]
        if only is not None and name != only:
            continue
        us = mlg.mlg_kernel_bench(grid, fixed, ws, scratch, kind, j, reps)
        d = out.setdefault(name, {"launches_per_cycle": 0, "us": [], "bytes": [], "cgs2": []})
        d["launches_per_cycle"] += 1
        d["us"].append(us)
        d["bytes"].append(byts)
        d["cgs2"].append(cg)
    for d in out.values():
        d["avg_us"] = statistics.fmean(d["us"])
        d["avg_bytes"] = statistics.fmean(d["bytes"])
        d["avg_cgs2"] = statistics.fmean(d["cgs2"])
        d["cycle_us"] = sum(d["us"])
    del ws, scratch
    return out


def roofline_of(kr):
    """Dominant kernel (by time per cycle, among kernels that move data) and
    the whole cycle: achieved GB/s on the CGS2 byte model and on the bytes
    the kernels themselves move."""
    dom = max((k for k in kr if kr[k]["avg_bytes"] > 0), key=lambda k: kr[k]["cycle_us"])
    d = kr[dom]
    us = sum(v["cycle_us"] for v in kr.values())
    cg = sum(sum(v["cgs2"]) for v in kr.values())
    own = sum(sum(v["bytes"]) for v in kr.values())
    return {"kernel": dom, "avg_us": d["avg_us"],
            "achieved": d["avg_cgs2"] / (d["avg_us"] * 1e-6) / 1e9,
            "achieved_own_bytes": d["avg_bytes"] / (d["avg_us"] * 1e-6) / 1e9,
            "cycle_us": us, "cycle_GBs_cgs2": cg / (us * 1e-6) / 1e9,
            "cycle_GBs_own": own / (us * 1e-6) / 1e9}


def copy_rate(nbytes=256 << 20, reps=5):
    """HBM rate of a plain device-to-device copy (torch's copy kernel), read +
    write bytes over the HIP-event time of one copy (median of `reps`)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    s = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        b.copy_(a)
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / statistics.median(ts) / 1e9


def scale_rooflines(mlg, seed):
    """Per-step rooflines of one restart cycle at the large single-system
    sizes, whose Krylov basis does not fit the 256 MB last-level cache:
    1024^2 FP64 GMRES(30), 2048^2 and 160^3 FP32 basis GMRES(40), each in its
    autotuned launch configuration, on a drifting-Gaussian right-hand side."""
    from synthetic import DriftingGaussians
    out = {"copy_reference_GBs": copy_rate()}
    for shape, prec, m, src, sigma in [((1024, 1024), mlg.MLG_FP64, 30, 5, 0.02),
                                       ((2048, 2048), mlg.MLG_FP32_IR, 40, 5, 0.02),
                                       ((160, 160, 160), mlg.MLG_FP32_IR, 40, 5, 0.03)]:
        opts = mlg.Opts(restart_m=m, precision=prec, rtol=1e-10)
        tile, fused, split, _ = mlg.mlg_autotune(mlg.grid_of(shape), opts)
        b = torch.from_numpy(DriftingGaussians(shape, src, sigma, seed=seed).field(0)).cuda()
        kr = kernel_roofline(mlg, shape, opts, b, tile, fused, split, reps=10)
        r = roofline_of(kr)
        key = "x".join(map(str, shape)) + ("_fp64" if prec == mlg.MLG_FP64 else "_fp32") + f"_m{m}"
        r.update({"frac": r["achieved"] / HBM_PEAK_GBS,
                  "cycle_frac_cgs2": r["cycle_GBs_cgs2"] / HBM_PEAK_GBS,
                  "cycle_frac_own": r["cycle_GBs_own"] / HBM_PEAK_GBS,
                  # the bytes the kernel moves against a plain device copy
                  "kernel_own_vs_copy": r["achieved_own_bytes"] / out["copy_reference_GBs"],
                  "us_per_step": r["cycle_us"] / m,
                  "tile": list(mlg.mlg_tile_shape(len(shape), tile - 1)),
                  "fused_steps": bin(fused).count("1"), "split_steps": bin(split).count("1"),
                  "kernels": {k: {"avg_us": v["avg_us"], "per_cycle": v["launches_per_cycle"],
                                  "GB/s_own": (v["avg_bytes"] / v["avg_us"] / 1e3
                                               if v["avg_us"] > 0 else 0.0)}
                              for k, v in kr.items()}})
        out[key] = r
        del b
        torch.cuda.empty_cache()
    return out


def config3_leg(mlg, seed, budget_2d=20000):
    """The mixed-precision configuration solved to rel. residual 1e-10: FP32
    Krylov basis (GMRES(40), FP64 refinement) and, for the error the FP32
    path leaves, the FP64 basis on the same right-hand side.  160^3 runs to
    the tolerance; 2048^2 needs of the order of 10^5-10^6 restarted steps, so
    it runs a budget of steps and reports the residual reached and a
    projection of the steps to 1e-10 from the measured reduction per restart
    cycle (labelled as such)."""
    import math
    from synthetic import DriftingGaussians
    out = {}
    shape = (160, 160, 160)
    b = torch.from_numpy(DriftingGaussians(shape, 5, 0.03, seed=seed + 3).field(0)).cuda()
    grid = mlg.grid_of(shape)
    res = {}
    for name, prec in (("fp32_basis", mlg.MLG_FP32_IR), ("fp64_basis", mlg.MLG_FP64)):
        opts = mlg.Opts(restart_m=40, precision=prec, rtol=1e-10)
        mlg.mlg_autotune(grid, opts)
        ws = mlg.workspace(mlg.gmres_workspace_bytes(grid, opts))
        x = torch.zeros_like(b)
        st = mlg.gmres_solve(grid, b, x, opts, ws)
        res[name] = (x, st)
        del ws
    x32, s32 = res["fp32_basis"]
    x64, s64 = res["fp64_basis"]
    out["160x160x160"] = {
        "workload": "3D 7-point Poisson 160^3, 5 drifting Gaussians (sigma 0.03), GMRES(40), rtol 1e-10",
        "fp32_basis": {"iters": s32.iters, "cycles": s32.cycles, "seconds": s32.seconds,
                       "relres_true": s32.relres_true},
        "fp64_basis": {"iters": s64.iters, "cycles": s64.cycles, "seconds": s64.seconds,
                       "relres_true": s64.relres_true},
        "fp32_vs_fp64_rel_error": float((x32 - x64).norm() / x64.norm()),
        "speedup_fp32_basis": s64.seconds / s32.seconds}
    del res, x32, x64, b
    torch.cuda.empty_cache()
    shape = (2048, 2048)
    b = torch.from_numpy(DriftingGaussians(shape, 5, 0.02, seed=seed + 3).field(0)).cuda()
    grid = mlg.grid_of(shape)
    opts = mlg.Opts(restart_m=40, precision=mlg.MLG_FP32_IR, rtol=1e-10, max_iters=budget_2d)
    mlg.mlg_autotune(grid, opts)
    ws = mlg.workspace(mlg.gmres_workspace_bytes(grid, opts))
    x = torch.zeros_like(b)
    st = mlg.gmres_solve(grid, b, x, opts, ws, allow_not_converged=True)
    rate = st.relres_true ** (1.0 / max(1, st.cycles))        # mean reduction per cycle
    proj = (math.log(1e-10) / math.log(rate)) * 40 if 0.0 < rate < 1.0 else None
    out["2048x2048"] = {
        "workload": "2D 5-point Poisson 2048^2, 5 drifting Gaussians (sigma 0.02), GMRES(40), "
                    f"FP32 basis, a budget of {budget_2d} steps",
        "iters": st.iters, "cycles": st.cycles, "seconds": st.seconds,
        "relres_true": st.relres_true, "ms_per_step": 1e3 * st.seconds / max(1, st.iters),
        "projected_steps_to_1e-10": proj,
        "projected_seconds_to_1e-10": proj * st.seconds / max(1, st.iters) if proj else None,
        "projection": "steps = 40 log(1e-10) / log(mean reduction per cycle over the budget)"}
    del ws, x, b
    torch.cuda.empty_cache()
    return out


def config2_leg(mlg, seed, steps):
    """A sample of the 1024^2 FP64 stream: `steps` consecutive right-hand
    sides of five drifting Gaussians (sigma 0.02), each solved to rel. residual
    1e-8 with GMRES(30) from zero and from the previous solution (the
    classical initial guess), in the tuned launch configuration."""
    from synthetic import DriftingGaussians
    shape = (1024, 1024)
    gen = DriftingGaussians(shape, 5, 0.02, seed=seed + 2)
    grid = mlg.grid_of(shape)
    opts = mlg.Opts(restart_m=30, precision=mlg.MLG_FP64, rtol=1e-8)
    mlg.mlg_autotune(grid, opts)
    ws = mlg.workspace(mlg.gmres_workspace_bytes(grid, opts))
    prev = None
    recs = {"zero": [], "prev": []}
    for t in range(steps + 1):
        b = torch.from_numpy(gen.field(t)).cuda()
        x = torch.zeros_like(b)
        st = mlg.gmres_solve(grid, b, x, opts, ws)
        if t > 0:                                   # step 0 only seeds u_{t-1}
            recs["zero"].append((st.seconds, st.iters))
            xp = prev.clone()
            sp = mlg.gmres_solve(grid, b, xp, opts, ws)
            recs["prev"].append((sp.seconds, sp.iters))
        prev = x
        print(json.dumps({"progress": f"config2 step {t}"}), flush=True)
    out = {"workload": "2D 5-point Poisson 1024^2, 5 drifting Gaussians (sigma 0.02), GMRES(30) FP64, "
                       f"rtol 1e-8, steps 1..{steps} of the stream"}
    for k, v in recs.items():
        out[k] = {"tos_mean": statistics.fmean(s for s, _ in v),
                  "iters_mean": statistics.fmean(i for _, i in v)}
    out["prev_over_zero_iters"] = out["prev"]["iters_mean"] / out["zero"]["iters_mean"]
    del ws
    torch.cuda.empty_cache()
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
    # algorithmic bytes of one cycle per point (FP32 basis), CGS2 model: the
    # steps' two sweeps and one write, + update + residual
    per_point = 4 * sum(2 * (j + 1) + 1 for j in range(m)) + (4 * m + 16) + 24
    return {"systems": len(shapes), "points": n, "steps_per_system": steps,
            "seconds": dt, "us_per_step": 1e6 * dt / steps,
            "point_steps_per_s": n * steps / dt,
            "GBs_cgs2": n * per_point * cycles / dt / 1e9,
            "iters_ok": all(st.iters == steps for st in stats)}


def config5_leg(mlg, seed, nrhs, m=30):
    """Configuration 5 to tolerance: the batched leg's 72 uneven systems (same
    seeded sizes), `nrhs` drifting-Gaussian right-hand sides each, FP32-basis
    GMRES(30) with FP64 refinement to relative residual 1e-8.  One batched call
    per right-hand side over all systems (fixed device buffers, so the engine
    keeps its plan), each system starting from its previous solution (the
    first from zero); a progress line after every call."""
    from synthetic import DriftingGaussians
    rng = np.random.default_rng(seed)
    shapes = [(int(s), int(s)) for s in rng.choice([128, 192, 256, 384, 512, 768, 1024], 64)]
    shapes += [(int(s),) * 3 for s in rng.integers(64, 129, 8)]
    opts = mlg.Opts(restart_m=m, precision=mlg.MLG_FP32_IR, rtol=1e-8)
    for dim in (2, 3):
        big = max((sh for sh in shapes if len(sh) == dim), key=lambda sh: int(np.prod(sh)))
        mlg.mlg_autotune(mlg.grid_of(big), mlg.Opts(restart_m=m, precision=mlg.MLG_FP32_IR))
    gens = [DriftingGaussians(sh, 4, 0.03, seed=seed + i) for i, sh in enumerate(shapes)]
    bs = [torch.zeros((1,) + sh, dtype=torch.float64, device="cuda") for sh in shapes]
    xs = [torch.zeros_like(b) for b in bs]
    systems = [mlg.make_system(b, x, 1) for b, x in zip(bs, xs)]
    ws = mlg.workspace(mlg.gmres_batched_workspace_bytes(systems, opts))
    steps = [[] for _ in shapes]
    worst, ok, total = 0.0, True, 0.0
    for t in range(nrhs):
        for b, g in zip(bs, gens):
            b[0].copy_(torch.from_numpy(g.field(t)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = mlg.gmres_solve_batched(systems, opts, ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        total += dt
        for k, st in enumerate(stats):
            steps[k].append(st.iters)
        ok = ok and all(st.status == 0 for st in stats)
        worst = max([worst] + [st.relres_true for st in stats])
        print(json.dumps({"progress": f"config5 rhs {t}", "seconds": round(dt, 2),
                          "max_steps": max(st.iters for st in stats), "all_converged": ok}),
              flush=True)
    by_size = {}
    for k, sh in enumerate(shapes):
        by_size.setdefault("x".join(map(str, sh)), []).append(steps[k])
    return {"systems": len(shapes), "rhs_per_system": nrhs,
            "points": sum(int(np.prod(sh)) for sh in shapes), "seconds": total,
            "all_converged": ok, "max_relres_true": worst,
            "max_steps": max(max(v) for v in steps),
            "mean_steps_by_size_and_rhs": {
                k: [float(np.mean([v[t] for v in lst])) for t in range(nrhs)]
                for k, lst in sorted(by_size.items(), key=lambda kv: -int(kv[0].split("x")[0]))}}


def counter_traffic(kernel, shape, precision_tag, m, tile):
    """HBM bytes per launch of `kernel` on tile shape `tile` (e.g. "64x16") from
    the committed FETCH_SIZE/WRITE_SIZE summary
    (profiles/<kernel>_<H>x<W>_traffic.md), or None when there is none for this
    workload or the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{'x'.join(map(str, shape))}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    if fields.get("workload_key") != f"{kernel} {'x'.join(map(str, shape))} {precision_tag} m{m}":
        return None
    h = hashlib.sha256()
    for src in fields.get("kernel_sources", "").split():
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != fields.get("kernel_source_sha256"):
        return None
    v = fields.get(f"traffic_bytes_per_launch tile={tile}")
    return float(v) if v else None


def host_cpu():
    """CPU model, sockets and cores of this host (from lscpu)."""
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    sockets = int(info.get("Socket(s)", "0") or 0)
    cps = int(info.get("Core(s) per socket", "0") or 0)
    return {"model": info.get("Model name", "unknown"), "sockets": sockets,
            "physical_cores": sockets * cps, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(shape, m, f0, plain_iters, budget_s):
    """The FP64 CPU oracle on a bounded sample: a fixed number of Arnoldi
    steps of plain GMRES(m) on the first timed RHS, projected to the
    plain-GMRES iteration count of the timed window; with one thread and with
    every thread this process may use (OpenMP over grid rows; the results are
    bitwise the same)."""
    from oracle import gmres as og
    cpu = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or cpu["usable_cpus"]
    runs = {}
    for nt in sorted({1, threads}):
        og.set_threads(nt)
        t0 = time.perf_counter()
        og.gmres(f0, m=m, fixed_iters=m)                   # one cycle, to size the sample
        per_cycle = time.perf_counter() - t0
        k = max(1, int(budget_s / max(per_cycle, 1e-6))) * m
        t0 = time.perf_counter()
        og.gmres(f0, m=m, fixed_iters=k)
        dt = time.perf_counter() - t0
        runs[nt] = {"steps": k, "seconds": dt, "ms_per_step": 1e3 * dt / k,
                    "s_per_rhs": dt / k * plain_iters}
    og.set_threads(1)
    best = min(runs, key=lambda t: runs[t]["s_per_rhs"])
    return {"value": runs[best]["s_per_rhs"], "unit": "s/RHS", "cores": best, "kind": "oracle",
            "sample": f"FP64 CGS2 GMRES({m}) Arnoldi steps of the first timed RHS on "
                      f"{'x'.join(map(str, shape))}, timed with "
                      + " and ".join(f"{t} thread(s) ({r['steps']} steps, {r['seconds']:.1f} s, "
                                     f"{r['ms_per_step']:.2f} ms/step)" for t, r in runs.items())
                      + f", projected to the {plain_iters:.0f} steps plain GMRES needs per RHS",
            "threads": {str(t): r for t, r in runs.items()}, "host": cpu}


def legs_on_window(mlg, sv, fields, prevs, t0, args):
    """The comparison legs on the timed right-hand sides, each started from the
    same previous solution the learned run had."""
    from paper_2103_10975_amd import stream as st
    shape = sv.shape
    grid = sv.grid
    K = sv.net_cfg.skip_modes
    fp32 = mlg.Opts(restart_m=args.restart, precision=mlg.MLG_FP32_IR, rtol=args.rtol)
    fp64 = mlg.Opts(restart_m=args.restart, precision=mlg.MLG_FP64, rtol=args.rtol)
    # the FP64 baselines in their own tuned launch configuration (the FP32
    # ones share the stream's)
    mlg.mlg_autotune(grid, fp64)
    ws = {p: mlg.workspace(mlg.gmres_workspace_bytes(grid, o)) for p, o in
          ((0, fp64), (1, fp32))}
    # the band at its analytic optimum (c_u / lambda_kl of the 5-point
    # Laplacian), convolutional output zero: nothing trained
    ana_cfg = mlg.NetCfg(skip_modes=K, seed=args.seed)
    ana = torch.zeros(mlg.guess_net_param_bytes(ana_cfg), dtype=torch.uint8, device="cuda")
    mlg.guess_net_init(ana_cfg, ana)
    H, W = shape
    k = np.arange(1, K + 1, dtype=np.float64)
    lam = (4.0 * (H + 1) ** 2 * np.sin(k * np.pi / (2 * (H + 1))) ** 2)[:, None] + \
          (4.0 * (W + 1) ** 2 * np.sin(k * np.pi / (2 * (W + 1))) ** 2)[None, :]
    mlg.net_set_band(ana_cfg, ana, 2.0 * np.pi ** 2 / lam)
    ana_ws = mlg.workspace(mlg.guess_net_workspace_bytes(ana_cfg, grid, 1, False))
    # the trained network with its convolutional output switched off
    bo = sv.params.clone()
    v = mlg.net_views(sv.net_cfg, bo)
    for i in (11, 12):                                  # conv6.w, conv6.b
        o0 = mlg.guess_net_param_offset(sv.net_cfg, i)
        o1 = mlg.guess_net_param_offset(sv.net_cfg, i + 1)
        v["master"][o0:o1].zero_()
    mlg.guess_net_refresh(sv.net_cfg, bo)

    def guess_fn(kind):
        def f(t, up, x):
            if kind == "zero":
                x.zero_()
            elif kind == "prev":
                x.copy_(up)
            elif kind == "config_net":
                sv.shadow_guess(0, fields[t], up, x)
            elif kind == "band_analytic":
                mlg.guess_net_infer(ana_cfg, ana, fields[t].view(1, *shape), up.view(1, *shape),
                                    x.view(1, *shape), ana_ws)
            elif kind == "learned_band_only":
                mlg.guess_net_infer(sv.net_cfg, bo, fields[t].view(1, *shape),
                                    up.view(1, *shape), x.view(1, *shape), sv.ws_infer)
        return f

    legs = {}
    x = torch.empty_like(prevs[0])
    for name, kind, prec in [("plain_fp64_zero", "zero", 0), ("fp64_prev", "prev", 0),
                             ("fp32_prev", "prev", 1), ("config_net_fp32", "config_net", 1),
                             ("learned_band_only_fp32", "learned_band_only", 1),
                             ("band_analytic_untrained_fp32", "band_analytic", 1)]:
        g = guess_fn(kind)
        recs = []
        for i, up in enumerate(prevs):
            t = t0 + i
            torch.cuda.synchronize()
            ts = time.perf_counter()
            g(t, up, x)
            stt = mlg.gmres_solve(grid, fields[t], x, fp64 if prec == 0 else fp32, ws[prec])
            recs.append((time.perf_counter() - ts, stt))
        legs[name] = leg_summary(recs)
    return legs


def leg_summary(recs):
    tos = [r[0] for r in recs]
    sts = [r[1] for r in recs]
    return {"tos_mean": statistics.fmean(tos), "tos_median": statistics.median(tos),
            "tos_p90": float(np.percentile(tos, 90)),
            "iters_mean": statistics.fmean(s.iters for s in sts),
            "relres_init_median": statistics.median(s.relres_init for s in sts),
            "E_k_median": statistics.median(s.relres_first_cycle for s in sts),
            "relres_iter5_median": statistics.median(s.relres_iter5 for s in sts),
            "relres_true_max": max(s.relres_true for s in sts)}


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
    if args.probe == "net":
        probe_net(mlg, shape, args)
        return
    if args.probe:
        probe(mlg, shape, args)
        return
    gen = DriftingGaussians(shape, 4, 0.03, seed=args.seed)
    t_warm, t_timed = args.learn, args.learn + args.warmup
    total = t_timed + args.steps
    fields = [torch.from_numpy(gen.field(t)).cuda() for t in range(total)]

    # the learned method, with the configuration's network without a band
    # path as a shadow trained on the same batches
    shadow = mlg.NetCfg(skip_modes=0, seed=args.seed)
    sv = StreamSolver(shape, guess="learned", restart_m=args.restart, rtol=args.rtol,
                      precision=mlg.MLG_FP32_IR, seed=args.seed, time_train=False,
                      shadow_cfgs=[shadow], log_path=args.log_jsonl)
    if args.schedule:
        sv.opts.schedule = args.schedule
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    for t in range(t_warm):
        sv.step(fields[t])
    torch.cuda.synchronize()
    learn_s = time.perf_counter() - ts0
    sv.train_shadows = False                  # the shadows are frozen from here on
    ts1 = time.perf_counter()
    for t in range(t_warm, t_timed):
        sv.step(fields[t])
    torch.cuda.synchronize()
    warm_s = time.perf_counter() - ts1
    prevs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(t_timed, total):
        prevs.append(sv.u_prev.clone())
        sv.step(fields[t])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed = sv.records[t_timed:]
    tos_learned = statistics.fmean(r.tos for r in timed)
    if args.records:
        import dataclasses
        with open(args.records, "w") as fh:
            for r in sv.records:
                fh.write(json.dumps({"phase": "learn" if r.t < t_warm else
                                     ("warmup" if r.t < t_timed else "timed"),
                                     **dataclasses.asdict(r)}) + "\n")
    learn = sv.records[:t_warm]
    K = sv.net_cfg.skip_modes
    w = mlg.net_band_weights(sv.net_cfg, sv.params).cpu().numpy()
    H, W = shape
    kk = np.arange(1, K + 1, dtype=np.float64)
    lam = (4.0 * (H + 1) ** 2 * np.sin(kk * np.pi / (2 * (H + 1))) ** 2)[:, None] + \
          (4.0 * (W + 1) ** 2 * np.sin(kk * np.pi / (2 * (W + 1))) ** 2)[None, :]
    werr = np.abs(w * lam / (2.0 * np.pi ** 2) - 1.0)
    stream_total_s = learn_s + warm_s + elapsed
    solve_s = sum(r.tos for r in sv.records)
    result = {
        "metric": METRIC, "value": tos_learned, "unit": "s/RHS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (f32 Krylov basis) + bf16 network", "data": "synthetic",
        "config": {"workload": f"2D 5-point Poisson {shape[0]}x{shape[1]}, 4 drifting Gaussian "
                               f"sources (sigma 0.03), GMRES({args.restart}), rtol {args.rtol}, "
                               "in-situ learned guess + FP32-basis refinement vs plain FP64 GMRES",
                   "grid": list(shape), "restart_m": args.restart, "rtol": args.rtol,
                   "seed": args.seed, "learn_steps": args.learn, "band_modes": K,
                   "timed_steps": [t_timed, total - 1]},
        "learned": {"tos_mean": tos_learned, "tos_median": statistics.median(r.tos for r in timed),
                    "tos_p90": float(np.percentile([r.tos for r in timed], 90)),
                    "iters_mean": statistics.fmean(r.iters for r in timed),
                    "relres_init_median": statistics.median(r.relres_init for r in timed),
                    "E_k_median": statistics.median(r.relres_first_cycle for r in timed),
                    "relres_iter5_median": statistics.median(r.relres_iter5 for r in timed),
                    "guess_kinds": sorted(set(r.guess for r in timed)),
                    "conv_output_gain": mlg.net_output_gain(sv.net_cfg, sv.params),
                    "band_weight_error_vs_analytic": {
                        "max_16x16": float(werr[:16, :16].max()), "median_band": float(np.median(werr))}},
        # the whole stream of the in-situ method, training included
        "stream": {"steps": total, "seconds": stream_total_s,
                   "solve_seconds": solve_s, "train_and_overhead_seconds": stream_total_s - solve_s,
                   "tos_mean": solve_s / total,
                   "iters_mean": statistics.fmean(r.iters for r in sv.records),
                   "learn_phase": {"steps": args.learn, "seconds": learn_s,
                                   "tos_mean": statistics.fmean(r.tos for r in learn),
                                   "iters_mean": statistics.fmean(r.iters for r in learn)},
                   "train_ms_per_step_timed": 1e3 * (elapsed - sum(r.tos for r in timed)) / args.steps},
    }
    print(json.dumps({"progress": "timed window done", "value": tos_learned}), flush=True)

    if not args.no_baseline:
        legs = legs_on_window(mlg, sv, fields, prevs, t_timed, args)
        result["legs"] = legs
        result["speedup_vs_plain_fp64"] = legs["plain_fp64_zero"]["tos_mean"] / tos_learned
        result["speedup_vs_prev_fp64"] = legs["fp64_prev"]["tos_mean"] / tos_learned
        result["speedup_vs_prev_fp32"] = legs["fp32_prev"]["tos_mean"] / tos_learned
        result["iters_learned_over_prev_fp32"] = (result["learned"]["iters_mean"]
                                                  / legs["fp32_prev"]["iters_mean"])
        result["stream"]["plain_fp64_projected_seconds"] = legs["plain_fp64_zero"]["tos_mean"] * total
        print(json.dumps({"progress": "legs done"}), flush=True)

    # roofline of the dominant kernel of the learned-guess solve
    tile, fused, split, launch = sv.tuned
    if args.schedule:                     # the pinned schedule, for every step
        allm = (1 << args.restart) - 1
        fused = allm if args.schedule >= 2 else 0
        split = allm if args.schedule == 3 else 0
        result["config"]["schedule"] = args.schedule
    tshape = mlg.mlg_tile_shape(2, tile - 1)
    result["config"]["tile"] = list(tshape)
    result["config"]["launch"] = "direct" if launch == 2 else "graph"
    result["config"]["fused_steps"] = bin(fused).count("1")
    result["config"]["split_steps"] = bin(split).count("1")
    kr = kernel_roofline(mlg, shape, sv.opts, fields[0], tile, fused, split)
    r = roofline_of(kr)
    tag = "fp64" if sv.opts.precision == mlg.MLG_FP64 else "fp32"
    result["roofline"] = {"kernel": r["kernel"], "bound": "hbm", "achieved": r["achieved"],
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": r["achieved"] / HBM_PEAK_GBS,
                          "traffic": counter_traffic(r["kernel"], shape, tag, args.restart,
                                                     f"{tshape[0]}x{tshape[1]}"),
                          "bytes_model": "CGS2 (2(j+1)+1) n s per Arnoldi step",
                          "achieved_own_bytes": r["achieved_own_bytes"],
                          "avg_us": r["avg_us"], "cycle_us": r["cycle_us"],
                          "cycle_frac_cgs2": r["cycle_GBs_cgs2"] / HBM_PEAK_GBS}
    result["kernels"] = {k: {"avg_us": v["avg_us"], "per_cycle": v["launches_per_cycle"],
                             "GB/s_own": v["avg_bytes"] / v["avg_us"] / 1e3 if v["avg_us"] else 0,
                             "cycle_us": v["cycle_us"]} for k, v in kr.items()}
    if not args.no_scale:
        result["roofline_at_scale"] = scale_rooflines(mlg, args.seed)
        print(json.dumps({"progress": "large-size rooflines done"}), flush=True)

    if not args.no_config3:
        result["config3"] = config3_leg(mlg, args.seed)
    if args.config2 > 0:
        result["config2_sample"] = config2_leg(mlg, args.seed, args.config2)
    if args.config5 > 0:
        result["config5_sample"] = config5_leg(mlg, args.seed, args.config5)
        print(json.dumps({"progress": "mixed-precision configuration done"}), flush=True)
    if not args.no_batched:
        result["batched"] = batched_leg(mlg, args.seed, args.batched_cycles)

    if not args.no_cpu:
        plain_iters = (result.get("legs", {}).get("plain_fp64_zero", {}).get("iters_mean")
                       or result["learned"]["iters_mean"])
        result["cpu_baseline"] = cpu_baseline(shape, args.restart, fields[t_timed].cpu().numpy(),
                                              plain_iters, args.cpu_seconds)
    line = json.dumps(result)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as fh:
            fh.write(line + "\n")


def probe_net(mlg, shape, args):
    """Guess-network launches for counter runs: the 256 MiB copy calibration,
    then three inference calls (batch 1) and three training steps (batch 8,
    the replay batch) of the benchmark's network at the benchmark's grid."""
    from synthetic import DriftingGaussians
    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")       # 256 MiB
    for _ in range(3):
        a.clone()
    torch.cuda.synchronize()
    gen = DriftingGaussians(shape, 4, 0.03, seed=args.seed)
    fs = [torch.from_numpy(gen.field(t)).cuda() for t in range(10)]
    grid = mlg.grid_of(shape)
    cfg = mlg.NetCfg(channels=32, modes=16, skip_modes=min(64, *shape), seed=1)
    params = torch.zeros(mlg.guess_net_param_bytes(cfg), dtype=torch.uint8, device="cuda")
    mlg.guess_net_init(cfg, params)
    wsi = mlg.workspace(mlg.guess_net_workspace_bytes(cfg, grid, 1, False))
    wst = mlg.workspace(mlg.guess_net_workspace_bytes(cfg, grid, 8, True))
    u = 0.01 * fs[0]
    x = torch.empty_like(u)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for _ in range(3):
        mlg.guess_net_infer(cfg, params, fs[1].view(1, *shape), u.view(1, *shape),
                            x.view(1, *shape), wsi)
    for _ in range(3):
        mlg.guess_net_train_step(cfg, params, fs[:8], [u] * 8, fs[1:9], wst, loss)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "net", "workload": "x".join(map(str, shape)),
                      "copy_bytes": 2 * a.numel() * 4}), flush=True)


def probe(mlg, shape, args):
    """Launches for hardware-counter runs (no timing is reported): a 256 MiB
    device copy (the byte-count calibration), then one restart cycle's
    launches of the probed kernel, each step index once.  On the benchmark's
    workload: for every tile shape, in the learned-guess solve's configuration
    (fused steps in the split form for `step` and `sums`).  With --probe-grid:
    that workload in its autotuned configuration."""
    from synthetic import DriftingGaussians
    names = {v.replace("k_", ""): v for v in mlg.KERNEL_NAMES.values()}
    if args.probe not in names:
        raise SystemExit(f"--probe takes one of {sorted(names)}")
    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")       # 256 MiB
    for _ in range(3):
        a.clone()
    torch.cuda.synchronize()
    if args.probe_grid:
        dims, prec, m = args.probe_grid.split(":")
        shape = tuple(int(v) for v in dims.split("x"))
        opts = mlg.Opts(restart_m=int(m), rtol=1e-10,
                        precision=mlg.MLG_FP64 if prec == "fp64" else mlg.MLG_FP32_IR)
        if args.probe_tile:
            allm = (1 << int(m)) - 1 if args.probe in ("step", "sums") and len(shape) == 2 else 0
            runs = [(args.probe_tile, allm, allm)]
        else:
            runs = [mlg.mlg_autotune(mlg.grid_of(shape), opts)[:3]]
    else:
        opts = mlg.Opts(restart_m=args.restart, rtol=args.rtol, precision=mlg.MLG_FP32_IR)
        fused = (1 << args.restart) - 1 if args.probe in ("step", "sums") else 0
        runs = [(t, fused, fused) for t in range(1, mlg.mlg_tile_count(2) + 1)]
    f0 = torch.from_numpy(DriftingGaussians(shape, 4, 0.03, seed=args.seed).field(0)).cuda()
    out = {}
    for tile, fused, split in runs:
        r = kernel_roofline(mlg, shape, opts, f0, tile, fused, split, reps=1,
                            only=names[args.probe])
        ts = mlg.mlg_tile_shape(len(shape), tile - 1)
        key = "x".join(map(str, ts[:len(shape)]))
        out[key] = {"launches": r[names[args.probe]]["launches_per_cycle"],
                    "avg_bytes": r[names[args.probe]]["avg_bytes"],
                    "avg_cgs2": r[names[args.probe]]["avg_cgs2"]}
    torch.cuda.synchronize()
    print(json.dumps({"probe": args.probe, "workload": "x".join(map(str, shape)),
                      "copy_bytes": 2 * a.numel() * 4, "per_tile": out}), flush=True)


if __name__ == "__main__":
    main()
