"""Build the HIP library libmlgmres.so for gfx950 (in-tree)."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmlgmres.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions stay off (wrong results have been seen with
         # some of their forms); hipcc's host pass warns that it ignores this.
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-munsafe-fp-atomics"]


# sweeps.hip holds the per-tile sweep kernels of one (basis precision, grid
# dimension, tile index); it is compiled once per triple so that the
# instantiations build in parallel.
SWEEP_UNITS = [(p, 2, t) for p in (0, 1) for t in range(5)] + \
              [(p, 3, t) for p in (0, 1) for t in range(5)]


def _units():
    out = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        if os.path.basename(src) == "sweeps.hip":
            for p, d, t in SWEEP_UNITS:
                out.append((src, f"sweeps_p{p}_d{d}_t{t}",
                            [f"-DMLG_SWEEP_PREC={p}", f"-DMLG_SWEEP_DIM={d}",
                             f"-DMLG_SWEEP_TILE={t}"]))
        else:
            out.append((src, os.path.basename(src), []))
    return out


def _compile(unit) -> str:
    src, name, defs = unit
    obj = os.path.join(OUT, name + ".o")
    cmd = [HIPCC, *FLAGS, *defs, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr[-6000:]}")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(OUT, exist_ok=True)
    units = _units()
    # the largest units first, so that they do not finish last alone
    units.sort(key=lambda u: (not u[1].startswith(("sweeps_p0_d2", "sweeps_p1_d2")),
                              u[1] != "net.hip"))
    jobs = jobs or min(len(units), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-6000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else None))
