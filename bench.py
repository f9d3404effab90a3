"""Throughput of the fused D2Q9 EOS-multiphase step on one MI355X.

A step is one pass of the whole hot path (pull streaming with walls and ends,
density and EOS field, nonideal force, velocity-shift MRT collision, wall
shear/pressure diagnostics with FP64 summaries) over the 4096x512 plug-in-channel
workload, FP32 storage and arithmetic.  Inputs are resident in HBM before the
timed region; W warm-up steps, then exactly K timed steps between two
synchronisations.  Prints one JSON line.

MLUPS = nx*ny*K / t / 1e6.  The roofline uses the algorithmic traffic of the
method: 9 populations read + 9 written per node and step (72 B in FP32, 36 B in
FP16/BF16, 144 B in FP64) against the 8 TB/s HBM3E peak.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"f64": 144, "f32": 72, "f32d": 72, "f32s": 72, "f16s": 36, "bf16s": 36}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def make_lattice(w: dict, check_every: int):
    from paper_2103_08301_amd import Lattice

    lat = Lattice(w["nx"], w["ny"], w["tau"], storage=w["storage"], check_every=check_every, **w["params"])
    pl = w["plug"]
    lat.init_plug(pl["plug_len"], pl["film"], pl["x_center"], pl["noise_amp"], pl["seed"])
    return lat


def time_steps(w: dict, steps: int, warmup: int):
    """Returns (seconds for `steps` timed steps, lattice)."""
    import torch

    lat = make_lattice(w, check_every=max(steps, warmup, 1))
    if warmup:
        lat.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    t0 = time.perf_counter()
    lat.step(steps)
    stop.record(lat.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu = start.elapsed_time(stop) / 1e3
    return gpu, wall, lat


def cpu_baseline(w: dict, budget_s: float) -> dict:
    """The oracle as it stands, on a bounded sample of the same workload."""
    import oracle

    keys = {"T_over_Tc", "dp"}
    p = oracle.params(tau=w["tau"], **{k: v for k, v in w["params"].items() if k in keys})
    sim = oracle.Sim(w["nx"], w["ny"], p)
    pl = w["plug"]
    sim.init_plug(pl["plug_len"], pl["film"], pl["x_center"], pl["noise_amp"], pl["seed"])
    t0 = time.perf_counter()
    sim.step(1)
    one = time.perf_counter() - t0
    n = max(1, min(1000, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    sim.step(n)
    dt = time.perf_counter() - t0
    return {"value": w["nx"] * w["ny"] * n / dt / 1e6, "unit": "MLUPS", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{n} steps of the {w['nx']}x{w['ny']} workload in FP64 on the host ({dt:.1f} s)"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f32", choices=sorted(BYTES_PER_NODE))
    ap.add_argument("--workload", default="large", choices=["large", "large-stable", "out-of-cache"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-control", action="store_true", help="skip the stable-physics control run")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes 10 times (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        return 2
    if "RANK" in os.environ and os.environ.get("WORLD_SIZE", "1") != "1":
        print("bench.py: multi-rank launch is not supported (one GPU only)", file=sys.stderr)
        return 2

    import torch

    from paper_2103_08301_amd import lbm, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 10}), flush=True)
        return 0
    lbm.library()  # fail loudly if the HIP library is missing

    w = {"large": workloads.plug_large, "large-stable": workloads.plug_large_stable,
         "out-of-cache": workloads.plug_out_of_cache}[args.workload](args.storage)
    nodes = w["nx"] * w["ny"]
    log(f"workload: {w['name']}; warmup {args.warmup}, timed {args.steps}")
    gpu_s, wall_s, lat = time_steps(w, args.steps, args.warmup)
    chk = lat.check()
    mlups = nodes * args.steps / gpu_s / 1e6
    ms_per_step = gpu_s * 1e3 / args.steps
    bpn = BYTES_PER_NODE[args.storage]
    achieved = bpn * nodes / (gpu_s / args.steps) / 1e9
    log(f"{mlups:.0f} MLUPS, {ms_per_step * 1e3:.2f} us/step, {achieved:.0f} GB/s algorithmic "
        f"(wall {wall_s:.3f} s); check: {chk}")
    out = {
        "metric": "MLUPS (D2Q9 EOS-multiphase step, 4096x512 plug-in-channel)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "f32d": "f32-store/f64", "f32s": "f32-shifted/f32",
                  "f16s": "f16-store/f32", "bf16s": "bf16-store/f32"}[args.storage],
        "data": "synthetic",
        "config": {"workload": w["name"], "nx": w["nx"], "ny": w["ny"], "tau": w["tau"], **w["params"],
                   **{k: v for k, v in w["plug"].items() if k != "x_center"}, "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_node": bpn, "kernel": "step_kernel (fused pull-stream/force/MRT/wall diagnostics)"},
        "physics": {"unstable_step": chk["unstable_step"], "vmax": chk["vmax"], "nan_cells": chk["nan_count"]},
    }
    if not args.no_control and args.workload == "large":
        ctl = workloads.plug_large_stable(args.storage)
        cg, _, cl = time_steps(ctl, args.steps, args.warmup)
        cc = cl.check()
        out["stable_control"] = {"workload": ctl["name"], "value": round(nodes * args.steps / cg / 1e6, 1),
                                 "unit": "MLUPS", "unstable_step": cc["unstable_step"], "vmax": cc["vmax"]}
        log(f"control: {out['stable_control']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
