"""Throughput of the fused D2Q9 EOS-multiphase step on one MI355X.

A step is one pass of the whole hot path (pull streaming with bounce-back walls
and extrapolated ends, density and EOS field, nonideal force of eq. 2.17,
velocity-shift MRT collision, wall shear/pressure diagnostics with FP64
per-step summaries) over the 4096x512 plug-in-channel workload.  Inputs are
resident in HBM before the timed region; W warm-up steps, then exactly K timed
steps between two device synchronisations, timed with HIP events on the stream
the kernels run on.  Prints one JSON line.

MLUPS = nx*ny*K / t / 1e6.  The roofline uses the algorithmic traffic of the
method: 9 populations read + 9 written per node and step (72 B in FP32, 36 B in
FP16/BF16 storage, 144 B in FP64) against the 8 TB/s HBM3E peak.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"f64": 144, "f32": 72, "f32d": 72, "f32s": 72, "f16s": 36, "bf16s": 36, "f16r": 36}
DTYPE = {"f32": "f32", "f64": "f64", "f32d": "f32-store/f64", "f32s": "f32-shifted/f32",
         "f16s": "f16-store/f32", "bf16s": "bf16-store/f32", "f16r": "f16-store-stochastic/f32"}
KERNEL_SRC = os.path.join(ROOT, "paper_2103_08301_amd", "csrc", "lbm_device.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tile_kernel_4096x512_f32_traffic.json")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


METRIC = "MLUPS and % HBM roofline, D2Q9 4096\u00d7512 FP32 vs FP16-store; adjoint/fwd time"
GRAPH_STEPS = 0  # steps per captured HIP graph (--graph-steps)
AUTOTUNE = False  # time every tile shape after the warm-up and keep the fastest (--autotune; always for --batch)


def make_lattice(w: dict, check_every: int):
    from paper_2103_08301_amd import Lattice

    lat = Lattice(w["nx"], w["ny"], w["tau"], storage=w["storage"], check_every=check_every,
                  graph_steps=GRAPH_STEPS, **w["params"])
    pl = w["plug"]
    lat.init_plug(pl["plug_len"], pl["film"], pl["x_center"], pl["noise_amp"], pl["seed"])
    return lat


CHECK_EVERY = 1000  # the library's default stability/interface check cadence


def time_steps(w: dict, steps: int, warmup: int, tune: bool = False):
    """Seconds for `steps` timed steps (HIP events on the library's stream), wall seconds, lattice.

    The timed call is one lbm_step of `steps` steps with the library's default check cadence; the
    HIP graphs it replays are captured beforehand (lbm_capture), so no capture falls in the timed
    region.  Every step's wall diagnostics are reduced on the device inside it.  With `tune` (or
    --autotune) the library's autotuner picks the launch configuration after the warm-up."""
    import torch

    lat = make_lattice(w, check_every=CHECK_EVERY)
    if warmup:
        lat.step(warmup)
    lat.tuned = lat.autotune(50) if (AUTOTUNE or tune) else None
    if lat.tuned:
        log(f"autotune: {lat.tuned}")
    lat.capture(steps)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    t0 = time.perf_counter()
    lat.step(steps)
    stop.record(lat.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / 1e3, wall, lat


_ORACLE_SAMPLE = r"""
import json, os, sys, time
sys.path.insert(0, sys.argv[1])
import oracle
w = json.loads(sys.argv[2])
budget = float(sys.argv[3])
keys = {"T_over_Tc", "dp"}
p = oracle.params(tau=w["tau"], **{k: v for k, v in w["params"].items() if k in keys})
sim = oracle.Sim(w["nx"], w["ny"], p)
pl = w["plug"]
sim.init_plug(pl["plug_len"], pl["film"], float("nan") if pl["x_center"] is None else pl["x_center"],
              pl["noise_amp"], pl["seed"])
t0 = time.perf_counter()
sim.step(1)
one = time.perf_counter() - t0
n = max(1, min(1000, int(budget / max(one, 1e-6))))
t0 = time.perf_counter()
sim.step(n)
dt = time.perf_counter() - t0
print(json.dumps({"steps": n, "seconds": dt, "threads": oracle.threads()}))
"""


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w: dict, budget_s: float) -> dict:
    """The oracle as it stands, on a bounded sample of the same workload, with all host threads and with one
    (each in a child process, so that OMP_NUM_THREADS takes effect)."""
    import subprocess

    spec = json.dumps({k: (None if isinstance(v, float) and v != v else v) for k, v in w.items() if k != "params"}
                      | {"params": w["params"], "plug": {k: (None if isinstance(v, float) and v != v else v)
                                                         for k, v in w["plug"].items()}})
    runs = {}
    for label, nthreads in (("all", None), ("one", 1)):
        env = dict(os.environ)
        if nthreads:
            env["OMP_NUM_THREADS"] = str(nthreads)
        out = subprocess.run([sys.executable, "-c", _ORACLE_SAMPLE, ROOT, spec,
                              str(budget_s if nthreads is None else budget_s / 2)],
                             capture_output=True, text=True, env=env, timeout=600)
        if out.returncode != 0:
            raise RuntimeError(f"oracle sample failed: {out.stderr[-2000:]}")
        runs[label] = json.loads(out.stdout.strip().splitlines()[-1])
    nodes = w["nx"] * w["ny"]
    a, o = runs["all"], runs["one"]
    return {"value": round(nodes * a["steps"] / a["seconds"] / 1e6, 2), "unit": "MLUPS", "cores": a["threads"],
            "kind": "oracle",
            "sample": f"{a['steps']} steps of the {w['nx']}x{w['ny']} workload, FP64 oracle on the host "
                      f"({a['seconds']:.1f} s, {a['threads']} threads)",
            "one_thread": {"value": round(nodes * o["steps"] / o["seconds"] / 1e6, 2), "unit": "MLUPS",
                           "sample": f"{o['steps']} steps ({o['seconds']:.1f} s)"},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def finite(v):
    """JSON has no NaN/Infinity: non-finite numbers become null."""
    if isinstance(v, float):
        return v if v == v and abs(v) != float("inf") else None
    if isinstance(v, dict):
        return {k: finite(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [finite(x) for x in v]
    return v


def measured_traffic(storage: str, shape=(8, 4)):
    """HBM bytes per launch from the committed counter profile, if it was taken on this kernel source and shape."""
    if storage != "f32" or tuple(shape) != (8, 4) or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    return t["bytes_per_launch"] if t.get("kernel_source_sha256_16") == kernel_hash() else None


def size_sweep(storage: str) -> int:
    """Step time against grid size (same physics as the timed workload): fits
    t = t0 + bytes / B, separating the fixed cost of a launch from streaming."""
    import torch

    from paper_2103_08301_amd import Lattice, workloads

    w = workloads.plug_large_stable(storage)
    bpn = BYTES_PER_NODE[storage]
    rows = []
    for nx, ny in [(64, 16), (256, 64), (1024, 128), (2048, 256), (2048, 512), (4096, 256), (4096, 512),
                   (4096, 640), (3072, 1024)]:
        lat = Lattice(nx, ny, w["tau"], storage=storage, check_every=100000, **w["params"])
        lat.init_plug(max(8, nx // 14), max(1, ny // 32), float("nan"), 1e-3, 2)
        n = 2000 if nx * ny < 1e6 else 500
        lat.step(50)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(n)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / n
        rows.append((nx * ny * bpn, t))
        print(json.dumps({"nx": nx, "ny": ny, "bytes_per_step": nx * ny * bpn, "us_per_step": round(t * 1e6, 3),
                          "MLUPS": round(nx * ny / t / 1e6, 1)}), flush=True)
        del lat
    big = [(b, t) for b, t in rows if b >= 3e7]
    if len(big) >= 2:
        import numpy as np

        b, t = np.array(big, dtype=float).T
        slope, t0 = np.polyfit(b, t, 1)
        print(json.dumps({"fit_over_bytes_ge_30MB": {"fixed_us": round(t0 * 1e6, 2),
                                                    "stream_GBps": round(1 / slope / 1e9, 1)}}), flush=True)
    return 0


def tangent_cost(steps: int, warmup: int) -> int:
    """Per-step time of the tangent-linear step (FP64 value + FP64 tangent per
    population, one parameter direction) against the FP64 step, 4096x512."""
    from paper_2103_08301_amd import workloads

    out = {"metric": "tangent-linear step cost, 4096x512", "steps": steps}
    for storage in ("f64", "f64t"):
        w = workloads.plug_large_stable("f64")
        w["storage"] = storage
        lat = make_lattice(w, check_every=max(steps, warmup, 1))
        if storage == "f64t":
            lat.set_tangent(dp=1.0)
        t, _, lat = _time_lattice(lat, steps, warmup)
        nodes = w["nx"] * w["ny"]
        out[storage] = {"us_per_step": round(t / steps * 1e6, 2), "MLUPS": round(nodes * steps / t / 1e6, 1),
                        "GBps_algorithmic": round((144 if storage == "f64" else 288) * nodes / (t / steps) / 1e9, 1)}
        if storage == "f64t":
            out["d_int_tau2"] = lat.history(1)[-1]["d_int_tau2"]
        del lat
    out["ratio_tangent_over_f64"] = round(out["f64t"]["us_per_step"] / out["f64"]["us_per_step"], 3)
    out["gradient_4_params_over_f64"] = round(4 * out["ratio_tangent_over_f64"], 2)
    print(json.dumps(finite(out)), flush=True)
    return 0


def adjoint_measure(storage: str, steps: int, segment: int, large: bool) -> dict:
    """Time of one gradient of J = int sum tau_w^2 (recorded forward run with checkpoints + one reverse sweep)
    against a plain forward run of the same steps, on the 1024x256 adjoint workload (or 4096x512)."""
    import torch

    from paper_2103_08301_amd import workloads

    w = workloads.plug_large_stable(storage) if large else workloads.plug_adjoint(storage)
    nodes = w["nx"] * w["ny"]
    # warm-up on throwaway lattices: the first launch of each kernel in a process loads its code (~10 ms),
    # which would otherwise land in whichever timed run comes first
    warm = make_lattice(w, check_every=200)
    warm.step(200)
    del warm
    warm = make_lattice(w, check_every=50)
    warm.adjoint_bind(50, 0)
    warm.adjoint_forward()
    warm.adjoint_backward()
    torch.cuda.synchronize()
    del warm
    fwd = make_lattice(w, check_every=steps)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record(fwd.stream)
    st = fwd.step(steps)
    e[1].record(fwd.stream)
    torch.cuda.synchronize()
    t_fwd = e[0].elapsed_time(e[1]) / 1e3
    J_fwd = fwd.history(1)[-1]["int_tau2"]
    del fwd
    lat = make_lattice(w, check_every=steps)
    lat.adjoint_bind(steps, segment)
    torch.cuda.synchronize()
    e[0].record(lat.stream)
    st2, J = lat.adjoint_forward()
    e[1].record(lat.stream)
    grad = lat.adjoint_backward()
    e[2].record(lat.stream)
    torch.cuda.synchronize()
    t_rec, t_bwd = e[0].elapsed_time(e[1]) / 1e3, e[1].elapsed_time(e[2]) / 1e3
    seg = segment or math.ceil(math.sqrt(steps))
    recompute_steps = steps  # every step is recomputed once from its segment's checkpoint
    t_adj_kernel = max(t_bwd - recompute_steps * t_fwd / steps, 0.0) / steps
    bpn = 23 * (4 if storage == "f32" else 8)  # 5 forward fields and 9 adjoint reads, 9 adjoint writes
    del lat
    return {"metric": "adjoint/fwd time (gradient of int sum tau_w^2 w.r.t. dp, a, b, T)", "workload": w["name"],
            "storage": storage, "steps": steps, "segment": seg, "checkpoints": math.ceil(steps / seg),
            "forward_s": round(t_fwd, 4), "record_s": round(t_rec, 4), "backward_s": round(t_bwd, 4),
            "adjoint_over_forward": round((t_rec + t_bwd) / t_fwd, 3),
            "forward_us_per_step": round(t_fwd / steps * 1e6, 2),
            "adjoint_kernel_us_per_step_est": round(t_adj_kernel * 1e6, 2),
            "adjoint_kernel_GBps_est": round(bpn * nodes / t_adj_kernel / 1e9, 1) if t_adj_kernel > 0 else None,
            "adjoint_bytes_per_node": bpn,
            "status": [st, st2], "J": J, "J_plain_forward": J_fwd,
            "dJ_ddp": grad[0], "dJ_da": grad[1], "dJ_db": grad[2], "dJ_dT": grad[3]}


def adjoint_cost(storage: str, steps: int, segment: int, large: bool) -> int:
    print(json.dumps(finite(adjoint_measure(storage, steps, segment, large))), flush=True)
    return 0


def _time_lattice(lat, steps: int, warmup: int):
    import torch

    if warmup:
        lat.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, None, lat


def batch_sweep(storage: str, steps: int, warmup: int) -> int:
    """Aggregate throughput of the 48 sweep cases drawn from seed 4 (workloads.c4_cases: nx 1024-4096,
    ny 128-512, dp, plug and film drawn per case; 42.3 M nodes) advanced as one batch (one launch for all cases
    per step or per two steps, as the autotuner picks; graphs captured beforehand) against the same cases
    stepped one after another (each case autotuned on its own), with each case's stability check after the
    timed steps.  The roofline fractions count the HBM bytes the chosen launches move per node and step (72 B
    in FP32 for one step per launch, 36 B for two)."""
    import numpy as np
    import torch

    from paper_2103_08301_amd import Batch, Lattice, workloads

    cases = workloads.c4_cases()
    nodes = sum(c["nx"] * c["ny"] for c in cases)
    init = ("plug", "film", "noise_amp", "seed")
    spec = [{k: v for k, v in c.items() if k not in init} for c in cases]
    batch = Batch(spec, storage=storage, check_every=CHECK_EVERY, v_limit=0.5, graph_steps=GRAPH_STEPS)
    for k, c in enumerate(cases):
        batch[k].init_plug(c["plug"], c["film"], float("nan"), c["noise_amp"], c["seed"])
    batch.step(warmup)
    tuned = batch.autotune(20)
    batch.capture(steps)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(batch.stream)
    batch.step(steps)
    e1.record(batch.stream)
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) / 1e3
    checks = [batch[k].check() for k in range(len(cases))]
    lats = []
    for k, (c, s) in enumerate(zip(cases, spec)):
        s = dict(s)
        lat = Lattice(s.pop("nx"), s.pop("ny"), s.pop("tau"), storage=storage, check_every=CHECK_EVERY,
                      v_limit=0.5, graph_steps=GRAPH_STEPS, **s)
        lat.init_plug(c["plug"], c["film"], float("nan"), c["noise_amp"], c["seed"])
        lat.step(warmup)
        lat.autotune(20)
        lat.capture(steps)
        lats.append(lat)
    torch.cuda.synchronize()
    e0.record(lats[0].stream)
    for lat in lats:
        lat.step(steps)
    e1.record(lats[0].stream)
    torch.cuda.synchronize()
    t_seq = e0.elapsed_time(e1) / 1e3
    same = all(np.array_equal(batch[k].fields()[0], lats[k].fields()[0]) for k in range(len(cases)))
    L = batch[0].launch_config()["fused_steps"]
    bpn = BYTES_PER_NODE[storage] // L
    seq_launch = [lat.launch_config()["fused_steps"] for lat in lats]
    # bytes moved by the sequential runs: each case at its own launch's rate
    seq_bytes = sum(BYTES_PER_NODE[storage] // f * c["nx"] * c["ny"] for f, c in zip(seq_launch, cases))
    out = {"metric": "aggregate MLUPS, 48 sweep cases drawn from seed 4", "unit": "MLUPS", "storage": storage,
           "cases": len(cases), "nodes": nodes, "steps": steps, "warmup": warmup,
           "batch": {"MLUPS": round(nodes * steps / t_batch / 1e6, 1), "us_per_step": round(t_batch / steps * 1e6, 2),
                     "steps_per_launch": L, "hbm_bytes_per_node_step": bpn,
                     "roofline_frac": round(bpn * nodes / (t_batch / steps) / 1e9 / HBM_PEAK_GBS, 4)},
           "sequential": {"MLUPS": round(nodes * steps / t_seq / 1e6, 1), "us_per_step": round(t_seq / steps * 1e6, 2),
                          "cases_with_two_steps_per_launch": sum(f == 2 for f in seq_launch),
                          "roofline_frac": round(seq_bytes / (t_seq / steps) / 1e9 / HBM_PEAK_GBS, 4)},
           "speedup": round(t_seq / t_batch, 3), "batch_equals_sequential": bool(same), "batch_tiles": tuned,
           "graph_steps": GRAPH_STEPS,
           "unstable_cases": [[k, ch["unstable_step"]] for k, ch in enumerate(checks) if ch["unstable_step"] >= 0],
           "ruptured_cases": [[k, ch["rupture_step"]] for k, ch in enumerate(checks) if ch["rupture_step"] >= 0],
           "max_vmax": max(ch["vmax"] for ch in checks)}
    print(json.dumps(finite(out)), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--storage", default="f32", choices=sorted(BYTES_PER_NODE))
    ap.add_argument("--workload", default="large-stable", choices=["large-stable", "large", "out-of-cache"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the FP16-storage run and the literal-config probe")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes 10 times (counter calibration)")
    ap.add_argument("--size-sweep", action="store_true",
                    help="only time the step on grids from 64x16 to 3072x1024 (fixed per-launch cost vs bytes)")
    ap.add_argument("--tangent", action="store_true",
                    help="only time the tangent-linear (F64T) step against the FP64 step on the timed workload")
    ap.add_argument("--adjoint", action="store_true",
                    help="only time one reverse-mode gradient against a forward run (1024x256, 20k steps)")
    ap.add_argument("--adjoint-large", action="store_true",
                    help="with --adjoint: the 4096x512 workload instead (--steps steps)")
    ap.add_argument("--segment", type=int, default=0, help="with --adjoint: checkpoint spacing (0: sqrt(steps))")
    ap.add_argument("--autotune", action="store_true",
                    help="time every tile shape after the warm-up and keep the fastest (the 4096x512 FP32 default "
                         "shape, 60x8 with 4 waves, is within 2%% of the best; --batch always tunes)")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="steps per captured HIP graph of the step loop (0: library default, -1: direct launches)")
    ap.add_argument("--batch", action="store_true",
                    help="only time 48 uneven sweep cases as one batch against the same cases stepped one by one")
    args = ap.parse_args()
    global GRAPH_STEPS, AUTOTUNE
    GRAPH_STEPS = args.graph_steps
    AUTOTUNE = args.autotune

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
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
        dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        gbs = 2 * n * 4 * 10 / (e0.elapsed_time(e1) / 1e3) / 1e9
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 10, "copy_GBps_read_plus_write": round(gbs, 1)}),
              flush=True)
        return 0
    lbm.library()  # fail loudly if the HIP library is missing
    if args.size_sweep:
        return size_sweep(args.storage)
    if args.tangent:
        return tangent_cost(steps=min(args.steps, 2000), warmup=min(args.warmup, 100))
    if args.adjoint:
        return adjoint_cost(args.storage, steps=args.steps, segment=args.segment, large=args.adjoint_large)
    if args.batch:
        return batch_sweep(args.storage, steps=min(args.steps, 2000), warmup=min(args.warmup, 100))

    if args.graph_steps == 0 and args.warmup > 256:
        # 256-step graphs: 0.3% faster per step than the library's default of 64 on 4096x512.  A warm-up of more
        # than 256 steps captures the graph the timed steps replay (an even step count keeps its parity); short
        # runs, such as the batch timing's, would pay the capture inside the timed steps
        GRAPH_STEPS = 256
    make = {"large-stable": workloads.plug_large_stable, "large": workloads.plug_large,
            "out-of-cache": workloads.plug_out_of_cache}[args.workload]
    w = make(args.storage)
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
    traffic = measured_traffic(args.storage, (lat.tuned["tile_rows"], lat.tuned["tile_waves"]) if lat.tuned else (8, 4))
    hist = lat.history(1)
    peak = None
    if hist:
        h = hist[-1]
        peak = max(abs(h["tau_max"][0]), abs(h["tau_min"][0]), abs(h["tau_max"][1]), abs(h["tau_min"][1]))
    out = {
        "metric": METRIC if args.workload == "large-stable" else f"MLUPS, D2Q9 {w['nx']}x{w['ny']} ({args.workload})",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic",
        "config": {"workload": w["name"], "nx": w["nx"], "ny": w["ny"], "tau": w["tau"], **w["params"],
                   **{k: v for k, v in w["plug"].items() if k != "x_center"}, "storage": args.storage,
                   "schedule": (f"tile 60x{lat.tuned['tile_rows']}, {lat.tuned['tile_waves']} waves (autotuned)"
                                if lat.tuned else ("tile 60x8" if args.storage not in ("f64", "f32d") else "tile 60x12")),
                   "graph_steps": GRAPH_STEPS, "check_every": CHECK_EVERY},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_node": bpn,
                     "fabric_bytes_per_node": round(traffic / nodes, 2) if traffic else None,
                     "fabric_GBps": round(traffic / (gpu_s / args.steps) / 1e9, 1) if traffic else None,
                     "kernel": "tile_kernel (fused pull-stream/force/MRT/wall diagnostics)"},
        "physics": {"unstable_step": chk["unstable_step"], "vmax": round(chk["vmax"], 5),
                    "nan_cells": chk["nan_count"], "liquid_columns": chk["liquid_columns"],
                    "x_rear": chk["x_rear"], "x_front": chk["x_front"], "wall_tau_peak_last_step": peak},
    }
    if not args.no_variants and args.workload == "large-stable":
        for key, st in (("fp16_store", "f16s"), ("fp16_store_stochastic", "f16r")):
            wh = make(st)
            hs, _, hl = time_steps(wh, args.steps, args.warmup)
            hc = hl.check()
            out[key] = {"value": round(nodes * args.steps / hs / 1e6, 1), "unit": "MLUPS",
                        "roofline_frac": round(36 * nodes / (hs / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
                        "x_rear": hc["x_rear"], "x_front": hc["x_front"], "liquid_columns": hc["liquid_columns"],
                        "unstable_step": hc["unstable_step"]}
            log(f"{key}: {out[key]}")
            del wh, hl
        # the same physics on 16384x2048: 2 x 1.2 GB of FP32 distributions, beyond the 256 MB Infinity Cache,
        # with the default one-step launch (its HBM roofline) and with the launch the library's autotuner picks
        # (two steps per launch there: half the HBM bytes per step)
        wo = workloads.plug_out_of_cache(args.storage)
        no = wo["nx"] * wo["ny"]
        os_, _, ol = time_steps(wo, args.steps, args.warmup)
        oc = ol.check()
        del ol
        ts_, _, tl = time_steps(wo, args.steps, args.warmup, tune=True)
        lc = tl.launch_config()
        tc = tl.check()
        del tl
        moved = bpn // lc["fused_steps"]  # HBM bytes per node and step of the chosen launch
        out["out_of_cache"] = {
            "workload": wo["name"], "value": round(no * args.steps / ts_ / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(ts_ * 1e3 / args.steps, 4),
            "launch": {"tile_rows": lc["tile_rows"], "tile_waves": lc["tile_waves"],
                       "steps_per_launch": lc["fused_steps"], "autotuned": True},
            "hbm_bytes_per_node_step": moved,
            "roofline_frac": round(moved * no / (ts_ / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
            "unstable_step": tc["unstable_step"],
            "one_step_launch": {"value": round(no * args.steps / os_ / 1e6, 1),
                                "ms_per_step": round(os_ * 1e3 / args.steps, 4), "hbm_bytes_per_node_step": bpn,
                                "roofline_frac": round(bpn * no / (os_ / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
                                "unstable_step": oc["unstable_step"]}}
        log(f"out_of_cache: {out['out_of_cache']}")
        # the gradient's cost: one reverse-mode gradient of int tau_w^2 over the 1024x256, 20000-step run
        # against a plain forward run of the same steps
        adj = adjoint_measure("f32", 20000, 0, False)
        out["adjoint"] = {k: adj[k] for k in ("workload", "steps", "checkpoints", "forward_s", "record_s",
                                              "backward_s", "adjoint_over_forward", "dJ_ddp", "dJ_da", "dJ_db",
                                              "dJ_dT")}
        log(f"adjoint: {out['adjoint']}")
        lit = workloads.plug_large(args.storage)
        ll = make_lattice(lit, check_every=50)
        ll.step(400)
        out["config_as_specified"] = {"workload": lit["name"], "unstable_step": ll.check()["unstable_step"],
                                      "note": "diverges under the method as read; not timed (NaN data runs at a "
                                              "different rate)"}
        log(f"literal config: {out['config_as_specified']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(finite(out), allow_nan=False), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
