"""Builds liblbm.so (HIP, gfx950) in-tree with hipcc.

Each source is compiled to an object of its own, in parallel (the step kernels
of each storage type sit in a translation unit of their own), then linked."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblbm.so")
SOURCES = ["lbm_api.cpp", "lbm_post.cpp", "lbm_kernels.hip", "lbm_noalloc.hip", "lbm_adjoint.hip", "lbm_step_f64.hip",
           "lbm_step_f32.hip", "lbm_step_f16s.hip", "lbm_step_bf16s.hip", "lbm_step_f32d.hip", "lbm_step_f32s.hip",
           "lbm_step_f64t.hip", "lbm_step_f16r.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # fused multiply-adds only within one source expression: every kernel that
    # inlines the same step code rounds identically (single, batched, pipelined)
    "-ffp-contract=on",
    # packed FP32 VALU forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # tile tickets are drawn by one lane and must stay in flight: no wave-level
    # rewrite of the atomic (which would wait for it at once to broadcast it)
    "-Xarch_device", "-mllvm=-amdgpu-atomic-optimizer-strategy=None",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build liblbm.so)")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}): {' '.join(cmd[-3:])}\n{res.stderr[-8000:]}")
    return [l for l in res.stderr.splitlines() if l.strip() and "packed-fp32-ops" not in l
            and "is not a recognized feature" not in l and "warning: argument unused" not in l]


def build_library(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP source for gfx950 into paper_2103_08301_amd/liblbm.so."""
    cc = hipcc()
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 16)))
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[cc, *FLAGS, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
        if verbose:
            print(" ".join(cmds[0]), flush=True)
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            noise = [l for out in pool.map(_run, cmds) for l in out]
        tmp = LIB + ".tmp"
        noise += _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    if verbose and noise:
        print("\n".join(noise[-40:]))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
