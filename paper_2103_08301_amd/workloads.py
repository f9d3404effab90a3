"""Seeded synthetic workloads shaped like the paper's airway-reopening runs.

The paper (Sec. 2.3, 3.1-3.3) runs a liquid plug spanning a 2-D channel with a
liquid film on both walls, driven by a pressure drop; it publishes no dataset,
so every input here is synthetic.  This module only holds the recipes (sizes,
physical parameters, seeds) and the seeded draws that pick a parameter; it
contains none of the method's arithmetic, and both the GPU library and the CPU
oracle take its values as inputs.
"""
from __future__ import annotations

import math

_GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(seed: int, n: int) -> int:
    """n-th output (0-based) of SplitMix64 seeded with `seed` (Steele, Lea & Flood 2014)."""
    z = (seed + (n + 1) * _GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def uniform(seed: int, n: int) -> float:
    return (splitmix64(seed, n) >> 11) * 2.0**-53


# Plug-in-channel workloads.  "noise" is the amplitude of the additive uniform
# density noise of the initial condition; x_center NaN puts the rear interface at nx/4.
PLUG_SMALL = dict(
    name="plug-channel 256x64 FP64 (CS 0.85 Tc, tau 1.0, plug 40 at x=80, film 4, dp 1e-3, 2000 steps)",
    nx=256, ny=64, tau=1.0, storage="f64", steps=2000,
    params=dict(T_over_Tc=0.85, dp=1e-3),
    plug=dict(plug_len=40, film=4, x_center=80.0, noise_amp=1e-3, seed=1),
)


def plug_large(storage: str = "f32") -> dict:
    """4096x512 channel, CS at 0.80 Tc, tau 0.8, plug 300, film 16, dp drawn from seed 2 in [5e-4, 3e-3]."""
    dp = 5e-4 + 2.5e-3 * uniform(2, 0)
    return dict(
        name=f"plug-channel 4096x512 {storage.upper()} (CS 0.80 Tc, tau 0.8, plug 300, film 16, dp {dp:.6g})",
        nx=4096, ny=512, tau=0.8, storage=storage, steps=100_000,
        params=dict(T_over_Tc=0.80, dp=dp),
        plug=dict(plug_len=300, film=16, x_center=math.nan, noise_amp=1e-3, seed=2),
    )


def plug_large_stable(storage: str = "f32") -> dict:
    """Same grid, tau, plug, film and pressure drop as plug_large, at 0.95 Tc.

    Under the method as implemented, the 0.80 Tc case diverges within ~50 steps
    and 0.85-0.90 Tc within 12-25k steps (the driven gas of a 512-row channel
    accelerates past the lattice's low-Mach range); 0.95 Tc with tau 0.8 stays
    finite beyond 30k steps, so timed runs use it."""
    w = plug_large(storage)
    w["name"] = w["name"].replace("CS 0.80 Tc", "CS 0.95 Tc")
    w["params"] = dict(w["params"], T_over_Tc=0.95)
    return w


def plug_out_of_cache(storage: str = "f32") -> dict:
    """16384x2048 control whose distributions (2 x 1.2 GB in FP32) exceed the 256 MB Infinity Cache: the
    4096x512 workload scaled by 4 in both directions (plug 1200, films 64 rows), with the pressure drop
    scaled with the length so that the body force density dp/nx is the same."""
    w = plug_large_stable(storage)
    dp = 4 * w["params"]["dp"]
    w.update(nx=16384, ny=2048,
             name=f"plug-channel 16384x2048 {storage.upper()} (CS 0.95 Tc, tau 0.8, plug 1200, film 64, dp {dp:.6g})")
    w["params"] = dict(w["params"], dp=dp)
    w["plug"] = dict(w["plug"], plug_len=1200, film=64)
    return w


def plug_adjoint(storage: str = "f32") -> dict:
    """1024x256 plug case for the wall-shear gradient: plug 120, film 8, 20k steps.

    At 0.85 Tc this channel diverges within 5-16k steps for every pressure
    drop from 1e-3 down to 1e-4 (tau 1), so the gradient runs use 0.95 Tc,
    tau 1 and dp 5e-4, which stay finite through the rupture (~11k steps)."""
    return dict(
        name=f"plug-channel 1024x256 {storage.upper()} (CS 0.95 Tc, tau 1.0, plug 120, film 8, dp 5e-4)",
        nx=1024, ny=256, tau=1.0, storage=storage, steps=20_000,
        params=dict(T_over_Tc=0.95, dp=5e-4),
        plug=dict(plug_len=120, film=8, x_center=math.nan, noise_amp=1e-3, seed=5),
    )


def c4_cases(n: int = 48, seed: int = 4) -> list:
    """The sweep of Sec. 3.3 (Figs 10-12: pressure drop, plug and film thickness varied) as n independent
    channels drawn from SplitMix64(seed): per case, in this order, nx uniform in [1024, 4096], ny uniform in
    [128, 512] (integers), dp uniform in [5e-4, 3e-3], plug length / ny uniform in [0.3, 1.2] and film
    thickness / ny uniform in [0.01, 0.08] (plug rounded to whole cells, films to whole rows, at least one).
    The state point is the 4096x512 workload's (CS 0.95 Tc, tau 0.8; the plug's rear interface at nx/4) and
    the initial noise 1e-3 with seed `seed`."""
    cases = []
    for k in range(n):
        u = [uniform(seed, 5 * k + j) for j in range(5)]
        nx = 1024 + int(u[0] * 3073)
        ny = 128 + int(u[1] * 385)
        cases.append(dict(nx=nx, ny=ny, tau=0.8, T_over_Tc=0.95, dp=5e-4 + 2.5e-3 * u[2],
                          plug=float(round((0.3 + 0.9 * u[3]) * ny)),
                          film=float(max(1, round((0.01 + 0.07 * u[4]) * ny))), noise_amp=1e-3, seed=seed))
    return cases
