"""Reduced-precision storage against the FP64 oracle (the storage codecs).

A plug in a 256x64 channel with periodic ends (CS 0.95 Tc, tau 0.8, plug 40 at
x = 80, film 4, noise 1e-3 seed 1, dp 1e-4) is run with each storage type
from the same density field as an FP64 oracle run and compared at fixed steps:
relative L-inf and L2 error of rho, the interface positions, the liquid-column
count, and the drift of the total mass.  This case stays stable beyond 100000
steps and, with periodic ends and bounce-back walls, conserves mass exactly in
exact arithmetic (the oracle's FP64 drift is ~5e-12 after 100000 steps), so the
drift measures what the storage rounding does to conservation.

Storage types: f32 (plain FP32), f32s (FP32 of f_i - w_i rho0), f16s and
bf16s (FP16/BF16 of f_i - w_i rho0, rho0 = rho_g), f16r (FP16 of f_i - w_i rho0
with stochastic rounding), all with FP32 arithmetic.

The default run stops at 5000 steps.  LBM_PRECISION_CAMPAIGN=1 extends it to
20000 and 100000 steps (about a minute of oracle time) and prints the table.
"""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_2103_08301_amd import Lattice  # noqa: E402

NX, NY, TAU = 256, 64, 0.8
KW = dict(T_over_Tc=0.95, dp=1e-4, x_periodic=1)
CAMPAIGN = os.environ.get("LBM_PRECISION_CAMPAIGN") == "1"
STEPS = [500, 2000, 5000] + ([20000, 100000] if CAMPAIGN else [])

# Upper bounds on rel L-inf(rho) and on |mass drift| per storage at each
# checkpoint: the measured values times about 3 (the runs are deterministic).
# Measured rel L-inf(rho) at 500 / 2000 / 5000 / 20000 / 100000 steps:
#   f32    3.7e-6  5.9e-6  7.2e-6  2.3e-5  3.6e-4   (mass drift <= 1.3e-6)
#   f32s   3.7e-6  6.4e-6  6.8e-6  2.7e-5  3.7e-4   (mass drift <= 1.4e-6)
#   f16s   1.2e-3  8.8e-3  7.4e-2  0.70    0.70     (drift -3.4e-4 at 5000, +9.7e-2 at 100000)
#   bf16s  8.5e-2  0.40    0.70    0.70    0.70     (drift -4.0e-3 at 500)
#   f16r   1.3e-3  2.5e-3  2.5e-2  0.11    0.42     (mass drift <= 2.3e-4)
# FP16 storage follows the trajectory for a few thousand steps and then drifts
# off it (its rounding acts as a mass source); BF16 storage does not follow it.
# FP16 with stochastic rounding (f16r) keeps the mass to 4e-5 over 20000 steps;
# its interfaces are 0.25 lattice units behind the oracle's at 5000 steps and
# 1.2 behind at 20000 (FP16 storage with round-to-nearest: 0.8 and 24 ahead).
BOUNDS = {
    "f32": {500: 1.2e-5, 2000: 2e-5, 5000: 3e-5, 20000: 6e-5, 100000: 1.2e-3},
    "f32s": {500: 1.2e-5, 2000: 2e-5, 5000: 3e-5, 20000: 1e-4, 100000: 1.2e-3},
    "f16s": {500: 4e-3, 2000: 3e-2, 5000: 0.25},
    "bf16s": {500: 0.3},
    "f16r": {500: 5e-3, 2000: 2e-2, 5000: 8e-2, 20000: 0.35},
}
# Upper bounds on the distance (lattice units) of the rear and front interfaces
# from the oracle's.  FP32 storage matches them to 1e-3.  For f16r the bound is
# the 0.5 lu interface criterion for reduced-precision storage; over six seeds
# of the initial noise the measured lag at 5000 steps was 0.17-0.28 lu.
INTERFACE_BOUNDS = {
    "f32": {500: 0.01, 2000: 0.01, 5000: 0.01, 20000: 0.01},
    "f32s": {500: 0.01, 2000: 0.01, 5000: 0.01, 20000: 0.01},
    "f16r": {500: 0.5, 2000: 0.5, 5000: 0.5},
}
MASS_BOUNDS = {
    "f32": {500: 3e-8, 2000: 3e-8, 5000: 3e-8, 20000: 1.5e-7, 100000: 4e-6},
    "f32s": {500: 3e-8, 2000: 3e-8, 5000: 3e-8, 20000: 1.5e-7, 100000: 4e-6},
    "f16s": {500: 4e-5, 2000: 5e-4, 5000: 1e-3},
    "bf16s": {500: 1.5e-2},
    # stochastic rounding is unbiased, but its errors still move the total mass as a random walk:
    # ~4600 liquid nodes with rounding noise of ~2.8e-5 each give ~1.2e-6 of the mass per step,
    # sigma ~2.6e-5, 5.2e-5, 8.2e-5 and 1.6e-4 after 500, 2000, 5000 and 20000 steps; the bounds
    # are about 3 sigma (one realisation measured +5.9e-5 at 2000 steps)
    "f16r": {500: 8e-5, 2000: 1.6e-4, 5000: 2.5e-4, 20000: 5e-4, 100000: 1.2e-3},
}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def reference():
    """Oracle snapshots (rho, interface, mass) at each checkpoint, and the initial density."""
    ref = O.Sim(NX, NY, O.params(tau=TAU, v_limit=1.0, check_every=200000, **KW))
    ref.init_plug(40, 4, 80, 1e-3, 1)
    rho0 = ref.fields()[0].copy()
    snaps = {}
    done = 0
    for s in STEPS:
        ref.step(s - done)
        done = s
        rho = ref.fields()[0].copy()
        snaps[s] = (rho, ref.interface(), float(rho.sum()))
    return rho0, float(rho0.sum()), snaps


@pytest.mark.parametrize("storage", ["f32", "f32s", "f16s", "bf16s", "f16r"])
def test_storage_error_against_oracle(reference, storage):
    rho0, mass0, snaps = reference
    lat = Lattice(NX, NY, TAU, storage=storage, v_limit=1.0, check_every=200000, **KW)
    lat.init_density(rho0)
    done = 0
    for s in STEPS:
        assert lat.step(s - done) == 0
        done = s
        rg = lat.fields()[0]
        rr, (xr, xf, cols), mass_ref = snaps[s]
        d = rg - rr
        e_inf = float(np.abs(d).max() / np.abs(rr).max())
        e_l2 = float(np.sqrt((d * d).sum() / (rr * rr).sum()))
        chk = lat.check()
        drift = (float(rg.sum()) - mass0) / mass0
        drift_ref = (mass_ref - mass0) / mass0
        log(f"{storage:6s} step {s:6d}: rel Linf rho {e_inf:.3e}  rel L2 {e_l2:.3e}  "
            f"rear {chk['x_rear']:.3f}/{xr:.3f}  front {chk['x_front']:.3f}/{xf:.3f}  "
            f"liquid cols {chk['liquid_columns']}/{cols}  mass drift {drift:+.3e} (oracle {drift_ref:+.3e})")
        assert math.isfinite(e_inf)
        if s in BOUNDS[storage]:
            assert e_inf <= BOUNDS[storage][s], (storage, s, e_inf)
        if s in INTERFACE_BOUNDS.get(storage, {}):
            lim = INTERFACE_BOUNDS[storage][s]
            assert abs(chk["x_rear"] - xr) <= lim and abs(chk["x_front"] - xf) <= lim, (storage, s, chk, xr, xf)
        if s in MASS_BOUNDS[storage]:
            assert abs(drift) <= MASS_BOUNDS[storage][s], (storage, s, drift)


@pytest.mark.parametrize("seed", [2, 4, 5])
def test_f16r_interfaces_within_half_a_lattice_unit_over_noise_seeds(seed):
    """The 0.5 lu interface bound of F16R storage at 5000 steps for other seeds of the initial noise
    (measured lags 0.24, 0.24 and 0.18 lu behind the oracle)."""
    ref = O.Sim(NX, NY, O.params(tau=TAU, v_limit=1.0, check_every=200000, **KW))
    ref.init_plug(40, 4, 80, 1e-3, seed)
    rho0 = ref.fields()[0].copy()
    ref.step(5000)
    xr, xf, cols = ref.interface()
    lat = Lattice(NX, NY, TAU, storage="f16r", v_limit=1.0, check_every=200000, **KW)
    lat.init_density(rho0)
    assert lat.step(5000) == 0
    chk = lat.check()
    log(f"f16r seed {seed} step 5000: rear {chk['x_rear']:.3f}/{xr:.3f}  front {chk['x_front']:.3f}/{xf:.3f}  "
        f"liquid cols {chk['liquid_columns']}/{cols}")
    assert abs(chk["x_rear"] - xr) <= 0.5 and abs(chk["x_front"] - xf) <= 0.5, (seed, chk, xr, xf)
