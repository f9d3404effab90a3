"""Liquid components through the device path (lbm_components on the density
the step kernel emits) against the oracle's labelling of its own field."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_2103_08301_amd import Lattice  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def same(a, b, rel=1e-12):
    assert len(a) == len(b)
    for ca, cb in zip(a, b):
        for k in ("first_cell", "cells", "wall"):
            assert ca[k] == cb[k], k
        for k in ("mass", "excess_mass", "cx", "cy"):
            assert ca[k] == pytest.approx(cb[k], rel=rel, abs=rel), k


@pytest.mark.parametrize("xper", [0, 1])
def test_synthetic_field(xper):
    nx, ny = 150, 48
    lat = Lattice(nx, ny, 1.0, storage="f64", x_periodic=xper)
    st = lat.state()
    rg, rl = st["rho_g"], st["rho_l"]
    rho = np.full((ny, nx), rg)
    rho[:3, :] = rl                      # films
    rho[ny - 3:, :] = rl
    rho[10:20, 40:52] = rl               # a droplet
    rho[25:30, nx - 4:] = rl             # a droplet across the seam (joined when periodic)
    rho[25:30, :3] = rl
    rho[20, 60] = rl                     # single cells touching diagonally
    rho[21, 61] = rl
    lat.init_density(rho)
    for conn in (4, 8):
        got, summ = lat.components(connectivity=conn)
        ref = O.components_field(rho, 0.5 * (rg + rl), rg, conn, x_periodic=xper)
        same(got, ref)
        assert summ["step"] == 0 and summ["components"] == len(ref)
        assert summ["aerosols"] == sum(1 for c in ref if c["wall"] == 0)
        log(f"x_periodic {xper} conn {conn}: {summ}")


def test_after_rupture_matches_oracle():
    """Periodic plug case that ruptures within 8000 steps (CS 0.95 Tc, tau 0.8,
    dp 5e-4, plug 40, film 4): after 9000 FP64 steps both sides label their own
    density fields identically."""
    nx, ny = 256, 64
    kw = dict(T_over_Tc=0.95, dp=5e-4, x_periodic=1, v_limit=1.0)
    lat = Lattice(nx, ny, 0.8, storage="f64", check_every=100000, **kw)
    ref = O.Sim(nx, ny, O.params(tau=0.8, check_every=100000, **kw))
    ref.init_plug(40, 4, 80, 1e-3, 1)
    lat.init_density(ref.fields()[0])
    assert lat.step(9000) == 0
    assert ref.step(9000) == 0
    got, summ = lat.components()
    exp = ref.components()
    log(f"after 9000 steps: {summ}")
    same(got, exp, rel=1e-9)
    assert lat.check()["liquid_columns"] == 0  # ruptured
