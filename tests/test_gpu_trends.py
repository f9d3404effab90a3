"""Verification sweeps of the aerosol trends of Sec. 3.3 (Figs 10-12), at reduced size.

The paper reports that the aerosol (detached droplet) mass rises with the
pressure drop (Fig 10) and with the plug thickness b (Fig 11, about linearly),
and falls with the liquid-film thickness h (Fig 12, about linearly).  Its
physical units cannot be mapped to lattice units, so these are trend checks,
not value checks (parity unpinned): a 512x128 channel of radius R = 64 with
periodic ends, CS 0.90 Tc, tau 1, FP32, plug and film in units of R, and the
pressure drop as a body force dp/nx.  Each case runs until 3000 steps after the
first droplet detaches; its aerosol mass is the largest total mass of
detached liquid components seen every 250 steps.
"""
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2103_08301_amd import Lattice  # noqa: E402

NX, NY, T, TAU = 512, 128, 0.90, 1.0
R = NY / 2


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def aerosol_mass(dp, b, h, max_steps=30000, every=250):
    lat = Lattice(NX, NY, TAU, storage="f32", check_every=1000, x_periodic=1, v_limit=0.5, T_over_Tc=T, dp=dp,
                  history_cap=1)
    lat.init_plug(b * R, h * R, float("nan"), 1e-3, 1)
    first, best = None, 0.0
    while lat.steps < max_steps:
        assert lat.step(every) == 0
        _, s = lat.components()
        if s["aerosols"] and first is None:
            first = lat.steps
        best = max(best, s["aerosol_mass"])
        if first is not None and lat.steps >= first + 3000:
            break
    log(f"dp {dp:.1e} b {b}R h {h}R: first droplet at step {first}, aerosol mass {best:.2f}")
    assert first is not None, "no droplet detached"
    return best


def test_aerosol_mass_rises_with_pressure_drop():
    m = [aerosol_mass(dp, 1.0, 0.15) for dp in (2e-4, 4e-4, 6e-4)]
    assert m[0] < m[1] < m[2]


def test_aerosol_mass_rises_with_plug_thickness():
    m = [aerosol_mass(4e-4, b, 0.15) for b in (0.6, 1.0, 1.2)]
    assert m[0] < m[1] < m[2]


def test_aerosol_mass_falls_with_film_thickness():
    m = [aerosol_mass(4e-4, 1.0, h) for h in (0.1, 0.15, 0.2)]
    assert m[0] > m[1] > m[2]
