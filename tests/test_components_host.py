"""The library's host labelling of liquid components (lbm_components_field,
union-find) against the oracle's flood fill on the same fields.  Host code
only: runs without a GPU."""
import numpy as np
import pytest

import oracle as O
from paper_2103_08301_amd import lbm

KEYS_EXACT = ("first_cell", "cells", "wall")
KEYS_FLOAT = ("mass", "excess_mass", "cx", "cy")


def same(a, b):
    assert len(a) == len(b)
    for ca, cb in zip(a, b):
        for k in KEYS_EXACT:
            assert ca[k] == cb[k], k
        for k in KEYS_FLOAT:
            assert ca[k] == pytest.approx(cb[k], rel=1e-12, abs=1e-12), k


def blobs(rng, ny, nx, n):
    """Smooth random liquid blobs over a gas background, touching edges and seams."""
    rho = np.full((ny, nx), 0.05)
    yy, xx = np.mgrid[0:ny, 0:nx]
    for _ in range(n):
        cx, cy, r = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(1.0, 7.0)
        dx = np.minimum(np.abs(xx - cx), nx - np.abs(xx - cx))
        rho = np.maximum(rho, 0.05 + 0.25 / (1 + np.exp(((dx ** 2 + (yy - cy) ** 2) ** 0.5 - r) * 2.0)))
    return rho


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("xper,yper", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("seed", [11, 12])
def test_library_matches_oracle(conn, xper, yper, seed):
    rng = np.random.default_rng(seed)
    rho = blobs(rng, 41, 67, 25)
    thr, rg = 0.17, 0.05
    ref = O.components_field(rho, thr, rg, conn, x_periodic=xper, y_periodic=yper)
    got, summ = lbm.lbm_components_field(rho, thr, rg, conn, x_periodic=xper, y_periodic=yper)
    same(got, ref)
    assert summ["components"] == len(ref)
    aer = [c for c in ref if c["wall"] == 0]
    assert summ["aerosols"] == len(aer)
    assert summ["aerosol_cells"] == sum(c["cells"] for c in aer)
    assert summ["aerosol_mass"] == pytest.approx(sum(c["mass"] for c in aer), rel=1e-12, abs=1e-12)
    assert summ["liquid_mass"] == pytest.approx(rho[rho > thr].sum(), rel=1e-12)


def test_random_noise_fields_match_oracle():
    rng = np.random.default_rng(5)
    for conn in (4, 8):
        rho = rng.uniform(0, 1, size=(29, 31))
        same(lbm.lbm_components_field(rho, 0.55, 0.0, conn, 1, 1)[0],
             O.components_field(rho, 0.55, 0.0, conn, x_periodic=1, y_periodic=1))


def test_limits_and_errors():
    rho = np.full((6, 9), 0.05)
    got, summ = lbm.lbm_components_field(rho, 0.1)
    assert got == [] and summ["components"] == 0 and summ["liquid_mass"] == 0.0
    rho[:] = 0.3
    got, summ = lbm.lbm_components_field(rho, 0.1, 0.05, 8, 1, 1)
    assert len(got) == 1 and got[0]["cells"] == 54 and got[0]["wall"] == 0
    with pytest.raises(lbm.LbmError):
        lbm.lbm_components_field(rho, 0.1, 0.05, 5)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_components_field(rho, float("nan"), 0.05, 4)


def test_wall_shear_objective_requires_a_fixed_wall_density():
    """The adjoint holds rho_wall fixed; a spec that leaves it to follow rho_l(theta) is refused before any
    device work (so this runs without a GPU)."""
    import math

    import pytest
    import torch

    from paper_2103_08301_amd.lbm import WallShearObjective

    theta = torch.tensor([1e-3, 1.0, 4.0, 0.08], dtype=torch.float64, requires_grad=True)
    base = dict(nx=32, ny=16, tau=1.0, nsteps=10, rho_init=None)
    for params in ({}, {"rho_wall": None}, {"rho_wall": math.nan}):
        with pytest.raises(ValueError, match="rho_wall"):
            WallShearObjective.apply(theta, dict(base, params=params))
