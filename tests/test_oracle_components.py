"""Pins of the oracle's liquid-component labelling (aerosol detection, Sec. 3.2-3.3).

Each check uses something independent of the oracle's flood fill: scipy's
ndimage.label (a library labelling routine) on random fields, brute-force
counts and symmetry of digitised disks, hand-built seams and diagonal
contacts, and additivity of mass.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle as O

STRUCT = {4: ndimage.generate_binary_structure(2, 1), 8: ndimage.generate_binary_structure(2, 2)}


def field(ny, nx, bg=0.05):
    return np.full((ny, nx), bg)


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_fields_match_scipy_label(conn, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.0, 1.0, size=(37, 53))
    thr = 0.62
    comps = O.components_field(rho, thr, 0.0, conn)
    lab, n = ndimage.label(rho > thr, structure=STRUCT[conn])
    assert len(comps) == n
    # scipy labels in raster order of first cell, as the oracle orders its output
    for k, c in enumerate(comps, start=1):
        cells = np.flatnonzero((lab == k).ravel())
        assert c["first_cell"] == cells[0]
        assert c["cells"] == cells.size
        assert c["mass"] == pytest.approx(rho.ravel()[cells].sum(), rel=1e-13)
        ys, xs = np.divmod(cells, rho.shape[1])
        assert c["cx"] == pytest.approx(xs.mean(), rel=1e-13)
        assert c["cy"] == pytest.approx(ys.mean(), rel=1e-13)
        assert c["wall"] == int(ys.min() == 0 or ys.max() == rho.shape[0] - 1)


def test_disk_count_and_centroid():
    ny, nx, cx, cy, r = 64, 96, 40.0, 30.0, 9.5
    rho = field(ny, nx)
    yy, xx = np.mgrid[0:ny, 0:nx]
    inside = (xx - cx) ** 2 + (yy - cy) ** 2 < r * r
    rho[inside] = 0.3
    (c,) = O.components_field(rho, 0.15, 0.05, 4)
    assert c["cells"] == int(inside.sum())  # brute-force count of lattice points in the disk
    assert c["wall"] == 0
    assert c["cx"] == pytest.approx(cx, abs=1e-12) and c["cy"] == pytest.approx(cy, abs=1e-12)  # symmetry
    assert c["mass"] == pytest.approx(0.3 * inside.sum(), rel=1e-13)
    assert c["excess_mass"] == pytest.approx(0.25 * inside.sum(), rel=1e-13)


def test_film_touches_wall_droplet_does_not():
    rho = field(40, 80)
    rho[0:4, :] = 0.3        # bottom film
    rho[36:40, 10:70] = 0.3  # top film
    rho[18:22, 30:36] = 0.3  # droplet
    comps = O.components_field(rho, 0.15, 0.05, 4)
    assert [c["wall"] for c in comps] == [1, 0, 1]
    assert [c["cells"] for c in comps] == [4 * 80, 4 * 6, 4 * 60]
    # with periodic y there are no walls
    assert all(c["wall"] == 0 for c in O.components_field(rho, 0.15, 0.05, 4, y_periodic=1))


def test_periodic_seam_joins_and_centres():
    nx, ny = 50, 20
    rho = field(ny, nx)
    rho[8:12, 0:3] = 0.3       # columns 0..2
    rho[8:12, nx - 2:nx] = 0.3  # columns 48, 49
    assert len(O.components_field(rho, 0.15, 0.05, 4, x_periodic=0)) == 2
    (c,) = O.components_field(rho, 0.15, 0.05, 4, x_periodic=1)
    assert c["cells"] == 20
    # columns 48, 49, 0, 1, 2 -> images -2, -1, 0, 1, 2 about column 0: mean 0
    assert c["cx"] == pytest.approx(0.0, abs=1e-12)
    rho2 = field(ny, nx)
    rho2[8:12, nx - 3:nx] = 0.3
    rho2[8:12, 0:1] = 0.3      # columns 47, 48, 49, 0 -> mean 48.5
    (c2,) = O.components_field(rho2, 0.15, 0.05, 4, x_periodic=1)
    assert c2["cx"] == pytest.approx(48.5, abs=1e-12)


def test_diagonal_contact_depends_on_connectivity():
    rho = field(10, 10)
    rho[4, 4] = rho[5, 5] = 0.3
    assert len(O.components_field(rho, 0.15, 0.05, 4)) == 2
    assert len(O.components_field(rho, 0.15, 0.05, 8)) == 1


def test_threshold_is_strict_and_mass_is_additive():
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.0, 1.0, size=(30, 30))
    rho[3, 3] = 0.5
    comps = O.components_field(rho, 0.5, 0.1, 8)
    assert sum(c["cells"] for c in comps) == int((rho > 0.5).sum())
    assert sum(c["mass"] for c in comps) == pytest.approx(rho[rho > 0.5].sum(), rel=1e-13)
    assert sum(c["excess_mass"] for c in comps) == pytest.approx((rho[rho > 0.5] - 0.1).sum(), rel=1e-13)


def test_invalid_arguments():
    rho = field(8, 8)
    with pytest.raises(ValueError):
        O.components_field(rho, 0.15, 0.05, 6)
    with pytest.raises(ValueError):
        O.components_field(rho, math.nan, 0.05, 4)


def test_sim_components_use_midpoint_threshold(orc):
    s = orc.Sim(120, 40, orc.params(T_over_Tc=0.85))
    s.init_plug(30, 3, 60.0, 0.0, 1)
    st = s.state()
    rg, rl = st["rho_g"], st["rho_l"]
    comps = s.components()
    ref = orc.components_field(s.fields()[0], 0.5 * (rg + rl), rg, 4)
    assert comps == ref
    # the plug and the two films form one liquid region attached to the walls
    assert len(comps) == 1 and comps[0]["wall"] == 1
