"""lbm_check_state_noalloc, the allocation-free variant of lbm_check_state, through the C ABI.

Each case builds two identical lattices, advances both to a step that is not a check step,
and asks one for lbm_check_state (which stages its results in a pinned buffer the library
allocates) and the other for lbm_check_state_noalloc (static device scratch): the results
must agree bit for bit.  The variant is called with a lattice as wide as its scratch allows
first and with smaller lattices after it, so stale scratch from a wider call would show.
"""
import ctypes as C
import math

import pytest

pytestmark = pytest.mark.gpu


def lattice(nx, ny, storage="f64", plug=True, **kw):
    from paper_2103_08301_amd import Lattice

    lat = Lattice(nx, ny, 1.0, storage=storage, check_every=10 ** 6, **kw)
    if plug:
        lat.init_plug(max(8, nx // 6), max(1, ny // 16), math.nan, 1e-3, 11)
    return lat


def check_via(lat, noalloc: bool):
    from paper_2103_08301_amd import lbm

    r = lbm.lbm_check_result()
    fn = lbm.library().lbm_check_state_noalloc if noalloc else lbm.library().lbm_check_state
    st = fn(lat.ctx, C.byref(r))
    assert st == lbm.LBM_OK, lbm.lbm_last_error(lat.ctx)
    return lbm.struct_dict(r)


def same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert repr(a[k]) == repr(b[k]), (k, a[k], b[k])


CASES = [
    # nx at the scratch limit first, then smaller lattices (two calls in a row, the second smaller)
    dict(nx=16384, ny=24, steps=40, kw=dict(T_over_Tc=0.9, dp=1e-3)),
    dict(nx=200, ny=40, steps=130, kw=dict(T_over_Tc=0.9, dp=2e-3)),
    dict(nx=64, ny=17, steps=9, kw=dict(T_over_Tc=0.85, dp=1e-3, storage="f32")),
]


def test_noalloc_check_equals_check():
    for case in CASES:
        kw = dict(case["kw"])
        storage = kw.pop("storage", "f64")
        a = lattice(case["nx"], case["ny"], storage, **kw)
        b = lattice(case["nx"], case["ny"], storage, **kw)
        assert a.step(case["steps"]) == 0 and b.step(case["steps"]) == 0
        want = check_via(a, noalloc=False)
        got = check_via(b, noalloc=True)
        print(f"noalloc check {case['nx']}x{case['ny']} step {got['step']}: x_rear {got['x_rear']:.6f} "
              f"x_front {got['x_front']:.6f} liquid columns {got['liquid_columns']}", flush=True)
        same(got, want)
        assert got["step"] == case["steps"]
        assert math.isfinite(got["x_rear"]) and got["liquid_columns"] > 0
        # a second call at the same step returns the stored result
        same(check_via(b, noalloc=True), want)


def test_noalloc_check_without_interfaces_and_unstable():
    import numpy as np

    # uniform periodic fluid: no interface, no liquid column
    for noalloc in (False, True):
        lat = lattice(96, 24, "f64", plug=False, T_over_Tc=0.9, x_periodic=1, y_periodic=1)
        lat.init_density(np.full((24, 96), 0.1))
        lat.step(5)
        r = check_via(lat, noalloc)
        if not noalloc:
            want = r
    same(r, want)
    assert math.isnan(r["x_rear"]) and r["liquid_columns"] == 0
    # a run driven past the velocity limit: the check reports the instability in its result
    outs = []
    for noalloc in (False, True):
        lat = lattice(64, 16, "f64", T_over_Tc=0.85, dp=2.0)
        lat.step(300)
        outs.append(check_via(lat, noalloc))
    same(outs[1], outs[0])
    assert outs[1]["unstable_step"] == 300


def test_noalloc_check_rejects_wider_lattices_and_uninitialised():
    from paper_2103_08301_amd import Lattice, lbm

    lat = Lattice(16385, 8, 1.0, storage="f32", check_every=10 ** 6, T_over_Tc=0.9)
    r = lbm.lbm_check_result()
    assert lbm.library().lbm_check_state_noalloc(lat.ctx, C.byref(r)) == lbm.LBM_ESTATE  # not initialised
    lat.init_plug(100, 1)
    assert lbm.library().lbm_check_state_noalloc(lat.ctx, C.byref(r)) == lbm.LBM_EINVAL
    assert "16384" in lbm.lbm_last_error(lat.ctx)
    assert lat.step(3) == 0 and lat.check()["step"] == 3  # the lattice works on
