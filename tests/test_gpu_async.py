"""lbm_step without a host wait: fields and checks formed on demand, and graph capture ahead of a call.

A call of lbm_step emits the fields and waits for the device only at a check step.  The fields
and the check of any other step are formed when they are asked for, by launching the latest
step again with field output.  These tests hold that to the bit: the on-demand fields equal
the ones a check step emits, asking for them leaves the state untouched (also for the
stochastic-rounding storage, whose random bits come from a step counter kept on the device,
and for the tangent-linear storage), and lbm_capture changes nothing but the time of the call.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KW = dict(T_over_Tc=0.9, dp=2e-3, v_limit=1.0)

VARIANTS = [
    ("f64", {}),
    ("f32", {}),
    ("f16r", {}),
    ("f16s", {}),
    ("f32", {"fused_steps": 2}),
    ("f64", {"schedule": 1}),
    ("f64", {"schedule": 2}),
    ("f32", {"graph_steps": -1}),
    ("f64t", {}),
]


def lattice(storage, extra, check_every):
    from paper_2103_08301_amd import Lattice

    lat = Lattice(150, 41, 0.9, storage=storage, check_every=check_every, **KW, **extra)
    if storage == "f64t":
        lat.set_tangent(dp=1.0, T=0.3)
    lat.init_plug(30, 3, math.nan, 1e-3, 7)
    return lat


def same_check(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert repr(a[k]) == repr(b[k]), k


@pytest.mark.parametrize("storage,extra", VARIANTS, ids=[f"{s}-{'-'.join(f'{k}{v}' for k, v in e.items())}"
                                                         for s, e in VARIANTS])
def test_fields_on_demand_equal_emitted_and_leave_the_state(storage, extra):
    # a: checks only at step 1000; fields and checks formed on demand after each call
    # b: a check step at 37 (emits the fields there) and nothing asked for in between
    # c: the same calls as a, with nothing asked for until the end
    a = lattice(storage, extra, 1000)
    b = lattice(storage, extra, 37)
    c = lattice(storage, extra, 1000)
    assert a.step(37) == 0 and b.step(37) == 0 and c.step(37) == 0
    fa, fb = a.fields(), b.fields()
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)
    same_check(a.check(), b.check())
    assert a.check()["step"] == 37
    wa, sa = a.wall()
    wb, sb = b.wall()
    for key in wa:
        assert np.array_equal(wa[key], wb[key]), key
    same_check(sa, sb)
    # ask again (a no-op), then go on: 40 more steps in three calls
    a.fields()
    for n in (1, 14, 25):
        assert a.step(n) == 0 and b.step(n) == 0 and c.step(n) == 0
        a.fields()
        a.check()
    assert a.steps == b.steps == c.steps == 77
    for lat in (b, c):
        assert np.array_equal(a.get_f(), lat.get_f())
        if storage == "f64t":
            assert np.array_equal(a.get_f_tangent(), lat.get_f_tangent())
    ha, hb, hc = a.history(), b.history(), c.history()
    assert len(ha) == len(hb) == len(hc) == 77
    for x, y, z in zip(ha, hb, hc):
        same_check(x, y)
        same_check(x, z)
    for x, y in zip(a.fields(), c.fields()):
        assert np.array_equal(x, y)
    same_check(a.check(), c.check())


@pytest.mark.parametrize("storage", ["f32", "f16r"])
def test_capture_changes_nothing_but_the_launch(storage):
    from paper_2103_08301_amd import Lattice

    lats = []
    for capture in (False, True):
        lat = Lattice(200, 48, 0.8, storage=storage, check_every=1000, graph_steps=16, **KW)
        lat.init_plug(40, 4, math.nan, 1e-3, 3)
        assert lat.step(5) == 0
        if capture:
            f0 = lat.get_f()
            lat.capture(70)
            lat.capture(70)  # already captured: nothing to do
            assert lat.steps == 5
            assert np.array_equal(lat.get_f(), f0)
        assert lat.step(70) == 0
        lats.append(lat)
    a, b = lats
    assert np.array_equal(a.get_f(), b.get_f())
    for x, y in zip(a.history(), b.history()):
        same_check(x, y)
    same_check(a.check(), b.check())


def test_autotune_and_set_f_keep_the_latest_fields():
    """Both overwrite a distribution buffer: the fields of the latest step are formed first."""
    from paper_2103_08301_amd import Lattice

    ref = lattice("f32", {}, 1000)
    ref.step(30)
    want = ref.fields()
    lat = lattice("f32", {}, 1000)
    lat.step(30)
    lat.autotune(3)
    for x, y in zip(lat.fields(), want):
        assert np.array_equal(x, y)
    lat2 = lattice("f32", {}, 1000)
    lat2.step(30)
    lat2.set_f(lat2.get_f())
    for x, y in zip(lat2.fields(), want):
        assert np.array_equal(x, y)
    assert lat2.step(10) == 0  # and stepping goes on from the state that was set
    ref.step(10)
    assert np.array_equal(lat2.get_f(), ref.get_f())


def test_batch_fields_on_demand_equal_emitted():
    from paper_2103_08301_amd import Batch

    cases = [dict(nx=96, ny=32, tau=1.0, dp=1e-3), dict(nx=130, ny=40, tau=0.8, dp=2e-3)]
    runs = []
    for check_every in (1000, 45):
        b = Batch(cases, storage="f32", check_every=check_every, v_limit=1.0, T_over_Tc=0.9)
        for k in range(2):
            b[k].init_plug(20, 2, math.nan, 1e-3, k + 1)
        b.capture(45)
        b.step(45)
        runs.append(b)
    for k in range(2):
        for x, y in zip(runs[0][k].fields(), runs[1][k].fields()):
            assert np.array_equal(x, y)
        same_check(runs[0][k].check(), runs[1][k].check())
    for b in runs:
        b.step(20)
    for k in range(2):
        assert np.array_equal(runs[0][k].get_f(), runs[1][k].get_f())
