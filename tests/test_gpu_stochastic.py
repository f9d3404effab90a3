"""FP16 storage with stochastic rounding (storage "f16r").

With the storage shift set to zero, an F16R lattice stores each post-collision
population v (computed in FP32) as one of the two FP16 values next to it, and
the round-to-nearest storage F16S stores the nearest one.  One step from a
state that all three storages represent exactly (FP16 values) therefore
checks the rounding itself against an FP32 lattice run of the same step:

  * every F16R value is the FP16 value just below or just above v (v itself
    when v is an FP16 value), and F16S gives numpy's round-to-nearest of v;
  * the F16R roundings are unbiased: over all populations, the fraction
    rounded up matches the mean fractional position of v between its two
    neighbours, and the mean rounding error is zero, both to within the
    sampling error of tens of thousands of independent draws;
  * the random bits depend on the step counter, node and direction only:
    two runs are bitwise equal, the next step draws other bits.

The FP32 lattice evaluates the EOS field phi and its gradient in FP64, the FP16
storages in FP32, so v can differ by ~1e-9 from the FP32 value the FP16 kernels
round.  The exact checks therefore accept the FP16 neighbours (F16R) and the
nearest FP16 value (F16S) of any value within TIE of v; the statistics use v.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2103_08301_amd import Lattice  # noqa: E402

NX, NY = 200, 60
KW = dict(T_over_Tc=0.9, dp=1e-3, rho0_shift=0.0, check_every=10 ** 6, v_limit=1.0)


def log(msg):
    print(msg, flush=True)


def start(storage, f0=None):
    lat = Lattice(NX, NY, 0.9, storage=storage, **KW)
    lat.init_plug(50, 5, math.nan, 1e-3, 5)
    if f0 is not None:
        lat.set_f(f0)
    return lat


TIE = 1e-7


def is_neighbour_within_tie(h, v):
    """h is an FP16 neighbour of v - TIE or of v + TIE."""
    v = v.astype(np.float64)
    lo_m, hi_m = neighbours(v - TIE)
    lo_p, hi_p = neighbours(v + TIE)
    return (h == lo_m) | (h == hi_m) | (h == lo_p) | (h == hi_p)


def is_nearest_within_tie(n, v):
    """n is the FP16 value nearest to v - TIE or to v + TIE."""
    v = v.astype(np.float64)
    return (n == (v - TIE).astype(np.float16).astype(np.float64)) | (n == (v + TIE).astype(np.float16).astype(np.float64))


def neighbours(v):
    """FP16 values just below and just above each value of v (equal when v is an FP16 value)."""
    h = v.astype(np.float16)
    hd = h.astype(v.dtype)
    lo = np.where(hd <= v, h, np.nextafter(h, np.float16(-np.inf)))
    hi = np.where(hd >= v, h, np.nextafter(h, np.float16(np.inf)))
    return lo.astype(np.float64), hi.astype(np.float64)


def test_one_step_rounds_to_a_neighbour_without_bias():
    r = start("f16r")
    f0 = r.get_f()
    assert np.array_equal(f0, f0.astype(np.float16).astype(np.float64))  # FP16 values (shift 0)
    s = start("f32", f0)
    n = start("f16s", f0)
    for lat in (r, s, n):
        assert lat.step(1) == 0
    v = s.get_f().astype(np.float32)
    h = r.get_f()
    lo, hi = neighbours(v)
    exact = (h == lo) | (h == hi)
    log(f"{int((~exact).sum())} of {v.size} values not rounded to a neighbour of the FP32 lattice's value")
    assert np.all(exact | is_neighbour_within_tie(h, v))
    assert np.all(is_nearest_within_tie(n.get_f(), v))  # round to nearest
    m = hi > lo
    t = (v[m].astype(np.float64) - lo[m]) / (hi[m] - lo[m])  # position of v between its neighbours
    up = (h[m] == hi[m]).astype(np.float64)
    k = int(m.sum())
    err = (h[m] - v[m]) / (hi[m] - lo[m])  # rounding error in units of the local FP16 spacing
    sigma = math.sqrt(float(np.mean(t * (1 - t))) / k)
    log(f"{k} inexact values: rounded up {up.mean():.4f}, mean position {t.mean():.4f}, "
        f"mean error {err.mean():+.2e} ulp (sampling sigma {sigma:.1e}); round to nearest {np.mean(np.abs(np.round(t) - t)):.3f}")
    assert k > 20000
    assert abs(up.mean() - t.mean()) < 5 * sigma + 1e-3  # 10 random bits: bias below 1/1024 ulp
    assert abs(err.mean()) < 5 * sigma + 1e-3
    # values close to a neighbour go there more often than values in the middle
    near = up[t < 0.25].mean(), up[t > 0.75].mean()
    assert near[0] < 0.3 and near[1] > 0.7


def test_runs_are_reproducible_and_steps_draw_new_bits():
    a, b = start("f16r"), start("f16r")
    assert a.step(37) == 0 and b.step(37) == 0
    assert np.array_equal(a.get_f(), b.get_f())
    # same state, different step counter: the roundings differ
    f = a.get_f()
    c = start("f16r", f)  # counter at zero, state of step 37
    a.step(1)
    c.step(1)
    d = np.count_nonzero(a.get_f() != c.get_f())
    log(f"values that rounded differently with another step counter: {d} of {f.size}")
    assert d > 1000


def test_values_just_above_powers_of_two_round_to_a_neighbour_without_bias():
    """Populations placed just above powers of two: at rho = 9/16 the rest populations w_i rho are 1/4,
    1/16 and 1/64.  A periodic state of FP16 values f_i = fp16(w_i rho(x)), rho(x) = 9/16 plus noise of
    1.5e-3 (a few FP16 spacings), gives post-collision values on both sides of those powers of two; the
    ones at most a quarter
    of the FP16 spacing above one must round to that power of two or the FP16 value above it (never
    into the finer binade below), and their mean rounding error must vanish."""
    rng = np.random.default_rng(17)
    nx, ny = 256, 128
    kw = dict(T_over_Tc=0.9, dp=0.0, rho0_shift=0.0, check_every=10 ** 6, v_limit=1.0, x_periodic=1, y_periodic=1)
    rho = 0.5625 + 1.5e-3 * (2 * rng.random((ny, nx)) - 1)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    f0 = (w[:, None, None] * rho[None]).astype(np.float16).astype(np.float64)
    lats = {}
    for storage in ("f16r", "f32"):
        lat = Lattice(nx, ny, 0.9, storage=storage, **kw)
        lat.set_f(f0)
        assert lat.step(1) == 0
        lats[storage] = lat
    v = lats["f32"].get_f().astype(np.float32)
    h = lats["f16r"].get_f()
    lo, hi = neighbours(v)
    assert np.all((h == lo) | (h == hi) | is_neighbour_within_tie(h, v))
    p2 = 2.0 ** np.floor(np.log2(v.astype(np.float64)))
    spacing = hi - lo
    t = np.where(spacing > 0, (v - lo) / np.where(spacing > 0, spacing, 1), 0)
    near = (lo == p2) & (spacing > 0) & (t <= 0.25)  # within a quarter spacing above a power of two
    k = int(near.sum())
    err = (h[near] - v[near]) / spacing[near]
    sigma = math.sqrt(float(np.mean(t[near] * (1 - t[near]))) / k)
    log(f"{k} values within s/4 above a power of two: mean position {t[near].mean():.4f}, "
        f"rounded up {np.mean(h[near] == hi[near]):.4f}, mean error {err.mean():+.2e} ulp (sigma {sigma:.1e})")
    assert k > 5000
    assert abs(err.mean()) < 5 * sigma + 1e-3
