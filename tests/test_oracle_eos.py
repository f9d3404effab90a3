"""Pins of the oracle's equations of state and Maxwell construction (paper Sec. 2.2, eq. 2.18).

Each check compares the oracle with something other than itself: literature
critical constants, finite differences of the oracle's own p0 (independent of
its analytic derivative code), the defining equal-area property evaluated with
scipy's quadrature, Pitzer's definition of the acentric factor, the mean-field
critical exponent, and the density ratio printed in the paper.
"""
import json
import warnings
import math
import os

import numpy as np
import pytest
import scipy.integrate as si
import scipy.optimize as so

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def lit():
    with open(os.path.join(GOLD, "eos_literature.json")) as fh:
        return json.load(fh)


def paper():
    with open(os.path.join(GOLD, "paper_constants.json")) as fh:
        return json.load(fh)


def pr_params(orc, omega=0.344):
    c = paper()["pr_water"]
    return orc.params(eos=orc.EOS_PR, a=c["a"], b=c["b"], R=c["R"], omega=omega)


def test_cs_critical_point_matches_literature(orc):
    ref = lit()["carnahan_starling_vdw"]
    p = orc.params(eos=orc.EOS_CS, a=ref["a"], b=ref["b"], R=ref["R"])
    rc, tc = orc.critical(p)
    assert tc == pytest.approx(ref["Tc"], rel=ref["rel_tol"])
    assert rc == pytest.approx(ref["rho_c"], rel=ref["rel_tol"])


def test_pr_critical_point_matches_peng_robinson_constants(orc):
    ref = lit()["peng_robinson"]
    for a, b in [(2.0 / 49.0, 2.0 / 21.0), (1.0, 1.0), (0.3, 0.05)]:
        p = orc.params(eos=orc.EOS_PR, a=a, b=b, R=1.0, omega=0.0)
        rc, tc = orc.critical(p)
        # a = Omega_a R^2 Tc^2/pc and b = Omega_b R Tc/pc  =>  Tc = Omega_b a / (Omega_a b R)
        assert tc == pytest.approx(ref["Omega_b"] * a / (ref["Omega_a"] * b), rel=ref["rel_tol"])
        pc = orc.p0(p, tc, rc)
        assert pc * b / (tc) == pytest.approx(ref["Omega_b"], rel=ref["rel_tol"])
        assert pc / (rc * tc) == pytest.approx(ref["Z_c"], rel=ref["rel_tol"])
    ref2 = lit()["peng_robinson_lbm_units"]
    p = orc.params(eos=orc.EOS_PR, a=ref2["a"], b=ref2["b"], R=ref2["R"])
    assert orc.critical(p)[1] == pytest.approx(ref2["Tc"], rel=ref2["rel_tol"])


@pytest.mark.parametrize("eos", [0, 1])
def test_critical_point_is_inflection_by_finite_differences(orc, eos):
    p = orc.params(eos=eos) if eos == 0 else pr_params(orc)
    rc, tc = orc.critical(p)
    h = rc * 1e-3
    f = lambda r: orc.p0(p, tc, r)
    d1 = (f(rc + h) - f(rc - h)) / (2 * h)
    d2 = (f(rc + h) - 2 * f(rc) + f(rc - h)) / h**2
    scale1 = f(rc) / rc
    scale2 = f(rc) / rc**2
    assert abs(d1) < 1e-5 * scale1
    assert abs(d2) < 1e-4 * scale2
    # slightly below Tc the isotherm is no longer monotone, slightly above it is
    r = np.linspace(0.5 * rc, 1.5 * rc, 2001)
    below = np.diff([orc.p0(p, 0.999 * tc, x) for x in r])
    above = np.diff([orc.p0(p, 1.001 * tc, x) for x in r])
    assert below.min() < 0 < above.min()


@pytest.mark.parametrize("eos", [0, 1])
def test_analytic_derivatives_match_finite_differences(orc, eos):
    """orc_dp0 (hand-derived derivatives) against Richardson-extrapolated central
    differences of orc_p0 itself."""
    p = orc.params(eos=eos) if eos == 0 else pr_params(orc)
    rc, tc = orc.critical(p)
    for T in [0.6 * tc, 0.85 * tc, 1.2 * tc]:
        for r in [0.05 * rc, 0.4 * rc, rc, 1.7 * rc]:
            f = lambda x: orc.p0(p, T, x)

            def d1(h):
                return (f(r + h) - f(r - h)) / (2 * h)

            def d2(h):
                return (f(r + h) - 2 * f(r) + f(r - h)) / h**2

            h = r * 1e-3
            fd1 = (4 * d1(h / 2) - d1(h)) / 3
            fd2 = (4 * d2(h / 2) - d2(h)) / 3
            s1 = abs(f(r)) / r + abs(fd1)
            assert abs(orc.dp0(p, T, r, 1) - fd1) < 1e-8 * s1
            assert abs(orc.dp0(p, T, r, 2) - fd2) < 1e-5 * (abs(fd2) + s1 / r)


@pytest.mark.parametrize("eos", [0, 1])
def test_ideal_gas_limit(orc, eos):
    p = orc.params(eos=eos) if eos == 0 else pr_params(orc)
    _, tc = orc.critical(p)
    T = 0.7 * tc
    for r in [1e-8, 1e-6]:
        assert orc.p0(p, T, r) / (r * p.R * T) == pytest.approx(1.0, rel=1e-4)


@pytest.mark.parametrize("eos,ratios", [(0, [0.95, 0.9, 0.85, 0.8, 0.7]), (1, [0.9, 0.8, 0.7, 0.6, 0.5])])
def test_maxwell_equal_area_and_equal_pressure(orc, eos, ratios):
    p = orc.params(eos=eos) if eos == 0 else pr_params(orc)
    _, tc = orc.critical(p)
    for tr in ratios:
        T = tr * tc
        rg, rl, ps = orc.coexistence(p, T)
        assert 0 < rg < rl
        assert orc.p0(p, T, rg) == pytest.approx(ps, rel=1e-10)
        assert orc.p0(p, T, rl) == pytest.approx(ps, rel=1e-10)
        g = lambda r: (orc.p0(p, T, r) - ps) / r**2
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            area, _ = si.quad(g, rg, rl, limit=400, epsabs=0, epsrel=1e-12)
            scale, _ = si.quad(lambda r: abs(g(r)), rg, rl, limit=400, epsabs=0, epsrel=1e-10)
        assert abs(area) < 1e-8 * scale
        # both roots are the outer roots of p0 = p*: a third root lies between them
        mid = so.brentq(lambda r: orc.p0(p, T, r) - ps, rg * 1.0001, rl * 0.9999) if (
            orc.p0(p, T, rg * 1.0001) - ps) * (orc.p0(p, T, rl * 0.9999) - ps) < 0 else None
        assert mid is not None and rg < mid < rl


def test_coexistence_width_has_mean_field_exponent(orc):
    beta = lit()["mean_field_exponent"]["beta"]
    for p in [orc.params(), pr_params(orc)]:
        _, tc = orc.critical(p)
        w = lambda tr: (lambda g, l, _: l - g)(*orc.coexistence(p, tr * tc))
        # (1 - 0.9999) / (1 - 0.9996) = 1/4  =>  width ratio (1/4)^beta
        assert w(0.9999) / w(0.9996) == pytest.approx(0.25**beta, rel=1e-3)


def test_pr_alpha_reproduces_pitzer_acentric_factor(orc):
    ref = lit()["pitzer_acentric_definition"]
    for omega in [paper()["pr_water"]["omega_water"], paper()["pr_water"]["omega_methane"]]:
        p = pr_params(orc, omega)
        rc, tc = orc.critical(p)
        pc = orc.p0(p, tc, rc)
        _, _, psat = orc.coexistence(p, ref["Tr"] * tc)
        assert -1.0 - math.log10(psat / pc) == pytest.approx(omega, abs=ref["tol"])
        assert orc.alpha(p, tc, tc) == pytest.approx(1.0, abs=1e-15)


def test_pr_water_density_ratio_nears_1000_at_tr_0_6(orc):
    """The paper states the density ratio nears 1000 at Tr = 0.6 (Sec. 2.3).

    The standard PR alpha(T) gives about 850; the alpha printed in the text,
    kappa_w = 0.37464 + 1.5422 w^2 (a garbled form), would give about 340,
    which is why the standard correlation is the reading taken."""
    c = paper()["airway_density_ratio"]
    p = pr_params(orc)
    _, tc = orc.critical(p)
    rg, rl, _ = orc.coexistence(p, c["Tr"] * tc)
    assert 0.7 * c["ratio_nears"] < rl / rg <= c["ratio_nears"]
    # the printed form, expressed through an equivalent acentric factor
    kw = 0.37464 + 1.5422 * 0.344**2
    w_eq = so.brentq(lambda w: 0.37464 + 1.54226 * w - 0.26992 * w * w - kw, 0.0, 1.0)
    rg2, rl2, _ = orc.coexistence(pr_params(orc, w_eq), c["Tr"] * tc)
    assert rl2 / rg2 < 0.5 * c["ratio_nears"]
