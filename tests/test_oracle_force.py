"""Pins of the oracle's force (eq. 2.17) and wall pressure (isotropic part of eq. 2.8) against the
mathematics, through orc_eval_force, which runs the time stepper's own ghost, EOS, Laplacian, force
and wall-pressure stages on a given density field.

Force: on smooth periodic fields the lattice force must converge at second order to the
continuum force F = -grad(k^2 p0(rho) - rho/3) + kappa rho grad(lap rho) + (dp/nx, 0), whose
derivatives are written out analytically here (the EOS slope p0'(rho) by central differences
of the oracle's p0, which the EOS pins fix).  The kappa term is pinned on its own, as
F(kappa) - F(0), since at long wavelengths it is small beside the pressure term.

Wall pressure: on density profiles that are polynomials in (x, y) and meet the wetting ghost
rows exactly, the isotropic stencils act in closed form (the gradient stencil adds (1/6) of the
gradient of the Laplacian, the Laplacian stencil is exact on cubics; both pinned in
test_oracle_lattice.py), so the wall pressure k^2 p0 - kappa rho lap(rho) - kappa/2 |grad rho|^2
is known to rounding.  Each test also evaluates the formula with a planted mistake (a flipped
sign or a factor of two in one term, a dropped k^2) and asserts that it misses by far more than
the tolerance, so the pin is shown to see such a mistake.
"""
import math

import numpy as np
import pytest


def sim(orc, nx, ny, **kw):
    p = orc.params(**kw)
    return orc.Sim(nx, ny, p), p


def eos_kw(eos):
    return {} if eos == 0 else dict(eos=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344)


def p0_slope(orc, p, T, rho):
    """dp0/drho by a fourth-order central difference of the oracle's p0."""
    f = np.vectorize(lambda v: orc.p0(p, T, v))
    h = 1e-4 * float(np.mean(rho))
    return (8 * (f(rho + h) - f(rho - h)) - (f(rho + 2 * h) - f(rho - 2 * h))) / (12 * h)


def wave_field(L, rm, A, B):
    """rho = rm + A sin(ax) cos(ay) + B cos(a(x + 2y)), a = 2 pi / L, with its gradient and the
    gradient of its Laplacian, written out by hand."""
    x = np.arange(L, dtype=float)[None, :]
    y = np.arange(L, dtype=float)[:, None]
    a = 2 * math.pi / L
    s1, c1 = np.sin(a * x) * np.cos(a * y), np.cos(a * x) * np.cos(a * y)
    s2 = np.sin(a * x) * np.sin(a * y)
    cb, sb = np.cos(a * (x + 2 * y)), np.sin(a * (x + 2 * y))
    rho = rm + A * s1 + B * cb
    rx = A * a * c1 - B * a * sb
    ry = -A * a * s2 - 2 * B * a * sb
    # lap rho = -2 a^2 A s1 - 5 a^2 B cb
    lx = -2 * a ** 3 * A * c1 + 5 * a ** 3 * B * sb
    ly = 2 * a ** 3 * A * s2 + 10 * a ** 3 * B * sb
    return rho, rx, ry, lx, ly


FORCE_CASES = [  # (eos, T/Tc, k, kappa)
    (0, 0.9, 0.6, 0.01),
    (0, 0.85, 1.0, 0.001),
    (1, 0.8, 0.3, 0.001),
    (1, 0.7, 0.1, 0.01),
]


@pytest.mark.parametrize("eos,Tr,k,kappa", FORCE_CASES)
def test_force_converges_to_the_continuum_force(orc, eos, Tr, k, kappa):
    dp = 3e-3
    errs, errs_k, wrong = [], [], {}
    for L in (32, 64, 128):
        kw = dict(T_over_Tc=Tr, k=k, kappa=kappa, x_periodic=1, y_periodic=1, dp=dp, **eos_kw(eos))
        s, p = sim(orc, L, L, **kw)
        s0, _ = sim(orc, L, L, **dict(kw, kappa=0.0))
        st = s.state()
        rg, rl = st["rho_g"], st["rho_l"]
        rho, rx, ry, lx, ly = wave_field(L, 0.5 * (rg + rl), 0.3 * (rl - rg), 0.1 * (rl - rg))
        Fx, Fy, _, _ = s.eval_force(rho)
        F0x, F0y, _, _ = s0.eval_force(rho)
        phi1 = k * k * p0_slope(orc, p, st["T"], rho) - 1.0 / 3.0  # d/drho of k^2 p0 - rho/3
        g = dp / L
        Kx, Ky = kappa * rho * lx, kappa * rho * ly
        Ex, Ey = -phi1 * rx + Kx + g, -phi1 * ry + Ky
        scale = max(np.abs(Ex - g).max(), np.abs(Ey).max())
        errs.append(max(np.abs(Fx - Ex).max(), np.abs(Fy - Ey).max()) / scale)
        kscale = max(np.abs(Kx).max(), np.abs(Ky).max())
        dKx, dKy = Fx - F0x, Fy - F0y
        errs_k.append(max(np.abs(dKx - Kx).max(), np.abs(dKy - Ky).max()) / kscale)
        if L == 128:
            # planted mistakes in the expected value: each must miss far beyond the tolerance
            wrong["kappa sign"] = max(np.abs(dKx + Kx).max(), np.abs(dKy + Ky).max()) / kscale
            wrong["kappa x2"] = max(np.abs(dKx - 2 * Kx).max(), np.abs(dKy - 2 * Ky).max()) / kscale
            phi1_nok = p0_slope(orc, p, st["T"], rho) - 1.0 / 3.0
            wrong["no k^2"] = max(np.abs(Fx - (-phi1_nok * rx + Kx + g)).max(),
                                  np.abs(Fy - (-phi1_nok * ry + Ky)).max()) / scale
            wrong["ideal part sign"] = max(np.abs(Fx - (-(phi1 + 2 / 3) * rx + Kx + g)).max(),
                                           np.abs(Fy - (-(phi1 + 2 / 3) * ry + Ky)).max()) / scale
    # second order: each halving of the wavenumber divides the error by 4
    for e in (errs, errs_k):
        assert 3.7 < e[0] / e[1] < 4.3 and 3.7 < e[1] / e[2] < 4.3, e
    tol_f, tol_k = 2e-3, 4e-3  # at L = 128
    assert errs[2] < tol_f and errs_k[2] < tol_k, (errs, errs_k)
    for name, w in wrong.items():
        if name == "no k^2" and k == 1.0:
            continue  # k^2 = 1: no mistake to see
        assert w > 10 * (tol_k if name.startswith("kappa") else tol_f), (name, w)


def test_body_force_is_the_pressure_drop_over_nx(orc):
    nx, ny = 40, 24
    rho = wave_field(40, 0.15, 0.05, 0.02)[0][:ny, :]
    kw = dict(T_over_Tc=0.9, x_periodic=1)
    s1, _ = sim(orc, nx, ny, dp=2.5e-3, **kw)
    s0, _ = sim(orc, nx, ny, dp=0.0, **kw)
    F1x, F1y, _, _ = s1.eval_force(rho)
    F0x, F0y, _, _ = s0.eval_force(rho)
    assert np.allclose(F1x - F0x, 2.5e-3 / nx, rtol=0, atol=1e-15)
    assert np.array_equal(F1y, F0y)


def wall_profile(nx, ny, rho_w, c, d):
    """rho = rho_w + (c + d x) (s + 1)(s + 2), s the row's distance from its wall in rows (s = y for the
    bottom rows, ny - 1 - y for the top rows, at most 1: the wall pressure of a first row reads rows
    s = -1, 0, 1 only): it equals rho_w on the ghost rows s = -1, -2."""
    x = np.arange(nx, dtype=float)[None, :]
    y = np.arange(ny)[:, None]
    s = np.minimum(np.minimum(y, ny - 1 - y), 1).astype(float)  # rows beyond s = 1 do not reach the wall rows
    return rho_w + (c + d * x) * (s + 1) * (s + 2)


def wall_pressure_closed_form(orc, p, T, k, kappa, rho_w, c, d, x, terms=(1, 1, 1)):
    """At the first fluid row (s = 0) of the profile above: rho = rho_w + 2 q with q = c + d x;
    stencil gradient = (2 d + d/3, 3 q) (the y part is exact on the quadratic; the x part is
    d q(0)-wise exact plus (1/6) d/dx lap rho = d/3); stencil Laplacian = lap rho = 2 q (exact on
    this cubic).  terms multiplies the three terms (k^2 p0, kappa rho lap rho, kappa/2 |grad|^2)."""
    q = c + d * x
    rho = rho_w + 2 * q
    gx, gy = 2 * d + d / 3.0, 3 * q
    lap = 2 * q
    p0 = np.array([orc.p0(p, T, v) for v in rho])
    return terms[0] * k * k * p0 - terms[1] * kappa * rho * lap - terms[2] * 0.5 * kappa * (gx * gx + gy * gy)


@pytest.mark.parametrize("eos,Tr,k,kappa,rho_w,c,d", [
    (0, 0.9, 0.6, 0.01, 0.1, 0.02, 0.006),
    (0, 0.85, 1.0, 0.001, 0.25, -0.01, 0.002),
    (1, 0.8, 0.4, 0.02, 1.0, 0.1, 0.02),
])
def test_wall_pressure_is_the_isotropic_pressure_of_eq_2_8(orc, eos, Tr, k, kappa, rho_w, c, d):
    nx, ny = 24, 9
    s, p = sim(orc, nx, ny, T_over_Tc=Tr, k=k, kappa=kappa, rho_wall=rho_w, **eos_kw(eos))
    T = s.state()["T"]
    rho = wall_profile(nx, ny, rho_w, c, d)
    assert rho.min() > 0
    _, _, pb, pt = s.eval_force(rho)
    xs = np.arange(1, nx - 1)  # the end columns see the extrapolated ghost columns
    want = wall_pressure_closed_form(orc, p, T, k, kappa, rho_w, c, d, xs)
    scale = np.abs(want).max()
    for got in (pb[1:-1], pt[1:-1]):
        assert np.abs(got - want).max() <= 1e-12 * scale, np.abs(got - want).max() / scale
    # the same profile without its x slope: every column, the ends included
    rho0 = wall_profile(nx, ny, rho_w, c, 0.0)
    _, _, pb0, pt0 = s.eval_force(rho0)
    want0 = wall_pressure_closed_form(orc, p, T, k, kappa, rho_w, c, 0.0, np.arange(nx))
    assert np.abs(pb0 - want0).max() <= 1e-12 * np.abs(want0).max()
    assert np.abs(pt0 - want0).max() <= 1e-12 * np.abs(want0).max()
    # planted mistakes: a flipped sign or a factor 2 in either gradient term, a dropped k^2, the
    # x part of the gradient dropped
    tol = 1e-12 * scale
    for terms in [(1, -1, 1), (1, 2, 1), (1, 1, -1), (1, 1, 2), (1 / (k * k) if k != 1 else 1, 1, 1)]:
        if terms[0] == 1 and terms[1:] == (1, 1):
            continue
        bad = wall_pressure_closed_form(orc, p, T, k, kappa, rho_w, c, d, xs, terms)
        assert np.abs(pb[1:-1] - bad).max() > 1e4 * tol, terms
    q = c + d * xs
    rr = rho_w + 2 * q
    no_x = k * k * np.array([orc.p0(p, T, v) for v in rr]) - kappa * rr * 2 * q - 0.5 * kappa * (3 * q) ** 2
    assert np.abs(pb[1:-1] - no_x).max() > 1e4 * tol
