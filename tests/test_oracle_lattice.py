"""Pins of the oracle's lattice building blocks (paper Sec. 2.1, eqs. 2.1-2.2, 2.12/2.17).

Checked against what the mathematics fixes: the D2Q9 weight identities that make
eq. 2.2 a second-order Hermite expansion with c_s^2 = 1/3, the Lallemand-Luo
moment polynomials, the moments of the equilibrium, the BGK special case of the
MRT collision, numpy's matrix inverse, the Taylor expansion of the isotropic
stencils on polynomials, and SplitMix64's published outputs.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def lattice(orc):
    v = orc.velocities()
    e = np.array([[a, b] for a, b, _ in v], dtype=float)
    w = np.array([c for _, _, c in v])
    return e, w


def test_d2q9_weight_identities(orc):
    e, w = lattice(orc)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w @ e, 0.0, atol=1e-16)
    # second moment: c_s^2 delta, c_s^2 = 1/3 as fixed by the 3, 9/2, 3/2 of eq. 2.2
    second = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.allclose(second, np.eye(2) / 3.0, atol=1e-15)
    # third moment vanishes, fourth is isotropic: c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    third = np.einsum("i,ia,ib,ic->abc", w, e, e, e)
    assert np.allclose(third, 0.0, atol=1e-16)
    fourth = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(fourth, iso, atol=1e-15)
    # every velocity has its opposite in the set
    for i in range(9):
        assert any(np.array_equal(e[j], -e[i]) for j in range(9))


def test_moment_matrix_is_lallemand_luo(orc):
    """Rows built from the Lallemand-Luo polynomials of the velocity (PRE 61, 6546, 2000)."""
    e, _ = lattice(orc)
    ex, ey = e[:, 0], e[:, 1]
    c2 = ex**2 + ey**2
    rows = [
        np.ones(9),                        # rho
        -4 + 3 * c2,                       # e
        4 - 21 / 2 * c2 + 9 / 2 * c2**2,   # epsilon
        ex,                                # jx
        (-5 + 3 * c2) * ex,                # qx
        ey,                                # jy
        (-5 + 3 * c2) * ey,                # qy
        ex**2 - ey**2,                     # pxx
        ex * ey,                           # pxy
    ]
    M = orc.moment_matrix()
    assert np.array_equal(M, np.array(rows))
    G = M @ M.T
    assert np.allclose(G, np.diag(np.diag(G)))
    assert np.array_equal(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])


def test_equilibrium_moments(orc):
    e, _ = lattice(orc)
    rng = np.random.default_rng(0)
    for _ in range(20):
        rho = rng.uniform(0.01, 9.0)
        u = rng.uniform(-0.2, 0.2, 2)
        f = orc.equilibrium(rho, u[0], u[1])
        assert f.sum() == pytest.approx(rho, rel=1e-14)
        assert np.allclose(f @ e, rho * u, rtol=1e-13, atol=1e-15)
        pi = np.einsum("i,ia,ib->ab", f, e, e)
        assert np.allclose(pi, rho * (np.eye(2) / 3.0 + np.outer(u, u)), rtol=1e-13, atol=1e-15)


def test_equilibrium_in_moment_space(orc):
    """M f_eq(rho, u) in exact rationals equals
    (rho, -2rho+3rho|u|^2, rho-3rho|u|^2, rho ux, -rho ux, rho uy, -rho uy, rho(ux^2-uy^2), rho ux uy)."""
    M = orc.moment_matrix().astype(int)
    e, _ = lattice(orc)
    W = [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4
    for rho, ux, uy in [(Fraction(3, 7), Fraction(1, 10), Fraction(-1, 25)), (Fraction(2), Fraction(0), Fraction(1, 5))]:
        feq = []
        for i in range(9):
            eu = int(e[i, 0]) * ux + int(e[i, 1]) * uy
            feq.append(rho * W[i] * (1 + 3 * eu + Fraction(9, 2) * eu * eu - Fraction(3, 2) * (ux * ux + uy * uy)))
        m = [sum(M[k, i] * feq[i] for i in range(9)) for k in range(9)]
        u2 = ux * ux + uy * uy
        want = [rho, -2 * rho + 3 * rho * u2, rho - 3 * rho * u2, rho * ux, -rho * ux, rho * uy, -rho * uy,
                rho * (ux * ux - uy * uy), rho * ux * uy]
        assert m == want
        fo = orc.equilibrium(float(rho), float(ux), float(uy))
        assert np.allclose(fo, [float(x) for x in feq], rtol=1e-15, atol=1e-17)


def random_populations(orc, rng, rho=None):
    rho = rng.uniform(0.02, 0.3) if rho is None else rho
    u = rng.uniform(-0.05, 0.05, 2)
    f = orc.equilibrium(rho, u[0], u[1]) * (1 + rng.uniform(-0.05, 0.05, 9))
    return f


def test_mrt_with_uniform_rates_is_bgk_with_velocity_shift(orc):
    """With every rate equal to 1/tau, M^-1 S M = I/tau and the MRT step of eq. 2.1
    is the BGK step with the velocity shift of Sec. 2.2: u_eq = u + tau F/rho."""
    e, _ = lattice(orc)
    rng = np.random.default_rng(1)
    for tau in [0.6, 1.0, 1.7]:
        p = orc.params(tau=tau, s_e=1 / tau, s_eps=1 / tau, s_q=1 / tau)
        for _ in range(10):
            f = random_populations(orc, rng)
            F = rng.uniform(-1e-3, 1e-3, 2)
            out, rho, vx, vy = orc.collide_node(p, f, F[0], F[1])
            r = f.sum()
            u = (f @ e) / r
            ueq = u + tau * F / r
            bgk = f - (f - orc.equilibrium(r, ueq[0], ueq[1])) / tau
            assert np.allclose(out, bgk, rtol=1e-13, atol=1e-16)
            assert rho == pytest.approx(r, rel=1e-15)
            assert [vx, vy] == pytest.approx(list(u + F / (2 * r)), rel=1e-12, abs=1e-16)


def test_mrt_collision_against_numpy_inverse(orc):
    """General rates: f* = f - M^-1 S (M f - M f_eq(rho, u + tau F/rho)), with M^-1 from numpy."""
    e, _ = lattice(orc)
    M = orc.moment_matrix()
    Minv = np.linalg.inv(M)
    rng = np.random.default_rng(2)
    p = orc.params(tau=0.8)
    S = np.diag([0, p.s_e, p.s_eps, 1 / p.tau, p.s_q, 1 / p.tau, p.s_q, 1 / p.tau, 1 / p.tau])
    for _ in range(20):
        f = random_populations(orc, rng)
        F = rng.uniform(-1e-3, 1e-3, 2)
        out, *_ = orc.collide_node(p, f, F[0], F[1])
        r = f.sum()
        ueq = (f @ e) / r + p.tau * F / r
        want = f - Minv @ S @ (M @ f - M @ orc.equilibrium(r, ueq[0], ueq[1]))
        assert np.allclose(out, want, rtol=1e-12, atol=1e-16)
        # mass is conserved and the momentum gains exactly F (momentum rows relax at 1/tau)
        assert out.sum() == pytest.approx(f.sum(), rel=1e-14)
        assert np.allclose(out @ e - f @ e, F, rtol=1e-9, atol=1e-16)


def poly_grid(fn, n=12):
    y, x = np.mgrid[0:n, 0:n].astype(float)
    x -= 4.3
    y -= 5.1
    return x, y, fn(x, y)


def test_isotropic_gradient_exact_on_quadratics(orc):
    c = [0.3, -1.1, 0.7, 0.25, -0.4, 0.9]
    fn = lambda x, y: c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
    x, y, a = poly_grid(fn)
    gx, gy = orc.grad_field(a)
    X, Y = x[1:-1, 1:-1], y[1:-1, 1:-1]
    assert np.allclose(gx, c[1] + 2 * c[3] * X + c[4] * Y, atol=1e-12)
    assert np.allclose(gy, c[2] + c[4] * X + 2 * c[5] * Y, atol=1e-12)


def test_isotropic_laplacian_exact_on_cubics(orc):
    fn = lambda x, y: 0.2 * x**3 - 0.5 * x * x * y + 0.3 * y**3 + 0.7 * x * y + 1.5 * y * y - x
    x, y, a = poly_grid(fn)
    lap = orc.lap_field(a)
    X, Y = x[1:-1, 1:-1], y[1:-1, 1:-1]
    want = 1.2 * X - 1.0 * Y + 1.8 * Y + 3.0
    assert np.allclose(lap, want, atol=1e-11)


def test_stencil_leading_errors(orc):
    """Taylor expansion: grad_h = grad + (1/6) grad lap + O(h^4),
    lap_h = lap + (1/12) lap^2 + O(h^4); both exact for these quartics/cubics."""
    # psi = x^3 : grad lap psi = (6, 0); grad_h x^3 = 3x^2 + 1
    x, y, a = poly_grid(lambda x, y: x**3)
    gx, gy = orc.grad_field(a)
    X = x[1:-1, 1:-1]
    assert np.allclose(gx, 3 * X**2 + 6.0 / 6.0, atol=1e-10)
    assert np.allclose(gy, 0.0, atol=1e-12)
    # psi = x^4 : lap^2 psi = 24; lap_h x^4 = 12 x^2 + 2
    x, y, a = poly_grid(lambda x, y: x**4)
    lap = orc.lap_field(a)
    X = x[1:-1, 1:-1]
    assert np.allclose(lap, 12 * X**2 + 24.0 / 12.0, atol=1e-9)
    # psi = x^2 y^2 : lap^2 = 8 and lap_h carries the mixed term as well
    x, y, a = poly_grid(lambda x, y: x * x * y * y)
    lap = orc.lap_field(a)
    X, Y = x[1:-1, 1:-1], y[1:-1, 1:-1]
    assert np.allclose(lap, 2 * X**2 + 2 * Y**2 + 8.0 / 12.0, atol=1e-9)


def test_splitmix64_published_outputs(orc):
    with open(os.path.join(GOLD, "eos_literature.json")) as fh:
        ref = json.load(fh)["splitmix64_seed0"]["outputs"]
    assert [orc.splitmix64(0, i) for i in range(3)] == [int(h, 16) for h in ref]
