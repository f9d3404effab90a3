"""The verification runs of Sec. 2.2 at reduced size, GPU against the oracle.

  * Peng-Robinson coexistence (Fig. 1a): flat PR-water slabs (k = 0.1, kappa = 0.001) in a fully
    periodic 256 x 8 box at tau 1.5 (0.9, 0.8, 0.7 Tc, 40000 steps) and tau 1.2 (0.9 Tc, 80000 steps),
    relaxed from tanh profiles of width 8 at the Maxwell densities.  The FP64 library equals the
    oracle element by element; FP32 storage and arithmetic reproduce the bulk densities, whose
    deviations from Maxwell (the oracle's table in test_oracle_coexistence_pr.py) the GPU therefore
    shares.
  * Laplace's law (eq. 2.19, Fig. 1d): static CS droplets of radius 8..16 in a periodic 64 x 64 box
    (0.9 Tc, tau 1, 9000 steps).  The FP64 library equals the oracle element by element, and the
    pressure jumps and the fitted surface tension of the FP32 runs match the oracle's.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_2103_08301_amd import Lattice  # noqa: E402

PR = dict(eos=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344)


def log(msg):
    print(msg, flush=True)


def relinf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def run_both(nx, ny, tau, steps, rho0, storages, **kw):
    ref = O.Sim(nx, ny, O.params(tau=tau, check_every=1000, v_limit=1.0, **kw))
    ref.init_density(rho0)
    assert ref.step(steps) == 0
    out = {}
    for storage in storages:
        lat = Lattice(nx, ny, tau, storage=storage, check_every=1000, v_limit=1.0, **kw)
        lat.init_density(rho0)
        assert lat.step(steps) == 0
        out[storage] = lat.fields()
    return ref.fields(), ref.state(), out


@pytest.mark.parametrize("tau,tr,steps", [(1.5, 0.9, 40000), (1.5, 0.8, 40000), (1.5, 0.7, 40000),
                                          (1.2, 0.9, 80000)])
def test_pr_slab_coexistence_matches_the_oracle(tau, tr, steps):
    nx, ny = 256, 8
    kw = dict(T_over_Tc=tr, k=0.1, kappa=0.001, x_periodic=1, y_periodic=1, dp=0.0, **PR)
    st = O.Sim(nx, ny, O.params(tau=tau, **kw)).state()
    x = np.arange(nx)
    prof = st["rho_g"] + (st["rho_l"] - st["rho_g"]) * 0.5 * (np.tanh((x - 64) / 8.0) - np.tanh((x - 192) / 8.0))
    rho0 = np.ascontiguousarray(np.tile(prof, (ny, 1)))
    (rr, vxr, vyr), st, out = run_both(nx, ny, tau, steps, rho0, ("f64", "f32"), **kw)
    e64 = relinf(out["f64"][0], rr)
    ev64 = float(np.abs(out["f64"][1] - vxr).max())
    r32 = out["f32"][0]
    dl = abs(r32[0, 128] - rr[0, 128]) / rr[0, 128]
    dg = abs(r32[0, 0] - rr[0, 0]) / rr[0, 0]
    log(f"PR slab tau {tau} T/Tc {tr}: oracle rho_l {rr[0, 128]:.6g} ({rr[0, 128] / st['rho_l'] - 1:+.3%} of Maxwell), "
        f"rho_g {rr[0, 0]:.6g} ({rr[0, 0] / st['rho_g'] - 1:+.3%}); f64 rel Linf {e64:.2e}, |dvx| {ev64:.1e}; "
        f"f32 bulk rho_l {dl:.1e}, rho_g {dg:.1e}")
    assert e64 <= 1e-9 and ev64 <= 1e-12
    assert dl <= 1e-4 and dg <= 1e-3


def droplet_rho(st, n, R):
    c = np.arange(n) + 0.5 - n / 2
    d = R - np.sqrt(c[None, :] ** 2 + c[:, None] ** 2)
    return np.ascontiguousarray(st["rho_g"] + (st["rho_l"] - st["rho_g"]) * 0.5 * (1 + np.tanh(d / 2.0)))


def jump(p, T, rho):
    n = rho.shape[0]
    rin = rho[n // 2 - 1:n // 2 + 1, n // 2 - 1:n // 2 + 1].mean()
    rout = rho[0, 0]
    req = math.sqrt(((rho - rout) / (rin - rout)).sum() / math.pi)
    return O.p0(p, T, rin) - O.p0(p, T, rout), req


def test_laplace_droplets_match_the_oracle():
    n, tau, steps = 64, 1.0, 9000
    kw = dict(T_over_Tc=0.9, k=1.0, kappa=0.001, x_periodic=1, y_periodic=1, dp=0.0)
    p = O.params(tau=tau, **kw)
    st = O.Sim(n, n, p).state()
    fits = {"oracle": [], "f64": [], "f32": []}
    for R in (8, 10, 12, 14, 16):
        (rr, _, _), _, out = run_both(n, n, tau, steps, droplet_rho(st, n, R), ("f64", "f32"), **kw)
        e64, e32 = relinf(out["f64"][0], rr), relinf(out["f32"][0], rr)
        fits["oracle"].append(jump(p, st["T"], rr))
        fits["f64"].append(jump(p, st["T"], out["f64"][0]))
        fits["f32"].append(jump(p, st["T"], out["f32"][0]))
        log(f"droplet R {R}: f64 rel Linf {e64:.2e}, f32 {e32:.2e}; jump oracle {fits['oracle'][-1][0]:.6e}, "
            f"f32 {fits['f32'][-1][0]:.6e}")
        assert e64 <= 1e-9 and e32 <= 1e-4
    sig = {}
    for k, rows in fits.items():
        dp = np.array([r[0] for r in rows])
        req = np.array([r[1] for r in rows])
        A = np.vstack([1 / req, np.ones_like(req)]).T
        (sig[k], _), *_ = np.linalg.lstsq(A, dp, rcond=None)
    log(f"surface tension: oracle {sig['oracle']:.6e}, f64 {sig['f64']:.6e}, f32 {sig['f32']:.6e}")
    assert sig["f64"] == pytest.approx(sig["oracle"], rel=1e-8)
    assert sig["f32"] == pytest.approx(sig["oracle"], rel=1e-3)
