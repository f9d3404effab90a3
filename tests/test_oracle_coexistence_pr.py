"""The reduced-size Peng-Robinson coexistence curve (Sec. 2.2 "Verification", Fig. 1a) on the oracle.

Sec. 2.2 runs PR water (a = 2/49, b = 2/21, R = 1, omega = 0.344) with k = 0.1, kappa = 0.001 and
tau = 1.2, a droplet of radius 30 relaxed for 150000 steps.  Under the method as read that droplet
diverges within 1000 steps at 0.9, 0.8 and 0.7 Tc, in a 128 x 128 periodic box, from tanh profiles
of width 4 to 12 and at tau 1.2 or 1.5.  A flat slab has no curvature and no spurious currents
around it, so the curve is taken on flat liquid slabs in a fully periodic 256 x 3 box instead,
relaxed from tanh profiles of width 8 at the Maxwell densities.  The bulk densities (slab centre,
gas far from it) are compared with the oracle's Maxwell construction, which the EOS pins fix
independently (equal area and equal pressure via scipy).

Measured (the slabs steady to |v| < 1e-4):

    tau   T/Tc   steps   rho_l / Maxwell   rho_g / Maxwell   density ratio
    1.2   0.9    80000      -2.2%             -7.7%             10.2
    1.2   0.8, 0.7         diverge within 4000 steps
    1.5   0.9    40000      -2.0%             +34%              10.2
    1.5   0.8    40000      -0.25%            -2.3%             36.6
    1.5   0.7    40000      -0.06%            -58%             145

The liquid branch follows Maxwell to within 2.5% wherever the slab is stable; the gas branch only
near 0.8 Tc at tau 1.5.  The gas error changes sign and size with tau (at 0.9 Tc: -7.7% at 1.2,
+34% at 1.5, +109% at 2.0), the signature of the forcing scheme's discretisation error, which grows
with the force and therefore with the density ratio.  The test pins the liquid branch and the
0.8 Tc gas density against Maxwell, and holds the other gas deviations and the divergences at their
measured size and sign, so a change to the oracle that moves them is seen.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.slow

PR = dict(eos=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344)
NX, NY = 256, 3


def slab(orc, tr, tau, steps):
    p = orc.params(T_over_Tc=tr, tau=tau, k=0.1, kappa=0.001, x_periodic=1, y_periodic=1, dp=0.0, v_limit=1.0,
                   check_every=1000, **PR)
    s = orc.Sim(NX, NY, p)
    st = s.state()
    x = np.arange(NX)
    prof = st["rho_g"] + (st["rho_l"] - st["rho_g"]) * 0.5 * (np.tanh((x - 64) / 8.0) - np.tanh((x - 192) / 8.0))
    s.init_density(np.tile(prof, (NY, 1)))
    status = s.step(steps)
    rho, vx, _ = s.fields()
    return status, s.unstable_step, rho, vx, st


@pytest.mark.parametrize("tau,tr,steps,gas_dev", [
    (1.2, 0.9, 80000, (-0.10, -0.05)),
    (1.5, 0.9, 40000, (0.25, 0.45)),
    (1.5, 0.8, 40000, (-0.03, 0.03)),
    (1.5, 0.7, 40000, (-0.65, -0.50)),
])
def test_pr_slab_against_maxwell(orc, tau, tr, steps, gas_dev):
    status, _, rho, vx, st = slab(orc, tr, tau, steps)
    assert status == 0
    dl = rho[0, 128] / st["rho_l"] - 1
    dg = rho[0, 0] / st["rho_g"] - 1
    print(f"PR k=0.1, tau {tau}, T/Tc {tr}: rho_l {rho[0, 128]:.6g} (Maxwell {st['rho_l']:.6g}, {dl:+.3%}), "
          f"rho_g {rho[0, 0]:.6g} (Maxwell {st['rho_g']:.6g}, {dg:+.3%}), |v|max {np.abs(vx).max():.1e}")
    assert np.abs(vx).max() < 1e-4
    assert np.ptp(rho, axis=0).max() < 1e-12  # a flat slab stays flat
    assert abs(dl) < 0.025
    assert gas_dev[0] < dg < gas_dev[1]


@pytest.mark.parametrize("tr", [0.8, 0.7])
def test_pr_slab_at_the_papers_relaxation_time_diverges_below_0_9_tc(orc, tr):
    status, unstable_step, *_ = slab(orc, tr, 1.2, 8000)
    print(f"PR k=0.1, tau 1.2, T/Tc {tr}: unstable at step {unstable_step}")
    assert status == -4 and 0 < unstable_step <= 5000
