"""The adjoint gradient at the length of run the gradient benchmark times.

J = int_tau2, the time integral over all steps of the squared wall shear on both walls, of the
1024x256 plug channel (CS 0.95 Tc, tau 1, plug 120, film 8, noise seed 5, dp 5e-4) over 20000
steps, through the rupture of the plug (about step 11000); theta = (dp, a, b, T) with T absolute,
the initial density and the wall ghost density held fixed.  The FP32 adjoint (FP32 storage and
arithmetic, sqrt(N) checkpoints) is compared with central differences, step 1e-4 relative, of
the library's FP64 forward runs (whose FP64 forward-mode derivatives the FP64 adjoint matches to
rounding on short runs, test_gpu_adjoint.py).

At the reduced size the oracle can run many times, the 128x32 version (plug 15, film 2, 2500
steps) is compared with differences of the FP64 oracle.  There J is strongly curved in the EOS
parameters: the central difference quotients for a, b and T at steps 1e-4 and 2e-4 (relative)
differ by 0.5%, so the plain 1e-4 quotient carries ~1.5e-3 of truncation error, while the
Richardson extrapolation of the two agrees with the FP64 adjoint to ~3e-6.  The reference there is
therefore the Richardson-extrapolated difference; the plain 1e-4 quotient is printed beside it.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_2103_08301_amd import Lattice, workloads  # noqa: E402

NAMES = ["dp", "a", "b", "T"]


def log(msg):
    print(msg, flush=True)


class Case:
    """A plug channel at theta = (dp, a, b, T absolute) from a fixed initial density."""

    def __init__(self, nx, ny, tau, Tr, dp, plug, film, seed, steps):
        self.nx, self.ny, self.tau, self.steps = nx, ny, tau, steps
        base = Lattice(nx, ny, tau, storage="f64", T_over_Tc=Tr, dp=dp, check_every=10 ** 6, v_limit=1.0)
        st = base.state()
        self.rho_w, self.Tc0 = st["rho_l"], st["Tc"]
        base.init_plug(plug, film, math.nan, 1e-3, seed)
        self.rho_init = base.fields()[0].copy()
        self.theta0 = np.array([dp, 1.0, 4.0, Tr * self.Tc0])
        self.Tr = Tr

    def kw(self, theta, storage):
        dp, a, b, T = theta
        return dict(storage=storage, a=a, b=b, dp=dp, rho_wall=self.rho_w, check_every=10 ** 6, v_limit=1.0)

    def lattice(self, theta, storage):
        kw = self.kw(theta, storage)
        probe = Lattice(self.nx, self.ny, self.tau, T_over_Tc=self.Tr, **kw)
        tc = probe.state()["Tc"]
        del probe
        lat = Lattice(self.nx, self.ny, self.tau, T_over_Tc=theta[3] / tc, **kw)
        lat.init_density(self.rho_init)
        return lat

    def J64(self, theta):
        lat = self.lattice(theta, "f64")
        assert lat.step(self.steps) == 0
        return lat.history(1)[-1]["int_tau2"]

    def fd(self, J, k, rel=1e-4):
        h = rel * abs(self.theta0[k])
        tp, tm = self.theta0.copy(), self.theta0.copy()
        tp[k] += h
        tm[k] -= h
        return (J(tp) - J(tm)) / (2 * h)


def test_fp32_adjoint_at_20000_steps_against_fp64_differences():
    w = workloads.plug_adjoint("f32")
    pl = w["plug"]
    c = Case(w["nx"], w["ny"], w["tau"], w["params"]["T_over_Tc"], w["params"]["dp"], pl["plug_len"],
             pl["film"], pl["seed"], w["steps"])
    lat = c.lattice(c.theta0, "f32")
    lat.adjoint_bind(c.steps, 0)
    st, J32 = lat.adjoint_forward()
    assert st == 0
    chk = lat.check()
    grad = lat.adjoint_backward()
    J64 = c.J64(c.theta0)
    log(f"1024x256, {c.steps} steps: J f32 {J32:.9e}, f64 {J64:.9e} (rel {abs(J32 - J64) / J64:.1e}); "
        f"liquid columns at the end {chk['liquid_columns']} (rupture step {chk['rupture_step']})")
    assert J32 == pytest.approx(J64, rel=1e-3)
    for k in range(4):
        d = c.fd(c.J64, k)
        rel = abs(grad[k] - d) / abs(d)
        log(f"  dJ/d{NAMES[k]}: FP32 adjoint {grad[k]:+.9e}, FP64 central difference {d:+.9e}, rel {rel:.2e}")
        assert rel <= 1e-3, (NAMES[k], grad[k], d)


def test_fp32_adjoint_128x32_2500_steps_against_oracle_differences():
    nx, ny, steps, tau, Tr, dp = 128, 32, 2500, 1.0, 0.95, 5e-4
    c = Case(nx, ny, tau, Tr, dp, 15, 2, 5, steps)

    def J_oracle(theta):
        d, a, b, T = theta
        p = O.params(tau=tau, a=a, b=b, dp=d, v_limit=1.0, check_every=10 ** 6)
        _, tc = O.critical(p)
        p = O.params(tau=tau, a=a, b=b, dp=d, v_limit=1.0, check_every=10 ** 6, T_over_Tc=T / tc,
                     rho_wall=c.rho_w)
        s = O.Sim(nx, ny, p)
        s.init_density(c.rho_init)
        assert s.step(steps) == 0
        return s.history()[-1]["int_tau2"]

    lat = c.lattice(c.theta0, "f32")
    lat.adjoint_bind(steps, 0)
    st, J32 = lat.adjoint_forward()
    assert st == 0
    grad = lat.adjoint_backward()
    Jo = J_oracle(c.theta0)
    log(f"128x32, {steps} steps: J f32 {J32:.9e}, oracle {Jo:.9e}")
    assert J32 == pytest.approx(Jo, rel=1e-4)
    for k in range(4):
        d1, d2 = c.fd(J_oracle, k, 1e-4), c.fd(J_oracle, k, 2e-4)
        d = (4 * d1 - d2) / 3  # Richardson: the step-squared truncation removed
        rel = abs(grad[k] - d) / abs(d)
        log(f"  dJ/d{NAMES[k]}: FP32 adjoint {grad[k]:+.9e}, oracle Richardson difference {d:+.9e} (rel {rel:.2e}); "
            f"plain 1e-4 central difference {d1:+.9e} (rel {abs(grad[k] - d1) / abs(d1):.2e})")
        assert rel <= 1e-3, (NAMES[k], grad[k], d)
