"""The wall-shear sensitivity problem shared by the tangent-linear and adjoint tests.

J(theta) = int_tau2 after S steps (the time integral of squared wall shear over
both walls) of a 96 x 32 plug channel, theta = (dp, a, b, T) with T absolute;
the initial density and the wall ghost density are held fixed.  J_oracle runs
the FP64 oracle, J_gpu the library in FP64; richardson() is the
Richardson-extrapolated central difference used as the reference derivative.
"""
import math
import sys

import numpy as np

import oracle as O
from paper_2103_08301_amd import Lattice


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


NX, NY, S = 96, 32, 200


CS = dict(name="CS", tau=1.0, eos=0, a=1.0, b=4.0, R=1.0, omega=0.344, Tr=0.85, dp=1e-3, k=1.0, kappa=0.001,
          dirs=[0, 1, 2, 3])
PR = dict(name="PR", tau=1.0, eos=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344, Tr=0.95, dp=1e-3, k=0.2, kappa=0.001,
          dirs=[0, 3])  # PR tangents: dp and T only


class Problem:
    def __init__(self, cfg, nx=NX, ny=NY, steps=S):
        self.cfg = cfg
        self.nx, self.ny, self.steps = nx, ny, steps
        base = self.oparams(cfg["dp"], cfg["a"], cfg["b"], None)
        _, self.tc0 = O.critical(base)
        self.T0 = cfg["Tr"] * self.tc0
        ref = O.Sim(nx, ny, base)
        ref.init_plug(24, 3, math.nan, 1e-3, 7)
        st = ref.state()
        self.rho_w = st["rho_l"]
        self.rho_init = ref.fields()[0].copy()
        self.theta0 = np.array([cfg["dp"], cfg["a"], cfg["b"], self.T0])

    def common(self):
        c = self.cfg
        return dict(eos=c["eos"], R=c["R"], omega=c["omega"], k=c["k"], kappa=c["kappa"])

    def oparams(self, dp, a, b, T):
        c = self.cfg
        p = O.params(tau=c["tau"], a=a, b=b, dp=dp, v_limit=1.0, check_every=10 ** 6, **self.common())
        if T is not None:
            _, tc = O.critical(p)
            p = O.params(tau=c["tau"], a=a, b=b, dp=dp, v_limit=1.0, check_every=10 ** 6, T_over_Tc=T / tc,
                         rho_wall=self.rho_w, **self.common())
        else:
            p = O.params(tau=c["tau"], a=a, b=b, dp=dp, v_limit=1.0, check_every=10 ** 6, T_over_Tc=c["Tr"],
                         **self.common())
        return p

    def J_oracle(self, theta):
        dp, a, b, T = theta
        s = O.Sim(self.nx, self.ny, self.oparams(dp, a, b, T))
        s.init_density(self.rho_init)
        assert s.step(self.steps) == 0
        return s.history()[-1]["int_tau2"]

    def lattice(self, theta, storage):
        dp, a, b, T = theta
        kw = dict(self.common(), a=a, b=b, dp=dp, v_limit=1.0, check_every=10 ** 6, rho_wall=self.rho_w,
                  storage=storage)
        probe = Lattice(self.nx, self.ny, self.cfg["tau"], T_over_Tc=self.cfg["Tr"], **kw)
        tc = probe.state()["Tc"]  # the library's own critical temperature for (a, b, R)
        del probe
        lat = Lattice(self.nx, self.ny, self.cfg["tau"], T_over_Tc=T / tc, **kw)
        lat.init_density(self.rho_init)
        return lat

    def J_gpu(self, theta):
        lat = self.lattice(theta, "f64")
        assert lat.step(self.steps) == 0
        return lat.history(1)[-1]["int_tau2"]

    def jvp(self, k):
        lat = self.lattice(self.theta0, "f64t")
        e = [0.0] * 4
        e[k] = 1.0
        lat.set_tangent(*e)
        assert lat.step(self.steps) == 0
        h = lat.history(1)[-1]
        return h["int_tau2"], h["d_int_tau2"]


def richardson(J, theta0, k, rel):
    h = rel * abs(theta0[k])

    def d(hh):
        tp, tm = theta0.copy(), theta0.copy()
        tp[k] += hh
        tm[k] -= hh
        return (J(tp) - J(tm)) / (2 * hh)

    return (4 * d(h / 2) - d(h)) / 3
