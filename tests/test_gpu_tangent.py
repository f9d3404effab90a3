"""Forward-mode sensitivities (F64T storage) against finite differences.

Objective: J = int_tau2 after S steps, the time integral of the squared wall
shear over both walls (the wall-stress measure of Sec. 3.2-3.3), as a function
of theta = (dp, a, b, T) with T the absolute temperature.  The initial density
and the wall ghost density are held fixed.  The tangent-linear run gives
dJ/dtheta . e_k in one pass per direction; it must match

  * central differences of the FP64 oracle (Richardson-extrapolated), which is
    independent of the HIP code, and
  * central differences of the library's own FP64 runs,

and its value part must reproduce the FP64 run.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_2103_08301_amd import Lattice  # noqa: E402

NX, NY, S = 96, 32, 200


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CS = dict(name="CS", tau=1.0, eos=0, a=1.0, b=4.0, R=1.0, omega=0.344, Tr=0.85, dp=1e-3, k=1.0, kappa=0.001,
          dirs=[0, 1, 2, 3])
PR = dict(name="PR", tau=1.0, eos=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344, Tr=0.95, dp=1e-3, k=0.2, kappa=0.001,
          dirs=[0, 3])  # PR tangents: dp and T only


class Problem:
    def __init__(self, cfg):
        self.cfg = cfg
        base = self.oparams(cfg["dp"], cfg["a"], cfg["b"], None)
        _, self.tc0 = O.critical(base)
        self.T0 = cfg["Tr"] * self.tc0
        ref = O.Sim(NX, NY, base)
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
        s = O.Sim(NX, NY, self.oparams(dp, a, b, T))
        s.init_density(self.rho_init)
        assert s.step(S) == 0
        return s.history()[-1]["int_tau2"]

    def lattice(self, theta, storage):
        dp, a, b, T = theta
        kw = dict(self.common(), a=a, b=b, dp=dp, v_limit=1.0, check_every=10 ** 6, rho_wall=self.rho_w,
                  storage=storage)
        probe = Lattice(NX, NY, self.cfg["tau"], T_over_Tc=self.cfg["Tr"], **kw)
        tc = probe.state()["Tc"]  # the library's own critical temperature for (a, b, R)
        del probe
        lat = Lattice(NX, NY, self.cfg["tau"], T_over_Tc=T / tc, **kw)
        lat.init_density(self.rho_init)
        return lat

    def J_gpu(self, theta):
        lat = self.lattice(theta, "f64")
        assert lat.step(S) == 0
        return lat.history(1)[-1]["int_tau2"]

    def jvp(self, k):
        lat = self.lattice(self.theta0, "f64t")
        e = [0.0] * 4
        e[k] = 1.0
        lat.set_tangent(*e)
        assert lat.step(S) == 0
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


@pytest.mark.parametrize("cfg", [CS, PR], ids=lambda c: c["name"])
def test_tangent_matches_finite_differences(cfg):
    P = Problem(cfg)
    j64 = P.J_gpu(P.theta0)
    names = ["dp", "a", "b", "T"]
    for k in cfg["dirs"]:
        val, dj = P.jvp(k)
        assert val == pytest.approx(j64, rel=1e-12)  # the value part is the FP64 run
        fd_o = richardson(P.J_oracle, P.theta0, k, 1e-3)
        fd_g = richardson(P.J_gpu, P.theta0, k, 1e-3)
        log(f"{cfg['name']} dJ/d{names[k]}: tangent {dj:.10e}  oracle FD {fd_o:.10e}  GPU FD {fd_g:.10e}  "
            f"rel diff {abs(dj - fd_o) / abs(fd_o):.2e} / {abs(dj - fd_g) / abs(fd_g):.2e}")
        assert dj == pytest.approx(fd_o, rel=1e-6)
        assert dj == pytest.approx(fd_g, rel=1e-6)


def test_tangent_api_rules():
    lat = Lattice(64, 16, 1.0, storage="f64")
    from paper_2103_08301_amd import lbm

    with pytest.raises(lbm.LbmError):
        lat.set_tangent(dp=1.0)  # not F64T storage
    lat_pr = Lattice(64, 16, 1.2, storage="f64t", eos=1, a=2 / 49, b=2 / 21, T_over_Tc=0.9, k=0.1)
    with pytest.raises(lbm.LbmError):
        lat_pr.set_tangent(a=1.0)  # PR: dp and T only
    lat_pr.set_tangent(dp=1.0, T=1.0)
    lat_pr.init_plug(10, 2, math.nan, 0.0, 1)
    assert np.array_equal(lat_pr.get_f_tangent(), np.zeros((9, 16, 64)))  # tangents start at zero
