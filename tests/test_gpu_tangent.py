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

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import numpy as np  # noqa: E402

from paper_2103_08301_amd import Lattice  # noqa: E402
from sensitivity_problem import CS, PR, Problem, log, richardson  # noqa: E402


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
