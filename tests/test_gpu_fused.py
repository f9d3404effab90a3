"""Two steps per launch (the tile schedule's temporally blocked kernel) against
one-step launches: states, fields, per-step wall summaries and checks must be
bit-identical, for every storage type, walls and ends of both kinds, ragged and
tiny grids, with and without captured graphs."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2103_08301_amd import Lattice  # noqa: E402

GRIDS = [
    # nx, ny, tau, kwargs
    (130, 37, 0.9, dict(dp=2e-3, T_over_Tc=0.95)),                          # ragged strips and tiles
    (61, 9, 1.0, dict(dp=1e-3, T_over_Tc=0.9)),                             # fewer rows than a tile
    (200, 40, 1.0, dict(dp=1e-3, T_over_Tc=0.9, x_periodic=1)),              # periodic ends
    (150, 33, 1.0, dict(dp=1e-3, T_over_Tc=0.9, x_periodic=1, y_periodic=1)),  # no walls
    (300, 70, 1.1, dict(dp=1e-3, T_over_Tc=0.9, rho_wall=0.4, kappa=0.005)),  # interior tiles, other wettability
    (110, 30, 1.2, dict(eos=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344, T_over_Tc=0.9, k=0.1, dp=1e-3)),  # PR
]


def run(nx, ny, tau, kw, storage, fused, graph_steps, calls):
    lat = Lattice(nx, ny, tau, storage=storage, fused_steps=fused, graph_steps=graph_steps, check_every=101,
                  v_limit=1.0, **kw)
    lat.init_plug(max(4, nx // 5), 0 if kw.get("y_periodic") else 2, math.nan, 1e-3, nx)
    for n in calls:
        assert lat.step(n) == 0
    return lat


@pytest.mark.parametrize("graph_steps", [0, -1])
@pytest.mark.parametrize("storage", ["f32", "f64", "f16s", "bf16s", "f32d", "f32s"])
@pytest.mark.parametrize("nx,ny,tau,kw", GRIDS)
def test_two_step_launch_equals_one_step_launches(nx, ny, tau, kw, storage, graph_steps):
    calls = [1, 2, 77, 3] if kw.get("eos") == 1 else [1, 2, 77, 150, 3]  # the PR plug diverges after ~200 steps
    one = run(nx, ny, tau, kw, storage, 1, graph_steps, calls)
    two = run(nx, ny, tau, kw, storage, 2, graph_steps, calls)
    assert one.steps == two.steps == sum(calls)
    assert np.array_equal(one.get_f(), two.get_f())
    for x, y in zip(one.fields(), two.fields()):
        assert np.array_equal(x, y)
    if not kw.get("y_periodic"):
        assert repr(one.history()) == repr(two.history())
        w1, w2 = one.wall()[0], two.wall()[0]
        for key in w1:
            assert np.array_equal(w1[key], w2[key]), key
    assert repr(one.check()) == repr(two.check())
