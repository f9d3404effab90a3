"""Captured HIP graphs of the step loop against direct launches.

lbm_step (and lbm_batch_step) replay captured graphs of graph_steps step
launches instead of launching kernel by kernel.  The graphs are replayed many
times, with the library's own eager launches, flushes, checks and host
synchronisations between replays, from odd and even wall-ring offsets and both
buffer parities; every state, field, per-step wall summary and check must be
bit-identical to direct launches of the same steps.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2103_08301_amd import Batch, Lattice, lbm  # noqa: E402


def run(graph_steps, storage, schedule, tile_rows, calls):
    lat = Lattice(130, 37, 0.9, storage=storage, dp=2e-3, T_over_Tc=0.95, schedule=schedule, tile_rows=tile_rows,
                  graph_steps=graph_steps, check_every=97, v_limit=1.0)
    lat.init_plug(30, 3, math.nan, 1e-3, 11)
    for n in calls:
        assert lat.step(n) == 0
    return lat


CALLS = [1, 70, 3, 300, 129, 64, 65, 400]  # odd ring offsets, both parities, flushes and checks between replays


@pytest.mark.parametrize("storage,schedule,tile_rows", [("f64", 0, 12), ("f32", 0, 8), ("f32", 1, 16),
                                                        ("f16s", 0, 8), ("f16r", 0, 8)])
@pytest.mark.parametrize("graph_steps", [0, 16, 2, 256])
def test_graph_replays_equal_direct_launches(storage, schedule, tile_rows, graph_steps):
    ref = run(-1, storage, schedule, tile_rows, CALLS)
    got = run(graph_steps, storage, schedule, tile_rows, CALLS)
    assert got.steps == ref.steps == sum(CALLS)
    assert np.array_equal(got.get_f(), ref.get_f())
    for a, b in zip(got.fields(), ref.fields()):
        assert np.array_equal(a, b)
    hg, hr = got.history(), ref.history()
    assert len(hg) == len(hr) > 0
    assert repr(hg) == repr(hr)  # repr is exact for floats and equal for NaN
    assert repr(got.check()) == repr(ref.check())


def test_batch_graph_replays_equal_direct_launches():
    cases = [dict(nx=96 + 8 * k, ny=24 + 4 * k, tau=1.0, dp=1e-3 * (1 + k), T_over_Tc=0.9) for k in range(3)]

    def go(graph_steps):
        b = Batch(cases, storage="f32", check_every=90, graph_steps=graph_steps, v_limit=1.0)
        for k in range(3):
            b[k].init_plug(20, 2, math.nan, 1e-3, 5 + k)
        for n in (1, 130, 300, 77):
            assert b.step(n) == 0
        return [(b[k].get_f(), b[k].history(), b[k].check()) for k in range(3)]

    ref, got = go(-1), go(0)
    for (f1, h1, c1), (f2, h2, c2) in zip(ref, got):
        assert np.array_equal(f1, f2)
        assert repr(h1) == repr(h2) and repr(c1) == repr(c2)


def test_graph_steps_validation():
    with pytest.raises(lbm.LbmError):
        Lattice(64, 16, 1.0, graph_steps=3)
    with pytest.raises(lbm.LbmError):
        Lattice(64, 16, 1.0, graph_steps=512)
