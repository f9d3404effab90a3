"""Checkpoint and resume (lbm_save / lbm_load) and the device copy of the fields.

A run split by a save and a load into a new context must continue bit for bit
as the uninterrupted run: distributions, fields, checks, wall arrays and the
per-step summaries (time integrals and running extremes included) of the
steps after the load.  Covered for FP64, FP32, FP16 with stochastic rounding
(its step counter travels in the file) and the tangent-linear storage (its
tangent direction too).  Files of another lattice, with other parameters,
truncated or with a flipped byte are refused.
"""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2103_08301_amd import Lattice, lbm  # noqa: E402

KW = dict(T_over_Tc=0.9, dp=2e-3, check_every=100, v_limit=1.0)


def make(storage, nx=150, ny=40, **kw):
    lat = Lattice(nx, ny, 0.9, storage=storage, **dict(KW, **kw))
    if storage == "f64t":
        lat.set_tangent(1.0, 0.0, 0.0, 0.5)
    return lat


@pytest.mark.parametrize("storage", ["f64", "f32", "f16r", "f64t"])
def test_resume_continues_bit_for_bit(tmp_path, storage):
    path = str(tmp_path / "run.ckpt")
    a = make(storage)
    a.init_plug(36, 4, math.nan, 1e-3, 3)
    assert a.step(301) == 0  # odd: the saved state sits in the second buffer
    a.save(path)
    saved_check = a.check()
    assert a.step(250) == 0

    b = make(storage)
    b.load(path)
    assert b.steps == 301
    assert repr(b.check()) == repr(saved_check)
    assert b.history() == []  # the history restarts with the next step
    assert b.step(250) == 0
    assert b.steps == a.steps == 551
    assert np.array_equal(b.get_f(), a.get_f())
    if storage == "f64t":
        assert np.array_equal(b.get_f_tangent(), a.get_f_tangent())
    for x, y in zip(b.fields(), a.fields()):
        assert np.array_equal(x, y)
    assert repr(b.check()) == repr(a.check())
    wb, sb = b.wall()
    wa, sa = a.wall()
    for k in wa:
        assert np.array_equal(wb[k], wa[k]), k
    assert repr(sb) == repr(sa)
    hb, ha = b.history(), a.history()
    assert len(hb) == 250
    assert repr(hb) == repr(ha[-250:])


def test_load_refuses_other_lattices_and_damaged_files(tmp_path):
    path = str(tmp_path / "run.ckpt")
    a = make("f32")
    a.init_plug(36, 4, math.nan, 1e-3, 3)
    a.step(10)
    a.save(path)
    for other in (make("f32", nx=151), make("f32", dp=3e-3), make("f64"), make("f32", x_periodic=1)):
        with pytest.raises(lbm.LbmError) as e:
            other.load(path)
        assert e.value.status == lbm.LBM_EINVAL
    raw = open(path, "rb").read()
    bad = str(tmp_path / "bad.ckpt")
    for damaged in (raw[:-9], raw[:100], bytearray(raw[:400]) + bytes([raw[400] ^ 1]) + raw[401:]):
        open(bad, "wb").write(bytes(damaged))
        with pytest.raises(lbm.LbmError):
            make("f32").load(bad)
    with pytest.raises(lbm.LbmError):
        make("f32").load(str(tmp_path / "missing.ckpt"))
    ok = make("f32")
    ok.load(path)  # the intact file still loads
    assert ok.steps == 10 and os.path.getsize(path) == len(raw)


def test_file_layout(tmp_path):
    """The documented layout: magic, header (nx, ny, tau, ... steps), the distributions, the FP64 fields, and an
    FNV-1a 64-bit hash of all preceding bytes."""
    path = str(tmp_path / "run.ckpt")
    a = make("f64", nx=70, ny=20)
    a.init_plug(20, 2, math.nan, 1e-3, 4)
    a.step(13)
    a.save(path)
    raw = open(path, "rb").read()
    assert raw[:8] == b"LBMCKPT1"
    nx, ny = np.frombuffer(raw[8:16], dtype=np.int32)
    tau = np.frombuffer(raw[16:24], dtype=np.float64)[0]
    assert (nx, ny, tau) == (70, 20, 0.9)
    h = 0xCBF29CE484222325
    for b in raw[:-8]:
        h = ((h ^ b) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    assert int.from_bytes(raw[-8:], "little") == h
    pitch = 128
    f_bytes = 9 * ny * pitch * 8
    rho = np.frombuffer(raw[-8 - 3 * nx * ny * 8:-8 - 2 * nx * ny * 8], dtype=np.float64).reshape(ny, nx)
    assert np.array_equal(rho, a.fields()[0])
    f = np.frombuffer(raw[-8 - 3 * nx * ny * 8 - f_bytes:-8 - 3 * nx * ny * 8], dtype=np.float64)
    assert np.array_equal(f.reshape(9, ny, pitch)[:, :, :nx], a.get_f())


def test_fields_device_equal_host_fields():
    a = make("f32")
    a.init_plug(36, 4, math.nan, 1e-3, 3)
    a.step(57)
    host = a.fields()
    dev64 = a.fields_device()
    dev32 = a.fields_device(torch.float32)
    torch.cuda.synchronize()
    for h, d64, d32 in zip(host, dev64, dev32):
        assert d64.dtype == torch.float64 and d64.shape == (40, 150) and d64.device.type == "cuda"
        assert np.array_equal(d64.cpu().numpy(), h)
        assert np.array_equal(d32.cpu().numpy(), h.astype(np.float32))


def test_fields_device_refuses_host_outputs():
    a = make("f32")
    a.init_plug(36, 4, math.nan, 1e-3, 3)
    a.step(5)
    dev = torch.empty((40, 150), dtype=torch.float64, device="cuda")
    host = torch.empty((40, 150), dtype=torch.float64)
    pinned = torch.empty((40, 150), dtype=torch.float64, pin_memory=True)
    for bad in (host, pinned):
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_fields_device(a.ctx, dev.data_ptr(), bad.data_ptr(), 0, True)
        assert e.value.status == lbm.LBM_EINVAL and "device memory" in str(e.value), str(e.value)
    # (whether a device buffer that is too short is caught depends on what lies after it,
    # so the remaining case tested is a misaligned output)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_fields_device(a.ctx, dev.data_ptr() + 4, 0, 0, True)
    assert e.value.status == lbm.LBM_EINVAL and "aligned" in str(e.value)
    # nothing was copied, and the calls that follow still work
    assert a.step(5) == lbm.LBM_OK
    rho = a.fields_device()[0]
    torch.cuda.synchronize()
    assert np.array_equal(rho.cpu().numpy(), a.fields()[0])
