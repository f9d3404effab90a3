"""Host-only checks of the C ABI library (no GPU needed, no kernel launched).

The library loads, exports every entry point declared in include/lbm.h,
validates parameters on the host, and its own (independent) EOS/Maxwell solver
agrees with the oracle's.
"""
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2103_08301_amd import lbm

    if not os.path.exists(lbm.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    lbm.library()
    return lbm


def declared_functions():
    with open(os.path.join(ROOT, "include", "lbm.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:lbm_status|void|const char\*)\s+(lbm_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 15
    lib = L.library()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTED) == names


def test_struct_layouts_match_header(L, tmp_path):
    """sizeof/offsetof of the three structs, as gcc computes them from lbm.h,
    against the ctypes mirrors of the binding."""
    import ctypes as C
    import subprocess

    structs = {"lbm_params": L.lbm_params, "lbm_stress_summary": L.lbm_stress_summary,
               "lbm_check_result": L.lbm_check_result, "lbm_component": L.lbm_component,
               "lbm_aerosol_summary": L.lbm_aerosol_summary}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                          check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(out[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset, f"{name}.{f}"


def test_defaults(L):
    p = L.lbm_params_default()
    assert (p.eos, p.a, p.b, p.R, p.T_over_Tc, p.k, p.kappa) == (0, 1.0, 4.0, 1.0, 0.85, 1.0, 0.001)
    assert (p.s_e, p.s_eps, p.s_q) == (1.64, 1.54, 1.7)
    assert math.isnan(p.rho_wall) and p.storage == L.LBM_F32 and p.check_every == 1000


@pytest.mark.parametrize("bad", [
    dict(T_over_Tc=0.0), dict(a=-1.0), dict(b=0.0), dict(k=0.0), dict(kappa=-1.0), dict(s_e=2.0),
    dict(s_q=0.0), dict(check_every=0), dict(v_limit=0.0), dict(history_cap=0), dict(storage=8),
    dict(eos=3), dict(x_periodic=2), dict(rho_wall=-1.0), dict(dp=math.inf), dict(tile_waves=6),
    dict(tile_waves=8, tile_rows=8), dict(schedule=0, tile_rows=16), dict(schedule=3), dict(schedule=2, tile_rows=20),
    dict(schedule=2, tile_waves=8, tile_rows=12), dict(schedule=2, pipe_blocks=4), dict(pipe_blocks=64),
    dict(schedule=1, tile_waves=4), dict(storage=6, schedule=1), dict(storage=6, tile_rows=8),
    dict(storage=6, tile_waves=4), dict(graph_steps=3), dict(graph_steps=512), dict(graph_steps=-2),
    dict(fused_steps=3), dict(fused_steps=-1),
])
def test_create_rejects_invalid_parameters(L, bad):
    with pytest.raises(L.LbmError) as e:
        L.lbm_create(64, 32, 1.0, L.lbm_params_default(**bad))
    assert e.value.status == L.LBM_EINVAL


@pytest.mark.parametrize("nx,ny,tau", [(3, 32, 1.0), (64, 3, 1.0), (64, 32, 0.5), (64, 32, 0.2)])
def test_create_rejects_invalid_grid(L, nx, ny, tau):
    with pytest.raises(L.LbmError):
        L.lbm_create(nx, ny, tau, L.lbm_params_default())


def test_calls_before_bind_are_rejected(L):
    ctx = L.lbm_create(64, 32, 1.0, L.lbm_params_default())
    with pytest.raises(L.LbmError) as e:
        L.lbm_init_plug(ctx, 10, 2)
    assert e.value.status == L.LBM_ESTATE
    assert L.library().lbm_step(ctx, 1) == L.LBM_ESTATE
    assert L.lbm_workspace(ctx) > 2 * 9 * 64 * 32 * 4
    assert L.lbm_workspace(ctx, with_align=True)[1] == 256
    import ctypes as C

    n = C.c_size_t()
    assert L.library().lbm_workspace(ctx, C.byref(n), None) == L.LBM_OK and n.value > 0  # align may be NULL
    L.lbm_destroy(ctx)


@pytest.mark.parametrize("kw,trs", [
    ({}, [0.95, 0.85, 0.8, 0.7, 0.5]),
    (dict(eos=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344), [0.9, 0.7, 0.6, 0.5]),
    (dict(eos=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.011), [0.8, 0.6]),
])
def test_library_coexistence_agrees_with_oracle(L, orc, kw, trs):
    """Two independent solvers: the oracle bisects the equal-area integral
    (Gauss-Legendre), the library bisects the chemical-potential difference
    (Romberg) with hyper-dual derivatives."""
    for tr in trs:
        a = L.lbm_state(L.lbm_create(32, 16, 1.0, L.lbm_params_default(T_over_Tc=tr, **kw)))
        b = orc.Sim(32, 16, orc.params(T_over_Tc=tr, **kw)).state()
        for k in ("Tc", "T", "rho_g", "rho_l", "rho_w"):
            assert a[k] == pytest.approx(b[k], rel=1e-11), (tr, k)


def test_batch_create_validates_cases(L):
    import ctypes as C

    def create(plist, sizes=((64, 32), (96, 40))):
        n = len(plist)
        nx = (C.c_int * n)(*[s[0] for s in sizes[:n]])
        ny = (C.c_int * n)(*[s[1] for s in sizes[:n]])
        tau = (C.c_double * n)(*([1.0] * n))
        params = (L.lbm_params * n)(*plist)
        b = L._P()
        st = L.library().lbm_batch_create(n, nx, ny, tau, params, C.byref(b))
        return st, b

    p = L.lbm_params_default
    st, b = create([p(), p(dp=2e-3, T_over_Tc=0.9)])
    assert st == L.LBM_OK
    size = C.c_size_t()
    assert L.library().lbm_batch_workspace(b, C.byref(size)) == L.LBM_OK and size.value > 0
    L.library().lbm_batch_destroy(b)
    for bad in ([p(), p(storage=L.LBM_F64)], [p(), p(eos=L.LBM_EOS_PR, a=2 / 49, b=2 / 21)], [p(), p(tile_rows=12)],
                [p(), p(check_every=10)], [p(), p(schedule=1)], [p(), p(T_over_Tc=-1.0)]):
        st, _ = create(bad)
        assert st == L.LBM_EINVAL


def test_adjoint_workspace_layout_and_rules(L):
    """Host-side arithmetic of the adjoint workspace (no device needed): ceil(N/S) checkpoints, the recompute's two
    states, two segments of S steps of forward fields (five planes and four wall rows of the arithmetic type), of
    wall shears and of peak-objective seeds, two adjoint fields, the per-launch partials and the FP64 state
    gradient."""
    def align(v):
        return (v + 255) // 256 * 256

    nx, ny = 200, 40
    pitch = (nx + 63) // 64 * 64
    for storage, sb, ab in (("f32", 4, 4), ("f64", 8, 8), ("f32d", 4, 8)):
        ctx = L.lbm_create(nx, ny, 1.0, L.lbm_params_default(storage=storage))
        for n, seg in ((1000, 0), (1000, 10), (7, 7), (1, 1)):
            s = seg or math.ceil(math.sqrt(n))
            k = (n + s - 1) // s
            ty = 4  # adjoint tile rows below 1M nodes
            blocks = ((nx + 59) // 60) * ((ny + ty - 1) // ty)
            ring = max(s, 64)
            want = (k * align(pitch * ny * 9 * sb) + 2 * align(pitch * ny * 9 * sb)
                    + 2 * s * align((5 * pitch * ny + 4 * nx) * ab) + 2 * align(pitch * ny * 9 * ab)
                    + 2 * align(2 * s * 2 * nx * 8) + align(ring * blocks * 4 * 8) + align(ring * 4 * 8) + 256
                    + align(4 * nx * 8) + align(9 * nx * ny * 8))
            assert L.lbm_adjoint_workspace(ctx, n, seg) == want, (storage, n, seg)
        for n, seg in ((0, 0), (10, 11), (10, -1)):
            with pytest.raises(L.LbmError):
                L.lbm_adjoint_workspace(ctx, n, seg)
        L.lbm_destroy(ctx)
    for bad in (dict(storage="f16s"), dict(storage="bf16s"), dict(storage="f64t"), dict(storage="f16r"),
                dict(schedule=1), dict(schedule=2)):
        ctx = L.lbm_create(nx, ny, 1.0, L.lbm_params_default(**bad))
        with pytest.raises(L.LbmError):
            L.lbm_adjoint_workspace(ctx, 100, 0)
        L.lbm_destroy(ctx)


def test_calls_before_binding_the_adjoint_are_rejected(L):
    import ctypes as C

    ctx = L.lbm_create(64, 32, 1.0, L.lbm_params_default(storage="f64"))
    J = C.c_double()
    g = (C.c_double * 4)()
    assert L.library().lbm_adjoint_forward(ctx, C.byref(J)) == L.LBM_ESTATE
    assert L.library().lbm_adjoint_backward(ctx, 1.0, g) == L.LBM_ESTATE
    assert L.library().lbm_adjoint_state_gradient(ctx, g) == L.LBM_ESTATE
    assert L.library().lbm_autotune(ctx, 10, None, None, None) == L.LBM_ESTATE
    assert L.library().lbm_adjoint_backward(ctx, math.nan, g) == L.LBM_EINVAL
    assert L.library().lbm_adjoint_objective(ctx, 1) == L.LBM_ESTATE  # before lbm_adjoint_bind
    assert L.library().lbm_adjoint_objective(ctx, 2) == L.LBM_EINVAL  # no such objective
    assert L.library().lbm_adjoint_objective(None, 0) == L.LBM_EINVAL
    L.lbm_destroy(ctx)


def test_stochastic_fp16_storage_rules(L):
    """F16R runs on the tile schedule with one step per launch; other schedules and two-step launches are refused."""
    ctx = L.lbm_create(64, 16, 1.0, L.lbm_params_default(storage="f16r"))
    assert L.lbm_workspace(ctx) > 2 * 9 * 64 * 16 * 2
    L.lbm_destroy(ctx)
    for bad in (dict(schedule=1), dict(schedule=2), dict(fused_steps=2)):
        with pytest.raises(L.LbmError):
            L.lbm_create(64, 16, 1.0, L.lbm_params_default(storage="f16r", **bad))


def test_checkpoint_and_device_fields_need_a_bound_lattice(L, tmp_path):
    """lbm_save, lbm_load and lbm_fields_device before binding or initialisation: LBM_ESTATE, no device access."""
    ctx = L.lbm_create(64, 16, 1.0, L.lbm_params_default())
    lib = L.library()
    path = str(tmp_path / "x.ckpt").encode()
    assert lib.lbm_save(ctx, path) == L.LBM_ESTATE
    assert lib.lbm_load(ctx, path) == L.LBM_ESTATE
    assert lib.lbm_fields_device(ctx, None, None, None, 1) == L.LBM_ESTATE
    assert lib.lbm_save(None, path) == L.LBM_EINVAL
    assert not (tmp_path / "x.ckpt").exists()
    L.lbm_destroy(ctx)


def test_launch_config_reports_the_parameters(L):
    """lbm_launch_config reads the host-side launch configuration (no device needed)."""
    lib = L.library()
    for kw, want in ((dict(), (8, 4, 1, 64)), (dict(storage="f64"), (12, 4, 1, 64)),
                     (dict(fused_steps=2, graph_steps=-1), (8, 4, 2, 0)), (dict(tile_waves=8), (12, 8, 1, 64)),
                     (dict(graph_steps=256), (8, 4, 1, 256))):
        ctx = L.lbm_create(64, 16, 1.0, L.lbm_params_default(**kw))
        v = [L.C.c_int() for _ in range(4)]
        assert lib.lbm_launch_config(ctx, *(L.C.byref(x) for x in v)) == L.LBM_OK
        assert tuple(x.value for x in v) == want, kw
        L.lbm_destroy(ctx)


def test_bind_checks_the_workspace_before_any_launch(L):
    """lbm_bind checks the workspace pointer on the host: without a GPU the call reports
    LBM_EDEVICE, with one a host buffer is LBM_EINVAL; nothing is launched either way."""
    import ctypes as C

    import numpy as np

    ctx = L.lbm_create(64, 16, 1.0, L.lbm_params_default())
    try:
        need = L.lbm_workspace(ctx)
        buf = np.zeros(need + 256, dtype=np.uint8)
        p = (buf.ctypes.data + 255) // 256 * 256
        st = L.library().lbm_bind(ctx, C.c_void_p(p), need, None)
        assert st in (L.LBM_EDEVICE, L.LBM_EINVAL), st
        msg = L.library().lbm_last_error(ctx).decode()
        assert msg.startswith("workspace: ") and ("no current HIP device" in msg or "device memory" in msg), msg
        # a step after the refused bind is out of order, not a launch
        assert L.library().lbm_step(ctx, 1) == L.LBM_ESTATE
    finally:
        L.lbm_destroy(ctx)


def test_binding_fails_loudly_without_the_library():
    """With liblbm.so absent the binding raises on first use; there is no CPU fallback."""
    import subprocess
    import sys

    code = (
        "import paper_2103_08301_amd.lbm as L\n"
        "L.LIB_PATH = '/nonexistent/liblbm.so'\n"
        "L._lib = None\n"
        "try:\n"
        "    L.Lattice(32, 8, 1.0, device='cpu')\n"
        "except RuntimeError as e:\n"
        "    assert 'no CPU fallback' in str(e), e\n"
        "    print('raised')\n"
    )
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "raised", (out.stdout, out.stderr)
