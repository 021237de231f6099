"""C-ABI boundary checks that need no GPU: the library loads, exports every
function include/ptyr.h declares, and its pure-host validators return the
documented status codes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2505_07814_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name="ptyr.h"):
    src = open(os.path.join(ROOT, "include", name)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ptyr_[a-z_]+)\s*\(", src)))


def geom(**kw):
    d = dict(N=128, M=6, S=12, H=640, W=640, B_max=64, dx=0.15, lam=0.0197, loss_kind=0, loss_p=0.5,
             wave_budget_bytes=64 * 6 * 24 * 128 * 128 * 8, flags=0, n_scan=16384, sparse_w=0.0, pacbed_w=0.0,
             n_obj=0, w_gaussian=0.0, w_poisson=0.0, p_gaussian=0.0, p_poisson=0.0)
    d.update(kw)
    return L.Geom(*[d[f[0]] for f in L.Geom._fields_])


def test_library_exports_every_header_function():
    lib = L.lib()
    names = header_functions()
    assert set(names) == set(L.HEADER_SYMBOLS), names
    cnn = header_functions("ptyr_cnn.h")
    assert set(cnn) == set(L.CNN_HEADER_SYMBOLS), cnn
    for n in names + cnn:
        assert hasattr(lib, n), n


def test_status_strings():
    lib = L.lib()
    for s in range(6):
        assert lib.ptyr_status_str(s)
    assert b"leaves" in lib.ptyr_status_str(L.PTYR_E_BOUNDS)


@pytest.mark.parametrize("kw,expect", [
    ({}, L.PTYR_OK),
    (dict(N=64, H=128, W=128), L.PTYR_OK),
    (dict(N=96), L.PTYR_E_ARG),
    (dict(N=256, H=1024, W=1024, B_max=16, M=8, S=30, wave_budget_bytes=16 * 8 * 60 * 256 * 256 * 8), L.PTYR_OK),
    (dict(N=256, H=1024, W=1024, B_max=16, M=8, S=30, wave_budget_bytes=0), L.PTYR_E_ARG),
    (dict(M=0), L.PTYR_E_ARG),
    (dict(S=0), L.PTYR_E_ARG),
    (dict(B_max=0), L.PTYR_E_ARG),
    (dict(H=100), L.PTYR_E_ARG),
    (dict(dx=0.0), L.PTYR_E_ARG),
    (dict(lam=-1.0), L.PTYR_E_ARG),
    (dict(loss_kind=7), L.PTYR_E_ARG),
    (dict(loss_p=0.0), L.PTYR_E_ARG),
    (dict(flags=0x80), L.PTYR_E_ARG),
    (dict(n_obj=2), L.PTYR_OK),
    (dict(n_obj=-1), L.PTYR_E_ARG),
    (dict(n_obj=65), L.PTYR_E_ARG),
    (dict(n_scan=-1), L.PTYR_E_ARG),
    (dict(w_gaussian=0.5, w_poisson=0.5), L.PTYR_OK),
    (dict(w_gaussian=0.5, p_gaussian=1.0), L.PTYR_OK),
    (dict(w_gaussian=-0.5), L.PTYR_E_ARG),
    (dict(w_poisson=float("nan")), L.PTYR_E_ARG),
    (dict(p_poisson=-1.0), L.PTYR_E_ARG),
    (dict(p_gaussian=float("inf")), L.PTYR_E_ARG),
])
def test_check_geom(kw, expect):
    g = geom(**kw)
    assert L.lib().ptyr_check_geom(C.byref(g)) == expect


def test_check_args_positions():
    lib = L.lib()
    g = geom(N=64, H=128, W=128, B_max=4)
    ok = (C.c_float * 4)(64.0, 64.0, 32.0, 96.0)
    assert lib.ptyr_check_args(C.byref(g), 2, ok) == L.PTYR_OK
    assert lib.ptyr_check_args(C.byref(g), 0, ok) == L.PTYR_E_ARG
    assert lib.ptyr_check_args(C.byref(g), 5, None) == L.PTYR_E_ARG
    for bad in [(31.4, 64.0), (64.0, 96.6), (float("nan"), 64.0), (1e30, 64.0)]:
        arr = (C.c_float * 2)(*bad)
        assert lib.ptyr_check_args(C.byref(g), 1, arr) == L.PTYR_E_BOUNDS, bad
    # round half to even: 31.5 -> 32 (corner 0) is inside, 96.5 -> 96 (corner 64) is inside
    edge = (C.c_float * 2)(31.5, 96.5)
    assert lib.ptyr_check_args(C.byref(g), 1, edge) == L.PTYR_OK


def test_workspace_and_checkpoint_plan():
    lib = L.lib()
    full = geom()
    k = C.c_int()
    assert lib.ptyr_checkpoint_plan(C.byref(full), C.byref(k)) == L.PTYR_OK and k.value == 1
    none = geom(wave_budget_bytes=0)
    assert lib.ptyr_checkpoint_plan(C.byref(none), C.byref(k)) == L.PTYR_OK and k.value == 13
    per = 64 * 6 * 128 * 128 * 8
    third = geom(wave_budget_bytes=(3 + 4) * per)     # scratch + 4 checkpoints of 12 slices -> stride 3
    assert lib.ptyr_checkpoint_plan(C.byref(third), C.byref(k)) == L.PTYR_OK and k.value == 3
    almost = geom(wave_budget_bytes=(2 * 12 - 1) * per)   # one wave short of keeping everything
    assert lib.ptyr_checkpoint_plan(C.byref(almost), C.byref(k)) == L.PTYR_OK and k.value == 2
    scratch_only = geom(wave_budget_bytes=3 * per)
    assert lib.ptyr_checkpoint_plan(C.byref(scratch_only), C.byref(k)) == L.PTYR_OK and k.value == 13
    assert lib.ptyr_workspace_bytes(C.byref(full)) > lib.ptyr_workspace_bytes(C.byref(none))
    assert lib.ptyr_workspace_bytes(C.byref(geom(N=96))) == 0


def test_create_rejects_small_workspace_without_device_work():
    lib = L.lib()
    g = geom()
    ctx = C.c_void_p()
    n = lib.ptyr_workspace_bytes(C.byref(g))
    assert lib.ptyr_create(C.byref(g), C.c_void_p(256), n - 1, None, C.byref(ctx)) == L.PTYR_E_NOMEM
    assert lib.ptyr_create(C.byref(g), None, n, None, C.byref(ctx)) == L.PTYR_E_ARG


# ---------------------------------------------------------------- learned initial guess
def test_cnn_param_count_and_layout():
    from paper_2505_07814_amd import cnn
    n = L.lib().ptyr_cnn_param_count()
    # per layer Cout_p * K_p + Cout_p: 32*160+32, 3 x (32*288+32), 16*288+16
    assert n == 5152 + 3 * 9248 + 4624
    rng = np.random.default_rng(0)
    layers = [(rng.standard_normal((co, ci, 3, 3)), rng.standard_normal(co))
              for ci, co in zip(cnn.CHANNELS[:-1], cnn.CHANNELS[1:])]
    v = cnn.pack_params(layers)
    assert v.shape == (n,)
    back = cnn.unpack_params(v)
    for (W, b), (W2, b2) in zip(layers, back):
        np.testing.assert_allclose(W2, W.astype(np.float32), rtol=0, atol=0)
        np.testing.assert_allclose(b2, b.astype(np.float32), rtol=0, atol=0)
    # W[o, c, u, v] sits at layer offset + o * K_p + (3u + v) * Cin_p + c
    assert v[1 * 160 + (3 * 2 + 1) * 16 + 5] == np.float32(layers[0][0][1, 5, 2, 1])
    off2 = 5152 + 9248
    assert v[off2 + 7 * 288 + (3 * 1 + 0) * 32 + 31] == np.float32(layers[2][0][7, 31, 1, 0])
    assert np.count_nonzero(v) == sum(W.size + b.size for W, b in layers)


def test_cnn_workspace_and_create_errors():
    lib = L.lib()
    assert lib.ptyr_cnn_workspace_bytes(0) == 0
    a, b = lib.ptyr_cnn_workspace_bytes(1), lib.ptyr_cnn_workspace_bytes(256)
    assert 0 < a < b
    ctx = C.c_void_p()
    assert lib.ptyr_cnn_create(0, C.c_void_p(256), 1 << 30, None, C.byref(ctx)) == L.PTYR_E_ARG
    assert lib.ptyr_cnn_create(4, None, 1 << 30, None, C.byref(ctx)) == L.PTYR_E_ARG
    assert lib.ptyr_cnn_create(4, C.c_void_p(256), lib.ptyr_cnn_workspace_bytes(4) - 1, None,
                               C.byref(ctx)) == L.PTYR_E_NOMEM
    assert lib.ptyr_cnn_create(4, C.c_void_p(256), 1 << 30, None, None) == L.PTYR_E_ARG
    assert lib.ptyr_cnn_forward(None, None, None, 1, None, 1, None) == L.PTYR_E_ARG
    assert lib.ptyr_cnn_sync(None) == L.PTYR_E_ARG


def test_constrain_rejects_a_null_context():
    from paper_2505_07814_amd import _lib as L
    import ctypes as C
    cfg = L.Constraints(1.0, 1, 0)
    assert L.lib().ptyr_constrain(None, None, None, None, C.byref(cfg)) == L.PTYR_E_ARG
    assert L.lib().ptyr_constrain(None, None, None, None, None) == L.PTYR_E_ARG
