"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and
rejects invalid arguments on the host before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2503_11731_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs2d.h")

need_lib = pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="libgs2d.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("gs_plan_create", "gs_render_forward", "gs_render_backward", "gs_decode_forward", "gs_decode_backward",
              "gs_query_status"):
        assert n in names
    assert set(names) == {s[0] for s in L.SIGNATURES}


@need_lib
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    lib = L.load()
    assert lib.gs_version().startswith(b"gs2d")
    assert lib.gs_status_string(2) == b"pair capacity exceeded"


def _desc(n=10, sensors=None, opts=None, scenes=None):
    off = (ctypes.c_int32 * 2)(0, n)
    sd = (L.SceneDesc * 1)(L.SceneDesc(n, -1, 0, 1, off))
    if sensors is None:
        sensors = [L.SensorDesc(0, 64, 48, 64.0, 64.0, 32.0, 24.0, None, 0.2, 0, 0, 0)]
    sa = (L.SensorDesc * len(sensors))(*sensors)
    o = opts or L.RenderOpts(1 / 255, 0.99, 1e-4, 11.08, 2.0, 1, (ctypes.c_float * 3)(0, 0, 0))
    d = L.PlanDesc(1 if scenes is None else scenes, sd, len(sensors), sa, o, 0, 0)
    return d, (off, sd, sa)


@need_lib
@pytest.mark.parametrize("case", ["null", "bad_focal", "bad_opts", "bad_tile", "no_scene", "lidar_no_elev",
                                  "bad_groups"])
def test_plan_create_rejects_invalid_arguments(case):
    lib = L.load()
    plan = ctypes.c_void_p()
    if case == "null":
        rc = lib.gs_plan_create(None, ctypes.byref(plan))
        assert rc == L.GS_ERR_INVALID_ARG
        return
    if case == "bad_focal":
        d, keep = _desc(sensors=[L.SensorDesc(0, 64, 48, 0.0, 64.0, 32.0, 24.0, None, 0.2, 0, 0, 0)])
    elif case == "bad_opts":
        d, keep = _desc(opts=L.RenderOpts(0, 1.5, 0, 11.0, 2.0, 1, (ctypes.c_float * 3)(0, 0, 0)))
    elif case == "bad_tile":
        d, keep = _desc(sensors=[L.SensorDesc(0, 64, 48, 64.0, 64.0, 32.0, 24.0, None, 0.2, 0, 12, 12)])
    elif case == "no_scene":
        d, keep = _desc(scenes=0)
    elif case == "lidar_no_elev":
        d, keep = _desc(sensors=[L.SensorDesc(1, 360, 16, 0, 0, 0, 0, None, 0.5, 0, 0, 0)])
    elif case == "bad_groups":
        d, keep = _desc()
        keep[0][1] = 5  # group offsets end != N
    rc = lib.gs_plan_create(ctypes.byref(d), ctypes.byref(plan))
    assert rc in (L.GS_ERR_INVALID_ARG, L.GS_ERR_UNSUPPORTED), rc
    buf = ctypes.create_string_buffer(256)
    assert lib.gs_last_error(buf, 256) == rc
    assert len(buf.value) > 0
    assert not plan.value


@need_lib
def test_valid_plan_and_workspace_size_without_gpu():
    lib = L.load()
    d, keep = _desc(n=1000)
    plan = ctypes.c_void_p()
    rc = lib.gs_plan_create(ctypes.byref(d), ctypes.byref(plan))
    assert rc == L.GS_OK
    nb = ctypes.c_size_t()
    assert lib.gs_plan_workspace_size(plan, ctypes.byref(nb)) == L.GS_OK
    assert nb.value > 1000 * 64
    v = L.WorkspaceView()
    assert lib.gs_plan_inspect(plan, 0, ctypes.byref(v)) == L.GS_OK
    assert v.n_tiles == 4 * 3
    assert lib.gs_plan_inspect(plan, 3, ctypes.byref(v)) == L.GS_ERR_INVALID_ARG
    # forward with null arguments fails on the host before touching the device
    assert lib.gs_render_forward(plan, None, None, None, None, None, None) == L.GS_ERR_INVALID_ARG
    lib.gs_plan_destroy(plan)


@need_lib
def test_decode_rejects_invalid_arguments():
    lib = L.load()
    off = (ctypes.c_int32 * 2)(0, 5)
    an = L.AnchorSet(5, 0, 0, 1, off, 0, 0, 0, 0, 0, 0, 0, 0, 0)  # k = 0
    assert lib.gs_decode_forward(ctypes.byref(an), None, None, None, None) == L.GS_ERR_INVALID_ARG
    an = L.AnchorSet(5, 10, 0, 1, off, 0, 0, 0, 0, 0, 0, 0, 0, 0)
    one = ctypes.c_float(0)
    assert lib.gs_decode_forward(ctypes.byref(an), ctypes.addressof(one), ctypes.addressof(one), None,
                                 None) == L.GS_ERR_INVALID_ARG


@need_lib
def test_noalloc_decode_backward_checks_arguments_and_size_before_any_device_call():
    # Host-side checks run before the library touches the device: a bad
    # shape, null gradients, and anchor sets whose weight-gradient partials
    # exceed the per-GPU array (the fake device addresses are never read).
    lib = L.load()
    off = (ctypes.c_int32 * 2)(0, 5)
    an = L.AnchorSet(5, 0, 0, 1, off, 0, 0, 0, 0, 0, 0, 0, 0, 0)  # k = 0
    one = ctypes.c_float(0)
    p1 = ctypes.addressof(one)
    assert lib.gs_decode_backward_noalloc(ctypes.byref(an), p1, p1, None, None, None) == L.GS_ERR_INVALID_ARG
    fake = 1 << 20
    A = 2000 * 64
    big = (ctypes.c_int32 * 2)(0, A)
    an = L.AnchorSet(A, 10, 0, 1, big, fake, fake, fake, fake, fake, fake, fake, fake, 0)
    nb = ctypes.c_size_t()
    assert lib.gs_decode_scratch_size(ctypes.byref(an), ctypes.byref(nb)) == L.GS_OK
    assert nb.value == 2000 * 4 * (10 * 10 * 33 + 32 * 36) > L.GS_DECODE_NOALLOC_SCRATCH_BYTES
    d = L.Decoded(fake, fake, fake, fake, fake, None)
    assert lib.gs_decode_backward_noalloc(ctypes.byref(an), p1, p1, ctypes.byref(d), None,
                                          None) == L.GS_ERR_INVALID_ARG
    g = L.AnchorGrads(None, None, None, None, None, None, fake, None)  # dW2 requested
    assert lib.gs_decode_backward_noalloc(ctypes.byref(an), p1, p1, ctypes.byref(d), ctypes.byref(g),
                                          None) == L.GS_ERR_INVALID_ARG
    buf = ctypes.create_string_buffer(256)
    lib.gs_last_error(buf, 256)
    assert b"scratch" in buf.value


@need_lib
def test_affinity_rejects_invalid_arguments_and_launches_nothing_for_empty_sizes():
    lib = L.load()
    buf = (ctypes.c_uint16 * 64)()
    p = ctypes.addressof(buf)
    assert lib.gs_affinity(None, None, -1, 4, 4, 64, None, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_affinity(None, None, 1, 4, 4, 48, None, None) == L.GS_ERR_INVALID_ARG    # d not a multiple of 32
    assert lib.gs_affinity(None, None, 1, 4, 4, 288, None, None) == L.GS_ERR_INVALID_ARG   # d above 256
    assert lib.gs_affinity(None, None, 70000, 4, 4, 64, None, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_affinity(None, None, 1, 4, 4, 64, None, None) == L.GS_ERR_INVALID_ARG    # null buffers
    assert lib.gs_affinity(p + 2, p, 1, 4, 4, 64, p, None) == L.GS_ERR_INVALID_ARG         # misaligned rows
    assert lib.gs_affinity(None, None, 0, 4, 4, 64, None, None) == 0                       # nothing to do
    assert lib.gs_affinity(None, None, 3, 4, 0, 64, None, None) == 0
