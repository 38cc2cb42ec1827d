"""The C ABI library loads, exports every entry point include/mb3dgs.h
declares, and rejects bad arguments on the host (no device work)."""
import ctypes
import os
import re

import pytest

from paper_2512_11800_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(mb_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = L.load()
    declared = _declared()
    assert {"mb_prepare", "mb_render_forward", "mb_render_backward"} <= declared
    for name in sorted(declared):
        assert hasattr(lib, name), name
    # and the binding declares each of them
    assert declared <= {n for n, _, _ in L.SIGNATURES}


def test_defaults_and_version():
    lib = L.load()
    o = L.MbOptions()
    lib.mb_default_options(ctypes.byref(o))
    assert (o.n_moments, o.n_intervals) == (4, 3)
    assert o.kappa == pytest.approx(3.0) and o.conf_c == pytest.approx(0.01)
    assert o.beta == pytest.approx(0.25) and o.eps == pytest.approx(1e-6)
    assert lib.mb_version() >= 1


def test_workspace_sizes_grow_and_reject_bad_sizes():
    lib = L.load()
    a = lib.mb_gauss_workspace_bytes(1000, 1)
    b = lib.mb_gauss_workspace_bytes(2000, 1)
    c = lib.mb_gauss_workspace_bytes(2000, 2)
    assert 0 < a < b < c
    assert lib.mb_gauss_workspace_bytes(-1, 1) == 0
    p0 = lib.mb_pair_workspace_bytes(0, 1, 128, 128)
    p1 = lib.mb_pair_workspace_bytes(10_000, 1, 128, 128)
    assert 0 < p0 < p1
    assert lib.mb_pair_workspace_bytes(-5, 1, 128, 128) == 0


@pytest.mark.parametrize("n_cams,width,height", [(1, 128, 128), (3, 1920, 1080), (2, 100, 75)])
def test_pair_capacity_inverts_the_pair_size(n_cams, width, height):
    """mb_pair_capacity(B) is the largest E with mb_pair_workspace_bytes(E) <= B
    (the layout a device-count render uses), -1 when even an empty list does
    not fit or an argument is bad."""
    lib = L.load()
    size = lambda e: int(lib.mb_pair_workspace_bytes(e, n_cams, width, height))
    base = size(0)
    assert lib.mb_pair_capacity(base - 1, n_cams, width, height) == -1
    assert lib.mb_pair_capacity(base, n_cams, width, height) >= 0
    for e in (0, 1, 2047, 2048, 2049, 123_457, 1_000_000, 5_000_000):
        for nbytes in (size(e), size(e) + 1, size(e + 1) - 1):
            cap = int(lib.mb_pair_capacity(nbytes, n_cams, width, height))
            assert size(cap) <= nbytes < size(cap + 1), (e, nbytes, cap)
    assert lib.mb_pair_capacity(1 << 30, 0, width, height) == -1
    assert lib.mb_pair_capacity(1 << 30, n_cams, 0, height) == -1


def test_entry_count_rejects_bad_arguments_on_the_host():
    lib = L.load()
    n = ctypes.c_int64(0)
    assert lib.mb_entry_count(-1, 1, None, 0, ctypes.byref(n), None) == L.MB_ERR_ARG
    assert lib.mb_entry_count(10, 1, None, 0, None, None) == L.MB_ERR_ARG
    assert lib.mb_entry_count(10, 1, None, 0, ctypes.byref(n), None) == L.MB_ERR_WORKSPACE


def _cam(width=64, height=48):
    c = L.MbCamera()
    c.world_to_cam = (ctypes.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 3)
    c.fx = c.fy = 50.0
    c.cx, c.cy = width / 2, height / 2
    c.width, c.height = width, height
    c.t_near = 0.2
    return c


@pytest.mark.parametrize("field,value,code", [
    ("n_moments", 5, L.MB_ERR_UNSUPPORTED),
    ("n_intervals", 4, L.MB_ERR_UNSUPPORTED),
    ("conf_c", 1.5, L.MB_ERR_ARG),
    ("kappa", 0.5, L.MB_ERR_ARG),
    ("eps", 0.0, L.MB_ERR_ARG),
])
def test_bad_options_rejected_before_device_work(field, value, code):
    lib = L.load()
    o = L.MbOptions()
    lib.mb_default_options(ctypes.byref(o))
    setattr(o, field, value)
    g = L.MbGaussians(0, -1, None, None, None, None, None)
    cam = _cam()
    n = ctypes.c_int64(0)
    rc = lib.mb_prepare(ctypes.byref(g), ctypes.byref(cam), 1, ctypes.byref(o), None, 0,
                        ctypes.byref(n), None)
    assert rc == code
    assert lib.mb_last_error()


def test_bad_cameras_and_pointers_rejected():
    lib = L.load()
    o = L.MbOptions()
    lib.mb_default_options(ctypes.byref(o))
    n = ctypes.c_int64(0)
    g = L.MbGaussians(10, -1, None, None, None, None, None)  # null parameter pointers
    cam = _cam()
    assert lib.mb_prepare(ctypes.byref(g), ctypes.byref(cam), 1, ctypes.byref(o), None, 0,
                          ctypes.byref(n), None) == L.MB_ERR_ARG
    g = L.MbGaussians(0, 7, None, None, None, None, None)  # SH degree out of range
    assert lib.mb_prepare(ctypes.byref(g), ctypes.byref(cam), 1, ctypes.byref(o), None, 0,
                          ctypes.byref(n), None) == L.MB_ERR_UNSUPPORTED
    g = L.MbGaussians(0, -1, None, None, None, None, None)
    cams = (L.MbCamera * 2)(_cam(64, 48), _cam(32, 48))  # mixed image sizes
    assert lib.mb_prepare(ctypes.byref(g), cams, 2, ctypes.byref(o), None, 0,
                          ctypes.byref(n), None) == L.MB_ERR_ARG
    bad = _cam()
    bad.fx = -1.0
    assert lib.mb_prepare(ctypes.byref(g), ctypes.byref(bad), 1, ctypes.byref(o), None, 0,
                          ctypes.byref(n), None) == L.MB_ERR_ARG
    assert lib.mb_prepare(ctypes.byref(g), ctypes.byref(cam), 0, ctypes.byref(o), None, 0,
                          ctypes.byref(n), None) == L.MB_ERR_ARG
    # workspace too small is reported, not written
    assert lib.mb_prepare(ctypes.byref(g), ctypes.byref(cam), 1, ctypes.byref(o), None, 0,
                          ctypes.byref(n), None) == L.MB_ERR_WORKSPACE


def test_device_count_accepted_only_where_documented():
    """MB_ENTRIES_ON_DEVICE is an n_entries value for mb_render_forward and
    mb_render_backward only; other negative counts, and the surrogate and
    harvest renders, reject it before any device work (the pointers below
    are never dereferenced)."""
    lib = L.load()
    o = L.MbOptions()
    lib.mb_default_options(ctypes.byref(o))
    g = L.MbGaussians(0, -1, None, None, None, None, None)
    cam = _cam()
    fake = ctypes.c_void_p(0x1000)
    # a negative count other than MB_ENTRIES_ON_DEVICE
    assert lib.mb_render_forward(ctypes.byref(g), ctypes.byref(cam), 1, ctypes.byref(o), None, 0, None, 0, -2,
                                 fake, fake, None, None) == L.MB_ERR_ARG
    assert lib.mb_render_backward(ctypes.byref(g), ctypes.byref(cam), 1, ctypes.byref(o), None, 0, None, 0, -2,
                                  fake, fake, None, None, None, None, None, None, None) == L.MB_ERR_ARG
    o.n_moments = 6
    assert lib.mb_render_forward_surrogate(ctypes.byref(g), ctypes.byref(cam), 1, ctypes.byref(o), None, 0, None,
                                           0, L.MB_ENTRIES_ON_DEVICE, fake, None, 0, 0, fake, fake,
                                           None) == L.MB_ERR_ARG
    assert lib.mb_render_forward_harvest(ctypes.byref(g), ctypes.byref(cam), 1, ctypes.byref(o), None, 0, None, 0,
                                         L.MB_ENTRIES_ON_DEVICE, 0.0, 0, None, 0, None, fake, fake,
                                         None) == L.MB_ERR_ARG
    # accepted by the plain forward: the next check is the workspace
    assert lib.mb_render_forward(ctypes.byref(g), ctypes.byref(cam), 1, ctypes.byref(o), None, 0, None, 0,
                                 L.MB_ENTRIES_ON_DEVICE, fake, fake, None, None) == L.MB_ERR_WORKSPACE
