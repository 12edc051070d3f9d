"""The C-ABI library loads and exports every symbol the header declares; host-side
argument validation rejects bad calls before touching a device (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2601_20429_amd import grtx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "grtx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(grtx_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_symbols_exported():
    names = _declared_functions()
    assert "grtx_trace" in names and "grtx_build" in names
    L = C.CDLL(grtx.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding knows every declared function
    assert set(names) <= set(grtx._SIGNATURES), set(names) - set(grtx._SIGNATURES)


def test_version_and_null_destroy():
    L = grtx.lib()
    assert L.grtx_version() == 5
    assert L.grtx_bvh_destroy(None) == grtx.OK


def test_build_rejects_bad_arguments():
    L = grtx.lib()
    h = C.c_void_p()
    p = grtx._BuildParams(1.0 / 255.0)
    assert L.grtx_build(None, 0, C.byref(p), None, C.byref(h)) == grtx.ERR_INVALID_ARG
    assert b"null" in L.grtx_last_error()
    g = grtx._Gaussians(None, None, None, None, None, 10, 0, 0)
    assert L.grtx_build(C.byref(g), 0, C.byref(p), None, C.byref(h)) == grtx.ERR_INVALID_ARG
    g = grtx._Gaussians(None, None, None, None, None, 0, 4, 0)
    assert L.grtx_build(C.byref(g), 0, C.byref(p), None, C.byref(h)) == grtx.ERR_INVALID_ARG
    assert b"sh_degree" in L.grtx_last_error()
    g = grtx._Gaussians(None, None, None, None, None, 0, 0, 0)
    bad = grtx._BuildParams(1.5)
    assert L.grtx_build(C.byref(g), 0, C.byref(bad), None, C.byref(h)) == grtx.ERR_INVALID_ARG
    assert L.grtx_build(C.byref(g), 7, C.byref(p), None, C.byref(h)) == grtx.ERR_INVALID_ARG
    for md in (-1, grtx.MAX_TREE_DEPTH + 1):
        bad = grtx._BuildParams(1.0 / 255.0, 0, md)
        assert L.grtx_build(C.byref(g), 0, C.byref(bad), None, C.byref(h)) == grtx.ERR_INVALID_ARG
        assert b"max_depth" in L.grtx_last_error()
    assert h.value is None  # out-param untouched


def test_trace_rejects_bad_arguments():
    L = grtx.lib()
    fake = C.c_void_p(1)  # never dereferenced: validation fails first
    rays = grtx._Rays(None, None, 4, 0.0, 0)
    out = grtx._TraceOutputs(None, None, None, None, None, None, 0, 0)
    for k, T, mode, tn, cc in [(0, 1e-3, 0, 0.0, 0), (65, 1e-3, 0, 0.0, 0), (4, 1.0, 0, 0.0, 0),
                               (4, 1e-3, 3, 0.0, 0), (4, 1e-3, 0, -1.0, 0), (4, 1e-3, 2, 0.0, 8193),
                               (4, 1e-3, 2, 0.0, -1)]:
        rays.t_near = tn
        prm = grtx._TraceParams(k, T, mode, (C.c_float * 3)(0, 0, 0), 0, 0, cc)
        assert L.grtx_trace(fake, C.byref(rays), C.byref(prm), C.byref(out), None) == grtx.ERR_INVALID_ARG
        assert L.grtx_trace_noalloc(fake, C.byref(rays), C.byref(prm), C.byref(out), None) == grtx.ERR_INVALID_ARG
    rays.t_near = 0.0
    prm = grtx._TraceParams(4, 1e-3, 0, (C.c_float * 3)(0, 0, 0), 0, 0)
    assert L.grtx_trace(fake, C.byref(rays), C.byref(prm), C.byref(out), None) == grtx.ERR_INVALID_ARG
    assert b"null" in L.grtx_last_error()
    assert L.grtx_trace_noalloc(fake, C.byref(rays), C.byref(prm), C.byref(out), None) == grtx.ERR_INVALID_ARG
    assert b"grtx_trace_noalloc: null" in L.grtx_last_error()
    # the image part: image_begin in 0..count, and only with an image width
    for width, begin in [(2, -1), (2, 5), (0, 2)]:
        bad = grtx._Rays(fake, fake, 4, 0.0, width)
        bad.image_begin = begin
        assert L.grtx_trace(fake, C.byref(bad), C.byref(prm), C.byref(out), None) == grtx.ERR_INVALID_ARG
        assert b"image_begin" in L.grtx_last_error()
    # one launch takes at most 2^31-1 work items; an image's 8x8 tiles count whole, so a
    # one-pixel-wide image of 2^28 rays makes 2^31 items
    for count, width in [(1 << 31, 0), (1 << 28, 1)]:
        big = grtx._Rays(fake, fake, count, 0.0, width)
        assert L.grtx_trace(fake, C.byref(big), C.byref(prm), C.byref(out), None) == grtx.ERR_INVALID_ARG
        assert b"2^31-1" in L.grtx_last_error()
    cam = grtx._Camera((C.c_float * 3)(0, -3, 0), (C.c_float * 3)(0, 0, 0), (C.c_float * 3)(0, 0, 1), 60.0, 0, 4)
    assert L.grtx_pinhole_rays(C.byref(cam), C.c_void_p(1), C.c_void_p(1), None) == grtx.ERR_INVALID_ARG


def test_secondary_ray_calls_reject_bad_arguments():
    L = grtx.lib()
    fake = C.c_void_p(1)  # never dereferenced: validation fails first
    rays = grtx._Rays(fake, fake, 4, 0.0, 0, None, None)
    ok = dict(sphere=(0, 0, 0, 0.5, 1.5), mirror=(1, 0, 0, 0, 0.4, 0, 0, 0, 0.3))
    for objs in [dict(ok, sphere=(0, 0, 0, 0.5, 0.0)), dict(ok, sphere=(0, 0, 0, 0.5, -1.0)),
                 dict(ok, mirror=(1, 0, 0, 0, 0.4, 0, 0, 0.3, 0.3)), dict(ok, eps=-1.0),
                 dict(ok, sphere=(float("nan"), 0, 0, 0.5, 1.5))]:
        ob = grtx._objects(objs)
        assert L.grtx_object_rays(C.byref(ob), C.byref(rays), fake, fake, fake, fake, fake, None) == \
            grtx.ERR_INVALID_ARG, objs
    ob = grtx._objects(ok)
    assert L.grtx_object_rays(C.byref(ob), C.byref(rays), None, fake, fake, fake, fake, None) == grtx.ERR_INVALID_ARG
    assert b"null" in L.grtx_last_error()
    assert L.grtx_object_rays(None, C.byref(rays), fake, fake, fake, fake, fake, None) == grtx.ERR_INVALID_ARG
    n = C.c_int64(-7)
    for bad_count in (-1, (1 << 24) + 1):
        assert L.grtx_continue_rays(bad_count, fake, fake, 1e-3, fake, fake, fake, fake, fake, fake, C.byref(n),
                                    None) == grtx.ERR_INVALID_ARG
    assert L.grtx_continue_rays(4, fake, fake, 1.0, fake, fake, fake, fake, fake, fake, C.byref(n), None) == \
        grtx.ERR_INVALID_ARG
    assert L.grtx_continue_rays(4, None, fake, 1e-3, fake, fake, fake, fake, fake, fake, C.byref(n), None) == \
        grtx.ERR_INVALID_ARG
    assert n.value == -7  # out-param untouched
    assert L.grtx_continue_composite(-1, *([fake] * 9), None) == grtx.ERR_INVALID_ARG
    assert L.grtx_continue_composite(3, None, *([fake] * 8), None) == grtx.ERR_INVALID_ARG
    # zero rays: nothing to do, no device touched
    assert L.grtx_continue_composite(0, *([None] * 9), None) == grtx.OK


def test_binding_raises_on_error():
    with pytest.raises(grtx.GrtxError):
        grtx._check(grtx.ERR_INVALID_ARG)


def test_serving_request_bytes_and_validation():
    """Admission accounting is host-only: a request holds its outputs (rgb, depth and
    opacity, 20 B per pixel; its rays are generated inside the serving kernel). Bad server
    configurations are refused before any device call."""
    from paper_2601_20429_amd import inputs
    cam = inputs.orbit_camera(800, 600)
    assert grtx.request_bytes(cam) == 800 * 600 * 20
    L = grtx.lib()
    h = C.c_void_p()
    bg = (C.c_float * 3)()
    for cfg in [grtx._ServeConfig(0, 16, 1e-3, 0, 0, bg, 0),               # no budget
                grtx._ServeConfig(1 << 30, 0, 1e-3, 0, 0, bg, 0),          # k = 0
                grtx._ServeConfig(1 << 30, 16, 1.0, 0, 0, bg, 0),          # T_min = 1
                grtx._ServeConfig(1 << 30, 16, 1e-3, 5, 0, bg, 0),         # unknown mode
                grtx._ServeConfig(1 << 30, 16, 1e-3, 0, (1 << 22) + 1, bg, 0),  # requests beyond 2^22 pixels
                grtx._ServeConfig(1 << 30, 16, 1e-3, 0, -1, bg, 0),
                grtx._ServeConfig(1 << 30, 16, 1e-3, 0, 0, bg, -5)]:       # negative idle time
        assert L.grtx_serve_create(C.byref(cfg), C.byref(h)) == grtx.ERR_INVALID_ARG
    assert h.value is None
    assert L.grtx_serve_destroy(None) == grtx.OK
