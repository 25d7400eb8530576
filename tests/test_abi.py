"""The C-ABI boundary on the CPU: librtw.so loads, exports every entry point
include/rtw.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2403_13856_amd import rtw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(rtw_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_builds_and_exports_every_declared_symbol():
    L = rtw.load()
    declared = _declared_functions()
    assert declared, "no declarations found in include/"
    for name in declared:
        assert hasattr(L, name), f"{name} declared in include/ but not exported"
    assert L.rtw_version().decode().startswith("rtw-mi355x")


def _ws(part, inc, opts, n_theta=10, n_phi=20):
    g = rtw.Grid(n_theta, 1, n_phi, 1)  # pointers are not dereferenced by the size query
    n = ctypes.c_size_t(0)
    rc = rtw.load().rtw_farfield_workspace_size(ctypes.byref(part), ctypes.byref(inc), ctypes.byref(opts),
                                                ctypes.byref(g), 0.0, ctypes.byref(n))
    return rc, n.value


def test_argument_validation_without_device():
    L = rtw.load()
    good = (rtw.make_particle((50, 40, 30), (10, 20, 30), 1.333), rtw.make_incident(0.6328, 2),
            rtw.make_opts(0, 3, 64, rtw.FP64))
    rc, n = _ws(*good)
    assert rc == rtw.RTW_OK and n > 0
    cases = [
        (rtw.make_particle((0, 40, 30)), good[1], good[2], rtw.RTW_ERR_INVALID_ARG),
        (rtw.make_particle((50, 40, 30), m=1.0), good[1], good[2], rtw.RTW_ERR_UNSUPPORTED),
        (rtw.make_particle((50, 40, 30), m=-1.3), good[1], good[2], rtw.RTW_ERR_INVALID_ARG),
        (good[0], rtw.make_incident(0.0, 1), good[2], rtw.RTW_ERR_INVALID_ARG),
        (good[0], rtw.make_incident(0.6, 3), good[2], rtw.RTW_ERR_INVALID_ARG),
        (good[0], good[1], rtw.make_opts(2, 1, 64), rtw.RTW_ERR_INVALID_ARG),
        (good[0], good[1], rtw.make_opts(0, 16, 64), rtw.RTW_ERR_UNSUPPORTED),
        (good[0], good[1], rtw.make_opts(0, 3, 1), rtw.RTW_ERR_INVALID_ARG),
        (good[0], good[1], rtw.make_opts(0, 3, 64, 7), rtw.RTW_ERR_INVALID_ARG),
        # point source: beyond the largest semi-axis (50 um), finite, not negative
        (good[0], rtw.make_incident(0.6328, 2, 50.0), good[2], rtw.RTW_ERR_INVALID_ARG),
        (good[0], rtw.make_incident(0.6328, 2, 30.0), good[2], rtw.RTW_ERR_INVALID_ARG),
        (good[0], rtw.make_incident(0.6328, 2, -200.0), good[2], rtw.RTW_ERR_INVALID_ARG),
        (good[0], rtw.make_incident(0.6328, 2, float("inf")), good[2], rtw.RTW_ERR_INVALID_ARG),
        (good[0], rtw.make_incident(0.6328, 2, float("nan")), good[2], rtw.RTW_ERR_INVALID_ARG),
        # observation radius: 0 (far field) or beyond the largest semi-axis, finite
        (good[0], rtw.make_incident(0.6328, 2, 0.0, 50.0), good[2], rtw.RTW_ERR_INVALID_ARG),
        (good[0], rtw.make_incident(0.6328, 2, 0.0, -500.0), good[2], rtw.RTW_ERR_INVALID_ARG),
        (good[0], rtw.make_incident(0.6328, 2, 200.0, float("inf")), good[2], rtw.RTW_ERR_INVALID_ARG),
        (good[0], rtw.make_incident(0.6328, 2, 0.0, float("nan")), good[2], rtw.RTW_ERR_INVALID_ARG),
        # corrections: known bits only; the Fraunhofer term needs a plane wave and the far field
        (good[0], good[1], rtw.make_opts(0, 3, 64, rtw.FP64, 4), rtw.RTW_ERR_INVALID_ARG),
        (good[0], rtw.make_incident(0.6328, 2, 60.0), rtw.make_opts(0, 3, 64, rtw.FP64, rtw.DIFFRACTION),
         rtw.RTW_ERR_UNSUPPORTED),
        (good[0], rtw.make_incident(0.6328, 2, 0.0, 60.0), rtw.make_opts(0, 3, 64, rtw.FP64, rtw.DIFFRACTION),
         rtw.RTW_ERR_UNSUPPORTED),
    ]
    for corr in (rtw.CAUSTIC, rtw.DIFFRACTION, rtw.CAUSTIC | rtw.DIFFRACTION):
        rc, n_c = _ws(good[0], good[1], rtw.make_opts(0, 3, 64, rtw.FP64, corr))
        assert rc == rtw.RTW_OK and n_c >= n  # the caustic form keeps phases per record and per hit
    rc, n_pc = _ws(good[0], rtw.make_incident(0.6328, 2, 60.0), rtw.make_opts(0, 3, 64, rtw.FP64, rtw.CAUSTIC))
    assert rc == rtw.RTW_OK
    rc, n_obs = _ws(good[0], rtw.make_incident(0.6328, 2, 0.0, 50.5), good[2])
    assert rc == rtw.RTW_OK and n_obs == n
    rc, n_src = _ws(good[0], rtw.make_incident(0.6328, 2, 50.5), good[2])
    assert rc == rtw.RTW_OK and n_src == n
    for part, inc, opts, code in cases:
        rc, _ = _ws(part, inc, opts)
        assert rc == code, (rc, code)
        assert L.rtw_last_error().decode() != ""
        # rtw_trace validates before launching anything
        rec = rtw.RayRecords()
        assert L.rtw_trace(ctypes.byref(part), ctypes.byref(inc), ctypes.byref(opts), ctypes.byref(rec), None) == code
    # NULL structs and NULL outputs
    assert L.rtw_trace(None, None, None, None, None) == rtw.RTW_ERR_INVALID_ARG
    g = rtw.Grid(10, 1, 20, 1)
    assert L.rtw_farfield(ctypes.byref(good[0]), ctypes.byref(good[1]), ctypes.byref(good[2]), ctypes.byref(g),
                          None, None, None, 0, None) == rtw.RTW_ERR_INVALID_ARG
    # misaligned workspace is rejected before any launch
    assert L.rtw_farfield(ctypes.byref(good[0]), ctypes.byref(good[1]), ctypes.byref(good[2]), ctypes.byref(g),
                          ctypes.c_void_p(256), None, ctypes.c_void_p(4096 + 8), 1 << 20,
                          None) == rtw.RTW_ERR_INVALID_ARG
    assert L.rtw_farfield_status(None, None, None) == rtw.RTW_ERR_INVALID_ARG


def test_workspace_size_scales_with_problem():
    part, inc = rtw.make_particle((50, 40, 30)), rtw.make_incident(0.6328, 1)
    _, n64 = _ws(part, inc, rtw.make_opts(0, 3, 64, rtw.FP64))
    _, n128 = _ws(part, inc, rtw.make_opts(0, 3, 128, rtw.FP64))
    _, m128 = _ws(part, inc, rtw.make_opts(0, 3, 128, rtw.MIXED))
    assert n128 > n64 and m128 < n128
    _, big_nodes = _ws(part, inc, rtw.make_opts(0, 3, 64, rtw.FP64), 1801, 720)
    assert big_nodes > n64


def _batch_ws(parts, sides, inc, opts, n_theta=361, n_phi=180, rays_per_chunk=0):
    n = len(parts)
    P = (rtw.Particle * n)(*parts)
    G = (ctypes.c_int * n)(*sides)
    g = rtw.Grid(n_theta, 1, n_phi, 1)
    bo = rtw.BatchOpts(rays_per_chunk, 0.0)
    out = ctypes.c_size_t(0)
    rc = rtw.load().rtw_batch_workspace_size(n, P, G, ctypes.byref(inc), ctypes.byref(opts), ctypes.byref(g),
                                             ctypes.byref(bo), ctypes.byref(out))
    return rc, out.value


def test_batch_workspace_and_validation_without_device():
    L = rtw.load()
    inc, opts = rtw.make_incident(0.6328, 2), rtw.make_opts(0, 3, 2, rtw.MIXED)
    parts = [rtw.make_particle((30 + i, 28, 25), (i, 2 * i, 3 * i), 1.33 + 0.01 * i) for i in range(6)]
    sides = [256, 512, 256, 1024, 384, 256]
    rc, whole = _batch_ws(parts, sides, inc, opts)
    assert rc == rtw.RTW_OK and whole > 0
    # a smaller chunk budget needs a smaller workspace (records are sized per chunk)
    rc, chunked = _batch_ws(parts, sides, inc, opts, rays_per_chunk=1 << 18)
    assert rc == rtw.RTW_OK and chunked < whole
    # one bad particle is named in the error
    bad = list(parts)
    bad[3] = rtw.make_particle((30, 28, 25), m=1.0)
    rc, _ = _batch_ws(bad, sides, inc, opts)
    assert rc == rtw.RTW_ERR_UNSUPPORTED and "particle 3" in L.rtw_last_error().decode()
    rc, _ = _batch_ws(parts, [256, 512, 1, 1024, 384, 256], inc, opts)
    assert rc == rtw.RTW_ERR_INVALID_ARG
    rc, _ = _batch_ws(parts, sides, inc, opts, n_theta=70000, n_phi=2)
    assert rc == rtw.RTW_ERR_INVALID_ARG
    # rtw_batch rejects NULL outputs, a misaligned workspace and a bad tuning before any device call
    n = len(parts)
    P = (rtw.Particle * n)(*parts)
    G = (ctypes.c_int * n)(*sides)
    g = rtw.Grid(361, 1, 180, 1)
    args = (n, P, G, ctypes.byref(inc), ctypes.byref(opts), ctypes.byref(g))
    assert L.rtw_batch(*args, None, None, None, None, None, None, 0, None) == rtw.RTW_ERR_INVALID_ARG
    assert L.rtw_batch(*args, ctypes.c_void_p(256), None, None, None, None, ctypes.c_void_p(4096 + 8), 1 << 30,
                       None) == rtw.RTW_ERR_INVALID_ARG
    t = rtw.Tune(300, 8, 32)
    assert L.rtw_batch(*args, ctypes.c_void_p(256), None, None, ctypes.byref(t), None, ctypes.c_void_p(4096), 1 << 30,
                       None) == rtw.RTW_ERR_INVALID_ARG
    assert L.rtw_batch(0, P, G, ctypes.byref(inc), ctypes.byref(opts), ctypes.byref(g), ctypes.c_void_p(256), None,
                       None, None, None, ctypes.c_void_p(4096), 1 << 30, None) == rtw.RTW_ERR_INVALID_ARG


def test_surrogate_rejects_point_source_incidence():
    """The surrogate models plane-wave incidence and the far field only (host-side check)."""
    L = rtw.load()
    part = rtw.make_particle((50, 40, 30), (10, 20, 30), 1.333)
    th = (ctypes.c_double * 1)(130.0)
    ph = (ctypes.c_double * 1)(10.0)
    feats = (ctypes.c_float * 64)()
    fn = L.rtw_surrogate_features
    for zs, R, code in ((0.0, 0.0, rtw.RTW_OK), (500.0, 0.0, rtw.RTW_ERR_UNSUPPORTED),
                        (0.0, 500.0, rtw.RTW_ERR_UNSUPPORTED)):
        inc = rtw.make_incident(0.6328, 2, zs, R)
        rc = fn(1, ctypes.byref(part), ctypes.byref(inc), 1, th, ph, feats)
        assert rc == code, (zs, rc)


def test_batch_rejects_a_source_inside_one_particle():
    """Every particle of a batch is checked against the point source (host side)."""
    L = rtw.load()
    parts = (rtw.Particle * 2)(rtw.make_particle((30, 25, 20), (0, 0, 0), 1.333),
                               rtw.make_particle((200, 150, 120), (10, 20, 30), 1.4))
    sides = (ctypes.c_int * 2)(64, 64)
    opts = rtw.make_opts(0, 3, 2, rtw.MIXED)
    g = rtw.Grid(10, 1, 20, 1)
    n = ctypes.c_size_t(0)
    for zs, code in ((500.0, rtw.RTW_OK), (150.0, rtw.RTW_ERR_INVALID_ARG)):
        inc = rtw.make_incident(0.6328, 2, zs)
        rc = L.rtw_batch_workspace_size(2, parts, sides, ctypes.byref(inc), ctypes.byref(opts), ctypes.byref(g), None,
                                        ctypes.byref(n))
        assert rc == code, (zs, rc)
    assert "source_distance" in L.rtw_last_error().decode()


def test_batch_chunks_keep_node_indices_32bit():
    """Node indices within a chunk (chunk particle, theta, phi) are 32-bit: on a
    node grid of 2^30 nodes a chunk holds one particle, so the per-node
    count and range arrays of a three-particle batch are those of one particle."""
    inc, opts = rtw.make_incident(0.6328, 1), rtw.make_opts(0, 0, 2, rtw.MIXED)
    parts = [rtw.make_particle((20.0, 20.0, 20.0), (0, 0, 0), 1.333) for _ in range(3)]
    n_theta, n_phi = 32768, 32768  # 2^30 nodes, the largest grid accepted
    assert 2 * n_theta * n_phi > (1 << 31) - 1
    rc1, one = _batch_ws(parts[:1], [16], inc, opts, n_theta, n_phi)
    rc3, three = _batch_ws(parts, [16, 16, 16], inc, opts, n_theta, n_phi)
    assert rc1 == rtw.RTW_OK and rc3 == rtw.RTW_OK
    per_node_arrays = 2 * 4 * n_theta * n_phi  # counts and range starts, int32
    assert three - one < per_node_arrays // 8, (one, three)
    # a grid of a few thousand nodes still packs the three particles in one chunk
    _, small1 = _batch_ws(parts[:1], [16], inc, opts, 64, 64)
    _, small3 = _batch_ws(parts, [16, 16, 16], inc, opts, 64, 64)
    assert small3 - small1 >= 2 * 2 * 4 * 64 * 64


def test_profile_filter_without_device():
    """rtw_profile_only takes a name or NULL and records nothing by itself:
    with no kernel launched, a read reports no kernels either way."""
    L = rtw.load()
    n = ctypes.c_int(-1)
    for name in (b"k_raster_mixed", b"", None):
        assert L.rtw_profile_only(name) == rtw.RTW_OK
        assert L.rtw_profile_read(0, None, None, None, ctypes.byref(n)) == rtw.RTW_OK
        assert n.value == 0
    assert L.rtw_profile_only(None) == rtw.RTW_OK
