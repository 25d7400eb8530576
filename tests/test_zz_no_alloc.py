"""rtw_farfield_static -- the far field with the library's static workspace,
for callers that cannot allocate device memory -- against rtw_farfield on the
same inputs.  Both run the same kernels, so the results must agree bit for
bit; two calls in a row (the second on a smaller problem) check that what a
call leaves in the shared array does not leak into the next."""
import sys

import numpy as np
import pytest

from paper_2403_13856_amd import inputs as I

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problem(rtw, N, step, prec):
    w = I.ellipsoid_mixed()
    part = rtw.make_particle(w.semi_axes, w.euler_deg, w.m)
    inc = rtw.make_incident(w.wavelength, 2)
    opts = rtw.make_opts(w.p_min, w.p_max, N, prec)
    th = I.uniform_angles(0.0, 180.0, step)
    ph = I.uniform_angles(0.0, 360.0 - step, step)
    return part, inc, opts, th, ph


@pytest.mark.gpu
@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_static_workspace_matches_farfield_on_two_calls(prec_name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_13856_amd import rtw
    rtw.load()
    prec = rtw.FP64 if prec_name == "fp64" else rtw.MIXED
    for N, step in ((128, 1.0), (40, 2.5)):  # the second call is the smaller one
        part, inc, opts, th, ph = _problem(rtw, N, step, prec)
        say(f"[static workspace] {prec_name} N={N} nodes={th.size}x{ph.size}")
        ff = rtw.FarField(part, inc, opts, th, ph)
        ref = ff().clone()
        nc_ref = ff.ncontrib.clone()
        out = torch.full_like(ff.out, float("nan"))
        nc = torch.full_like(ff.ncontrib, -1)
        status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
        rtw.farfield_static(part, inc, opts, ff.theta, ff.phi, out, nc, status)
        torch.cuda.synchronize()
        assert int(status.item()) == rtw.RTW_OK
        assert torch.equal(out, torch.view_as_real(ref)), "static-workspace far field differs"
        assert torch.equal(nc, nc_ref)
        assert int(nc.sum().item()) > 0
        say(f"   bitwise equal, {int(nc.sum().item())} contributions")


def test_static_workspace_rejects_a_problem_beyond_its_size():
    """The full-size 2048^2 ellipsoid far field needs far more than the static
    array: the call is refused on the host, before any device work."""
    import ctypes

    from paper_2403_13856_amd import rtw
    L = rtw.load()
    part, inc, opts, th, ph = _problem(rtw, 2048, 0.5, rtw.MIXED)
    g = rtw.Grid(th.size, 1, ph.size, 1)  # node pointers are not dereferenced before the size check
    rc = L.rtw_farfield_static(ctypes.byref(part), ctypes.byref(inc), ctypes.byref(opts), ctypes.byref(g),
                               ctypes.c_void_p(256), None, None, None)
    assert rc == rtw.RTW_ERR_WORKSPACE
    assert "static" in L.rtw_last_error().decode()
