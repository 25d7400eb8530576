"""Pins of the oracle's non-plane incidence: a point source on the lab axis
(the incident phase term Phi_i of Eq. 10 with a curved incident wavefront).

None of these re-types the oracle's formulas: the wavefront curvatures are
checked against paraxial (Gaussian) optics -- the mirror equation and the
vergence form of refraction and transfer -- and the off-axis amplitude and
phase against a separate 2-D reflection tracer with ray-tube energy balance.
"""
import math

import numpy as np
import pytest

import oracle as O

LAM = 0.6328
K = 2 * math.pi / LAM
M = 1.333
A = 50.0


def _sphere():
    return O.particle((A, A, A), (0, 0, 0), M)


def _emit(ray, p):
    e = ray.emit[p]
    f = np.array(e.field[:]).reshape(2, 3, 2)
    return dict(q=np.array(e.q[:]), amp=e.amp, phase=e.phase, nf=e.nf, dir=np.array(e.dir[:]),
                rexit=np.array(e.rexit[:]), field=f[..., 0] + 1j * f[..., 1], valid=e.valid)


@pytest.mark.parametrize("zs", [60.0, 120.0, 1000.0, 1e5])
def test_on_axis_reflection_follows_the_mirror_equation(zs):
    """Convex spherical mirror of radius a, source at s = z_s - a from its
    vertex: the reflected wave diverges from the virtual image, 1/s' = 1/s + 2/a;
    the far-field amplitude is z_s |r| s'/s (angular magnification s/s')."""
    st = O.setup(LAM, 1, 0, 0, 8, source_distance=zs)
    ray = O.trace_rays(_sphere(), st, [(0.0, 0.0)])[0]
    e = _emit(ray, 0)
    s = zs - A
    q = 1 / s + 2 / A
    assert e["q"] == pytest.approx([q, 0.0, q], rel=1e-12, abs=1e-15)
    assert e["nf"] == 0
    r = (1 - M) / (1 + M)
    expect = zs * r * (1 / q) / s * np.exp(-2j * K * A)  # phase: -2 k a, path S -> vertex -> far field
    assert abs(e["field"][0, 0] - expect) <= 1e-10 * abs(expect)
    assert np.abs(e["field"][0, 1:]).max() <= 1e-12 * abs(expect)


@pytest.mark.parametrize("zs", [70.0, 200.0, 5000.0])
def test_on_axis_ball_lens_follows_vergence_optics(zs):
    """Vergence V = -n Q (positive converging); refraction adds the surface
    power (n' - n)/R_c, transfer over d in index n gives V / (1 - d V / n)."""
    st = O.setup(LAM, 1, 1, 1, 8, source_distance=zs)
    ray = O.trace_rays(_sphere(), st, [(0.0, 0.0)])[0]
    s = zs - A
    V0 = -1.0 / s
    V1 = V0 + (M - 1) / A            # entry surface, centre of curvature beyond it
    Qt = -V1 / M
    assert np.array(ray.q_cont[0][:]) == pytest.approx([Qt, 0.0, Qt], rel=1e-12, abs=1e-15)
    V1d = V1 / (1 - 2 * A * V1 / M)  # across the diameter
    V2 = V1d + (1 - M) / (-A)        # exit surface, centre of curvature behind it
    e = _emit(ray, 1)
    assert e["q"] == pytest.approx([-V2, 0.0, -V2], rel=1e-11, abs=1e-15)
    # amplitude: height ratio h2/h1 = 1 - 2a V1/m, exit angle h2 |Q_out|, entry angle h1 / s
    t1 = 2 / (1 + M)
    t2 = 2 * M / (M + 1)
    mag = s * abs(1 - 2 * A * V1 / M) * abs(V2)
    assert abs(e["field"][0, 0]) == pytest.approx(zs * t1 * t2 / mag, rel=1e-11)


def _fresnel_r(ci):
    st = math.sqrt(1 - ci * ci)
    ct = math.sqrt(1 - (st / M) ** 2)
    r_perp = (ci - M * ct) / (ci + M * ct)
    r_par = (M * ci - ct) / (M * ci + ct)
    return r_perp, r_par


def _reflect_2d(zs, alpha):
    """Ray from S = (0, 0, -z_s) at angle alpha to the axis off the sphere of
    radius A at the origin; returns (hit point, reflected direction, cos i) in
    the plane (transverse, z)."""
    d = np.array([math.sin(alpha), math.cos(alpha)])
    S = np.array([0.0, -zs])
    b = S @ d
    t = -b - math.sqrt(b * b - (S @ S - A * A))
    P = S + t * d
    n = P / A
    ci = -(d @ n)
    return P, d + 2 * ci * n, ci, t


@pytest.mark.parametrize("zs,alpha_deg", [(150.0, 5.0), (150.0, 12.0), (400.0, 4.0), (2000.0, 0.8)])
def test_off_axis_reflection_matches_ray_tube_balance(zs, alpha_deg):
    """Power per unit source solid angle is z_s^2 (unit amplitude at the
    centre's distance); after reflection it spreads over d Omega_out, so
    |S|^2 = |r|^2 z_s^2 sin(alpha) / (sin(theta) |d theta / d alpha|).  The
    phase is the optical path S -> P -> far field against the centre."""
    al = math.radians(alpha_deg)
    P, dr, ci, rho = _reflect_2d(zs, al)
    th = math.atan2(dr[0], dr[1])
    h = 1e-6
    dth = (math.atan2(*_reflect_2d(zs, al + h)[1]) - math.atan2(*_reflect_2d(zs, al - h)[1])) / (2 * h)
    amp = zs * math.sqrt(math.sin(al) / (abs(math.sin(th)) * abs(dth)))
    phase = K * (rho - zs) - K * (dr @ P)
    r_perp, r_par = _fresnel_r(ci)
    st = O.setup(LAM, 1, 0, 0, 8, source_distance=zs)
    y = zs * math.tan(al)
    # plane y-z: x polarisation is perpendicular to the plane of incidence
    e = _emit(O.trace_rays(_sphere(), st, [(0.0, y)])[0], 0)
    assert e["dir"] == pytest.approx([0.0, dr[0], dr[1]], abs=1e-12)
    assert e["rexit"] == pytest.approx([0.0, P[0], P[1]], abs=1e-10)
    expect = amp * r_perp * np.exp(1j * phase)
    assert abs(e["field"][0, 0] - expect) <= 2e-8 * abs(expect)
    # plane x-z: x polarisation lies in the plane of incidence
    e = _emit(O.trace_rays(_sphere(), st, [(y, 0.0)])[0], 0)
    f = e["field"][0]
    assert np.linalg.norm(f) == pytest.approx(amp * abs(r_par), rel=2e-8)
    assert abs(f[1]) <= 1e-12 * np.linalg.norm(f)
    # the field is transverse to the ray and its phase is the path phase (up to the basis sign)
    assert abs(f @ e["dir"]) <= 1e-12 * np.linalg.norm(f)
    w = f[0] / (amp * r_par * np.exp(1j * phase))
    assert min(abs(w / abs(w) - 1), abs(w / abs(w) + 1)) <= 2e-8


@pytest.mark.parametrize("zs", [51.0, 75.0, 150.0, 1e4])
def test_grid_halfwidth_of_a_sphere_is_its_shadow_cone(zs):
    """A sphere's tangent cone from S has half-angle asin(a / z_s); it crosses
    z = 0 at radius z_s tan(asin(a / z_s))."""
    L = O.grid_halfwidth(_sphere(), zs)
    assert L == pytest.approx(zs * A / math.sqrt(zs * zs - A * A), rel=1e-12)


def _scan_hits(part, st, pts):
    rays = O.trace_rays(part, st, pts)
    return np.array([rays[i].active for i in range(len(pts))], bool)


@pytest.mark.parametrize("euler", [(30, 20, 10), (80, 55, -35)])
def test_grid_halfwidth_is_tight_around_the_particle(euler):
    """Traced rays (the entry quadratic, not the cone formula): no ray just
    outside the half-width on any side meets the tilted ellipsoid, and some
    ray just inside it does on at least one side."""
    part = O.particle((60.0, 50.0, 40.0), euler, M)
    zs = 150.0
    L = O.grid_halfwidth(part, zs)
    st = O.setup(LAM, 1, 0, 0, 8, source_distance=zs)
    u = np.linspace(-L, L, 40001)
    inside_any = False
    for f in (1 + 1e-6, 1 - 1e-4):
        hit = False
        for sx, sy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            c = f * L
            pts = np.stack([np.full_like(u, sx * c) if sx else u, np.full_like(u, sy * c) if sy else u], 1)
            hit |= bool(_scan_hits(part, st, pts).any())
        if f > 1:
            assert not hit
        else:
            inside_any = hit
    assert inside_any
    # the point source sees the particle wider than the plane wave, and the
    # width tends to the plane wave's as 1/z_s when the source recedes
    L0 = O.grid_halfwidth(part)
    assert L > L0
    ex = [O.grid_halfwidth(part, z) / L0 - 1 for z in (1e7, 1e9, 1e13)]
    assert ex[1] / ex[0] == pytest.approx(1e-2, rel=1e-3)
    assert abs(ex[2]) < 1e-11


def test_far_source_converges_to_the_plane_wave():
    """z_s -> infinity: the far field of the point source tends to the plane
    wave's, with an error falling as 1/z_s (the incident curvature phase
    across the particle is about k a^2 / (2 z_s))."""
    part = O.particle((40.0, 36.0, 32.0), (20, 30, 40), M)
    th = np.arange(20.0, 170.0, 7.0)
    ph = np.arange(0.0, 360.0, 15.0)
    ref = O.farfield(part, O.setup(LAM, 1, 0, 1, 96), th, ph)["field"]
    med, mx = [], []
    for zs in (1e5, 1e6, 1e7):
        F = O.farfield(part, O.setup(LAM, 1, 0, 1, 96, source_distance=zs), th, ph)["field"]
        d = np.abs(F - ref) / np.abs(ref).max()
        med.append(np.median(d))
        mx.append(d.max())
    assert mx[2] < 1e-3 and 0.05 < mx[2] / mx[1] < 0.2
    assert 0.08 < med[1] / med[0] < 0.12 and 0.08 < med[2] / med[1] < 0.12


@pytest.mark.parametrize("zs", [-1.0, 30.0, 60.0])
def test_source_inside_the_bounding_sphere_is_rejected(zs):
    part = O.particle((60.0, 50.0, 40.0), (0, 0, 0), M)
    with pytest.raises(ValueError):
        O.trace_rays(part, O.setup(LAM, 1, 0, 1, 8, source_distance=zs), [(0.0, 0.0)])
