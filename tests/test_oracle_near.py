"""Pins of the oracle's observation at a finite distance (the point M of Eqs. 6
and 9: the field on the sphere of radius R about the particle, reported as
R e^{-ikR} E(M)).

None of these re-types the oracle's formulas: the on-axis values come from
paraxial (Gaussian) optics -- the mirror equation and vergence transfer, with
the Gouy phase of a focus -- the off-axis amplitude and phase from a separate
2-D reflection tracer with ray-tube energy balance on the sphere, the
assembly from rays root-found on the oracle's own per-ray trace (pinned here),
and the far field of the plane-wave pins is the limit R -> infinity.
"""
import math

import numpy as np
import pytest

import oracle as O

LAM = 0.6328
K = 2 * math.pi / LAM
M = 1.333
A = 50.0


def _sphere(m=M):
    return O.particle((A, A, A), (0, 0, 0), m)


def _emit(ray, p):
    e = ray.emit[p]
    f = np.array(e.field[:]).reshape(2, 3, 2)
    return dict(amp=e.amp, phase=e.phase, nf=e.nf, dir=np.array(e.dir[:]), obs=np.array(e.obs[:]),
                rexit=np.array(e.rexit[:]), field=f[..., 0] + 1j * f[..., 1], valid=e.valid)


@pytest.mark.parametrize("zs", [0.0, 150.0])
@pytest.mark.parametrize("R", [60.0, 200.0, 1e4])
def test_on_axis_reflection_at_finite_distance(zs, R):
    """Convex mirror of radius a: the reflected wave diverges from the virtual
    image at s' behind the vertex (1/s' = 1/s + 2/a, s the source distance from
    the vertex; s' = a/2 for a plane wave), so at M = (0, 0, -R) the amplitude
    is r A_v s' / (s' + R - a) with A_v the incident amplitude at the vertex.
    Relative to the particle centre the path is 2 a shorter than R (plus z_s)."""
    st = O.setup(LAM, 1, 0, 0, 8, source_distance=zs, observation_radius=R)
    e = _emit(O.trace_rays(_sphere(), st, [(0.0, 0.0)])[0], 0)
    r = (1 - M) / (1 + M)
    if zs > 0:
        s = zs - A
        sp = 1 / (1 / s + 2 / A)
        Av = zs / s
    else:
        sp, Av = A / 2, 1.0
    expect = R * r * Av * sp / (sp + R - A) * np.exp(-2j * K * A)
    assert e["nf"] == 0
    assert e["obs"] == pytest.approx([0.0, 0.0, -1.0], abs=1e-15)
    assert e["dir"] == pytest.approx([0.0, 0.0, -1.0], abs=1e-15)
    assert abs(e["field"][0, 0] - expect) <= 1e-11 * abs(expect)
    assert np.abs(e["field"][0, 1:]).max() <= 1e-12 * abs(expect)


@pytest.mark.parametrize("R,nf", [(80.0, 0), (200.0, 2)])
def test_on_axis_ball_lens_before_and_beyond_its_focus(R, nf):
    """Vergence optics of the ball lens (V = -Q, positive converging): entry
    power (m - 1)/a, transfer over the diameter in index m, exit power
    (m - 1)/a; the axial amplitude falls as 1/|1 - d V| over a distance d.
    The paraxial focus lies 1/V_2 ~ 50 um beyond the exit vertex: the point at
    R = 200 lies beyond it and carries the focus's two focal lines
    (-pi in all)."""
    st = O.setup(LAM, 1, 1, 1, 8, observation_radius=R)
    e = _emit(O.trace_rays(_sphere(), st, [(0.0, 0.0)])[0], 1)
    V1 = (M - 1) / A
    h = 1 - 2 * A * V1 / M
    V2 = V1 / h + (M - 1) / A
    d = R - A
    assert (d * V2 > 1) == (nf == 2)
    t = (2 / (1 + M)) * (2 * M / (M + 1))
    amp = R / (abs(h) * abs(1 - d * V2))  # the ray tube's factor; the Fresnel product t is in the field
    phase = 2 * K * A * (M - 1) - nf * math.pi / 2
    assert e["nf"] == nf
    assert e["obs"] == pytest.approx([0.0, 0.0, 1.0], abs=1e-15)
    assert e["amp"] == pytest.approx(amp, rel=1e-11)
    expect = t * amp * np.exp(1j * phase)
    assert abs(e["field"][0, 0] - expect) <= 1e-10 * abs(expect)


def _reflect_to_sphere(zs, s, R):
    """2-D reflection off the sphere in the plane (transverse, z): a plane wave
    (zs = 0) ray at impact parameter s, or a ray from (0, -z_s) at angle s to
    the axis.  Returns the hit point P, the reflected direction, cos i, the
    incident path from the source (point source) and the point M where the
    reflected ray meets the circle of radius R."""
    if zs > 0:
        d = np.array([math.sin(s), math.cos(s)])
        S = np.array([0.0, -zs])
        b = S @ d
        rho = -b - math.sqrt(b * b - (S @ S - A * A))
        P = S + rho * d
    else:
        d = np.array([0.0, 1.0])
        P = np.array([s, -math.sqrt(A * A - s * s)])
        rho = 0.0
    n = P / A
    ci = -(d @ n)
    dr = d + 2 * ci * n
    c = P @ dr
    dM = -c + math.sqrt(c * c - (P @ P - R * R))
    return P, dr, ci, rho, P + dM * dr, dM


def _fresnel_r(ci):
    st = math.sqrt(1 - ci * ci)
    ct = math.sqrt(1 - (st / M) ** 2)
    return (ci - M * ct) / (ci + M * ct), (M * ci - ct) / (M * ci + ct)


@pytest.mark.parametrize("zs,s,R", [(0.0, 20.0, 120.0), (0.0, 42.0, 500.0), (150.0, math.radians(9.0), 90.0),
                                    (400.0, math.radians(4.0), 3000.0)])
def test_off_axis_reflection_matches_ray_tube_balance_on_the_sphere(zs, s, R):
    """The power a tube carries (|E|^2 times the annulus 2 pi s ds of a plane
    wave, or z_s^2 times 2 pi sin(alpha) d alpha of the source normalised to unit
    amplitude at the centre) crosses the sphere over 2 pi R^2 sin(theta_M)
    |d theta_M| at incidence cos = d.u, so
    R |E(M)| = |r| sqrt(w / (sin theta_M |d theta_M / ds| d.u)), w = s or
    z_s^2 sin(alpha).  The phase is the optical path source -> P -> M minus R."""
    P, dr, ci, rho, Mp, dM = _reflect_to_sphere(zs, s, R)
    thM = math.atan2(Mp[0], Mp[1])
    h = 1e-5
    th = [math.atan2(*_reflect_to_sphere(zs, s + j * h, R)[4]) for j in (-2, -1, 1, 2)]
    dth = (th[0] - 8 * th[1] + 8 * th[2] - th[3]) / (12 * h)  # fourth-order central difference
    u = Mp / R
    w = s if zs == 0 else zs * zs * math.sin(s)
    amp = math.sqrt(w / (abs(math.sin(thM)) * abs(dth) * (dr @ u)))
    if zs == 0:
        phase = K * P[1] + K * dM - K * R
        y = s
    else:
        phase = K * (rho - zs) + K * dM - K * R
        y = zs * math.tan(s)
    r_perp, r_par = _fresnel_r(ci)
    st = O.setup(LAM, 1, 0, 0, 8, source_distance=zs, observation_radius=R)
    # plane y-z: x polarisation is perpendicular to the plane of incidence
    e = _emit(O.trace_rays(_sphere(), st, [(0.0, y)])[0], 0)
    assert e["nf"] == 0
    assert e["obs"] == pytest.approx([0.0, u[0], u[1]], abs=1e-12)
    assert e["dir"] == pytest.approx([0.0, dr[0], dr[1]], abs=1e-12)
    expect = amp * r_perp * np.exp(1j * phase)
    assert abs(e["field"][0, 0] - expect) <= 2e-8 * abs(expect)
    # plane x-z: x polarisation in the plane of incidence, field transverse to the ray
    e = _emit(O.trace_rays(_sphere(), st, [(y, 0.0)])[0], 0)
    f = e["field"][0]
    assert np.linalg.norm(f) == pytest.approx(amp * abs(r_par), rel=2e-8)
    assert abs(f @ e["dir"]) <= 1e-12 * np.linalg.norm(f)


def _exact_near_field(p, R, theta, lam):
    """R e^{-ikR} E at (theta, 90 deg) from p-order rays of the plane x = 0,
    each root-found (bisection on its direction of M) on the per-ray trace;
    its tangential part projected on (e_theta, e_phi)."""
    P = _sphere()
    S = O.setup(lam, 1, p, p, 16, observation_radius=R)
    ys = np.linspace(-A * (1 - 1e-9), A * (1 - 1e-9), 8001)

    def trace(y):
        rays = O.trace_rays(P, S, np.stack([np.zeros_like(y), y], 1))
        u = np.array([rays[i].emit[p].obs[:] for i in range(y.size)])
        v = np.array([rays[i].emit[p].valid for i in range(y.size)])
        f = np.array([np.array(rays[i].emit[p].field[:6]).reshape(3, 2) for i in range(y.size)])
        return np.arctan2(u[:, 1], u[:, 2]), v, f[..., 0] + 1j * f[..., 1]

    psi, v, _ = trace(ys)
    F = np.zeros((theta.size, 2), complex)
    for j, th in enumerate(theta):
        g = np.angle(np.exp(1j * (psi - th)))
        idx = np.where(v[:-1] & v[1:] & (np.sign(g[:-1]) != np.sign(g[1:])) & (np.abs(g[:-1]) < 0.5))[0]
        for i in idx:
            lo, hi, glo = ys[i], ys[i + 1], g[i]
            for _ in range(55):
                mid = 0.5 * (lo + hi)
                gm = np.angle(np.exp(1j * (trace(np.array([mid]))[0][0] - th)))
                if np.sign(gm) == np.sign(glo):
                    lo, glo = mid, gm
                else:
                    hi = mid
            f = trace(np.array([0.5 * (lo + hi)]))[2][0]
            F[j, 0] += f @ np.array([0.0, np.cos(th), -np.sin(th)])
            F[j, 1] += f @ np.array([-1.0, 0.0, 0.0])
    return F


@pytest.mark.parametrize("p,R,t_lo,t_hi,Ns,bar", [(0, 150.0, 35.0, 80.0, (1024, 2048), 2e-4),
                                                   (1, 400.0, 6.0, 30.0, (512, 1024), 5e-5)])
def test_assembly_at_finite_distance_converges_to_the_ray_sum(p, R, t_lo, t_hi, Ns, bar):
    """The interpolated field on the sphere converges to the exact ray sum at
    second order in the ray spacing: the carry between a vertex and a node has
    the ray's own phase gradient on the sphere (a carry with another gradient
    converges at first order only).  lambda = 6.328 um (k a ~ 50) reaches the
    asymptotic rate at these grids; at k a ~ 500 the second-order phase term
    k a h^2 keeps the error pre-asymptotic to N ~ 1000 even in the far field."""
    lam = 6.328
    th_deg = np.arange(t_lo, t_hi + 1e-9, 3.0)
    Fe = _exact_near_field(p, R, np.radians(th_deg), lam)
    assert np.abs(Fe).max(axis=1).min() > 0  # every node is reached
    errs = []
    for N in Ns:
        r = O.farfield(_sphere(), O.setup(lam, 1, p, p, N, observation_radius=R), th_deg, np.array([90.0]))
        F = r["field"][0, :, :, 0].T
        errs.append(np.abs(F - Fe).max() / np.abs(Fe).max())
    assert errs[1] < bar, errs
    assert errs[0] / errs[1] > 3.0, errs


def test_far_observation_converges_to_the_far_field():
    """R -> infinity: the field tends to the far field F with an error falling
    as 1/R (the phase term k (|r_exit|^2 - (d.r_exit)^2) / 2R and the offset
    of M's direction from d, about |r_exit| / R)."""
    part = O.particle((40.0, 36.0, 32.0), (20, 30, 40), M)
    th = np.arange(20.0, 170.0, 7.0)
    ph = np.arange(0.0, 360.0, 15.0)
    ref = O.farfield(part, O.setup(LAM, 1, 0, 1, 96), th, ph)["field"]
    med, mx = [], []
    for R in (1e5, 1e6, 1e7):
        F = O.farfield(part, O.setup(LAM, 1, 0, 1, 96, observation_radius=R), th, ph)["field"]
        d = np.abs(F - ref) / np.abs(ref).max()
        med.append(np.median(d))
        mx.append(d.max())
    assert mx[2] < 1e-3 and 0.05 < mx[2] / mx[1] < 0.2, mx
    assert 0.08 < med[1] / med[0] < 0.12 and 0.08 < med[2] / med[1] < 0.12, med


def test_point_source_and_finite_distance_combine_reciprocally():
    """Reciprocity of reflection off a sphere on the axis: a source at distance
    z_s observed back at R equals a source at R observed at z_s, once each is
    divided by its own normalisation (unit incident amplitude at the centre
    times z_s; R e^{-ikR} on the observation side)."""
    a = _emit(O.trace_rays(_sphere(), O.setup(LAM, 1, 0, 0, 8, source_distance=120.0, observation_radius=700.0),
                           [(0.0, 0.0)])[0], 0)
    b = _emit(O.trace_rays(_sphere(), O.setup(LAM, 1, 0, 0, 8, source_distance=700.0, observation_radius=120.0),
                           [(0.0, 0.0)])[0], 0)
    ga = a["field"][0, 0] / (120.0 * 700.0)
    gb = b["field"][0, 0] / (700.0 * 120.0)
    assert abs(ga - gb) <= 1e-12 * abs(ga)


@pytest.mark.parametrize("R", [-1.0, 30.0, 60.0])
def test_observation_inside_the_bounding_sphere_is_rejected(R):
    part = O.particle((60.0, 50.0, 40.0), (0, 0, 0), M)
    with pytest.raises(ValueError):
        O.trace_rays(part, O.setup(LAM, 1, 0, 1, 8, observation_radius=R), [(0.0, 0.0)])
