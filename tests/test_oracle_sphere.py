"""Pins of the oracle's per-ray trace on the sphere, where geometric optics has
closed forms (van de Hulst, Light Scattering by Small Particles, ch. 12; cited
by the paper in its amplitude and phase paragraphs):

* deflection  Theta_p = 2 theta_i - 2 p theta_r + (p - 1) pi
* far-field intensity (divergence) a^2 sin(ti) cos(ti) / (sin(theta) |dTheta/dti|) |eps|^2
* path phase  2 x (p m cos(theta_r) - cos(theta_i))  (phase referenced to the centre)
* focal-line count from the sagittal (axis crossings) and meridional (neighbour
  rays crossing) foci of an independent 2-D trace
* p = 0: |F|^2 = a^2 |r|^2 / 4 (isotropic external reflection)
"""
import numpy as np
import pytest

A = 50.0
M = 1.333
LAM = 0.6328
K = 2 * np.pi / LAM


def _trace_2d(a, m, b, p):
    """Independent 2-D trace in the (y, z) plane of a ray entering at y=b
    moving along +z: returns interaction points and the direction after each
    interaction (last one = exit direction of order p)."""
    def circle_hit(P, d):
        # second intersection of P + s d with |x| = a, P on or outside the circle
        B = 2 * P @ d
        C = P @ P - a * a
        disc = B * B - 4 * C
        return (-B + np.sqrt(disc)) / 2 if C <= 1e-9 * a * a else (-B - np.sqrt(disc)) / 2

    def snell2(d, n_out_vec, n1, n2, reflect):
        nu = n_out_vec if d @ n_out_vec > 0 else -n_out_vec
        c = d @ nu
        if reflect:
            return d - 2 * c * nu
        mr = n2 / n1
        ct = np.sqrt(1 - (1 - c * c) / (mr * mr))
        return (d - c * nu) / mr + ct * nu

    P = np.array([b, -np.sqrt(a * a - b * b)])
    d = np.array([0.0, 1.0])
    pts, dirs = [P], []
    if p == 0:
        dirs.append(snell2(d, P / a, 1, m, True))
        return pts, dirs
    d = snell2(d, P / a, 1, m, False)
    dirs.append(d)
    for q in range(p):
        s = circle_hit(P, d)
        P = P + s * d
        pts.append(P)
        last = q == p - 1
        d = snell2(d, P / a, m, 1, False) if last else snell2(d, P / a, m, m, True)
        dirs.append(d)
    return pts, dirs


def _focal_count_2d(a, m, b, p, h=1e-5):
    pts, dirs = _trace_2d(a, m, b, p)
    pp, dp = _trace_2d(a, m, b + h, p)
    pm, dm = _trace_2d(a, m, b - h, p)
    count = 0
    nseg = len(pts)
    for q in range(nseg):
        C0, d0 = pts[q], dirs[q]
        far = q == nseg - 1
        L = np.inf if far else np.linalg.norm(pts[q + 1] - C0)
        # sagittal focus: the ray crosses the symmetry axis y = 0
        if abs(d0[0]) > 0:
            s = -C0[0] / d0[0]
            if 0 < s < L:
                count += 1
        # meridional focus: neighbouring rays cross (finite-difference tube width)
        n0 = np.array([-d0[1], d0[0]])

        def offset_coeffs(Pn, dn):
            # offset(s) = alpha + beta * s of the neighbour ray measured across the central ray
            t0 = -(Pn - C0) @ d0 / (dn @ d0)
            t1 = 1.0 / (dn @ d0)
            alpha = (Pn + t0 * dn - C0) @ n0
            beta = (t1 * dn - d0) @ n0
            return alpha, beta
        ap, bp = offset_coeffs(pp[q], dp[q])
        am, bm = offset_coeffs(pm[q], dm[q])
        alpha, beta = (ap - am) / (2 * h), (bp - bm) / (2 * h)
        if beta != 0:
            s = -alpha / beta
            if 0 < s < L:
                count += 1
    return count


def _closed_forms(b, p):
    ti = np.arcsin(b / A)
    tr = np.arcsin(np.sin(ti) / M)
    Th = 2 * ti - 2 * p * tr + (p - 1) * np.pi
    ths = np.arccos(np.cos(Th))
    dTh = 2 - 2 * p * np.cos(ti) / (M * np.cos(tr))
    I = A * A * np.sin(ti) * np.cos(ti) / (np.sin(ths) * abs(dTh))
    phase = 2 * K * A * (p * M * np.cos(tr) - np.cos(ti))
    return ti, tr, ths, I, phase


def _fresnel_perp(n1, n2, ci):
    ct = np.sqrt(1 - (n1 / n2) ** 2 * (1 - ci * ci))
    r = (n1 * ci - n2 * ct) / (n1 * ci + n2 * ct)
    t = 2 * n1 * ci / (n1 * ci + n2 * ct)
    return r, t


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_sphere_per_ray_closed_forms(oracle, p):
    P = oracle.particle((A, A, A), (0, 0, 0), M)
    S = oracle.setup(LAM, 1, 0, 3, 16)
    # rays in the plane x = 0 (perpendicular polarisation), away from the rainbow rays
    cr2 = np.sqrt((M * M - 1) / 3)
    cr3 = np.sqrt((M * M - 1) / 8)
    b_rb = [A * np.sqrt(1 - cr2 ** 2), A * np.sqrt(1 - cr3 ** 2)]
    bs = np.linspace(0.01, 0.99, 199) * A
    bs = bs[[all(abs(b - r) > 0.3 for r in b_rb) for b in bs]]
    rays = oracle.trace_rays(P, S, np.stack([np.zeros_like(bs), bs], 1))
    for i, b in enumerate(bs):
        e = oracle.ray_emit(rays[i], p)
        assert e["valid"]
        ti, tr, ths, I, phase = _closed_forms(b, p)
        # deflection
        assert abs(np.arccos(np.clip(e["dir"][2], -1, 1)) - ths) < 1e-12
        # divergence factor: amp^2 = I / |eps|^2 (eps carried separately in the Jones matrix)
        assert abs(e["amp"] ** 2 / I - 1) < 1e-11
        # focal lines from an independent 2-D construction
        nf = _focal_count_2d(A, M, b, p)
        assert e["nf"] == nf, (b, p, e["nf"], nf)
        # path phase (with the focal-line term removed)
        assert abs(e["phase"] + e["nf"] * np.pi / 2 - phase) < 1e-9
        # Fresnel product for the perpendicular channel (no cross-polarisation in a symmetry plane)
        r01, t01 = _fresnel_perp(1, M, np.cos(ti))
        r11, t10 = _fresnel_perp(M, 1, np.cos(tr))
        eps = r01 if p == 0 else t01 * t10 * r11 ** (p - 1)
        fx = e["field"][0, 0]
        expect = np.sqrt(I) * np.exp(1j * (phase - nf * np.pi / 2)) * eps
        assert abs(fx - expect) < 1e-9 * abs(expect)
        assert abs(e["field"][0, 1]) < 1e-12 * abs(expect) and abs(e["field"][0, 2]) < 1e-12 * abs(expect) + 1e-12


def test_sphere_focal_counts_match_known_pattern(oracle):
    """Sagittal + meridional focal lines: p=0 none, p=1 two, p=2 two (inner
    branch) / three (outer branch), p=3 four / five."""
    cr2 = np.sqrt((M * M - 1) / 3)
    b2 = A * np.sqrt(1 - cr2 ** 2)
    cr3 = np.sqrt((M * M - 1) / 8)
    b3 = A * np.sqrt(1 - cr3 ** 2)
    cases = [(0, 0.5 * A, 0), (1, 0.5 * A, 2), (2, 0.5 * b2, 2), (2, 0.5 * (b2 + A), 3),
             (3, 0.5 * b3, 4), (3, 0.5 * (b3 + A), 5)]
    P = oracle.particle((A, A, A), (0, 0, 0), M)
    S = oracle.setup(LAM, 1, 0, 3, 16)
    for p, b, expect in cases:
        assert _focal_count_2d(A, M, b, p) == expect
        ray = oracle.trace_rays(P, S, np.array([[0.0, b]]))[0]
        assert oracle.ray_emit(ray, p)["nf"] == expect


def test_sphere_p0_isotropic(oracle):
    """|F_0|^2 = a^2 |r|^2 / 4 for external reflection, any incidence plane."""
    P = oracle.particle((A, A, A), (0, 0, 0), M)
    S = oracle.setup(LAM, 2, 0, 0, 16)
    rng = np.random.default_rng(5)
    xy = rng.uniform(-A, A, size=(200, 2))
    xy = xy[np.hypot(xy[:, 0], xy[:, 1]) < 0.99 * A]
    rays = oracle.trace_rays(P, S, xy)
    for i in range(xy.shape[0]):
        e = oracle.ray_emit(rays[i], 0)
        assert abs(e["amp"] - A / 2) < 1e-12 * A
        ci = np.sqrt(1 - (np.hypot(*xy[i]) / A) ** 2)
        r_perp, _ = _fresnel_perp(1, M, ci)
        # perpendicular fraction of x-polarised light: sin^2 of the incidence-plane azimuth
        psi = np.arctan2(xy[i, 1], xy[i, 0])
        j = e["jones"]
        assert abs(abs(j[0, 0]) - abs(r_perp * np.sin(psi))) < 1e-12


def test_sphere_no_cross_polarisation_in_parallel_plane(oracle):
    """Rays in the incidence plane y = 0 keep x polarisation in the scattering
    plane (parallel channel): the field has no y component."""
    P = oracle.particle((A, A, A), (0, 0, 0), M)
    S = oracle.setup(LAM, 1, 0, 3, 16)
    bs = np.linspace(0.05, 0.95, 19) * A
    rays = oracle.trace_rays(P, S, np.stack([bs, np.zeros_like(bs)], 1))
    for i in range(bs.size):
        for p in range(4):
            e = oracle.ray_emit(rays[i], p)
            f = e["field"][0]
            assert abs(f[1]) <= 1e-12 * np.linalg.norm(f) + 1e-300
            # the field is transverse to the exit direction
            assert abs(np.dot(f, e["dir"])) <= 1e-12 * np.linalg.norm(f) + 1e-300
