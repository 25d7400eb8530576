"""Pins of the oracle's corrections (readings R12, R13 of the oracle):

* the special functions they use against scipy's (an independent library);
* the fold-caustic (uniform Airy) form against the paper's Table 1 main bow
  (K = 0, printed in italics: RTW with the wave correction) -- geometric
  optics has no maximum there;
* far from the fold the uniform form tends to the geometric-optics sum;
* the forward-diffraction term against a brute-force quadrature of the
  shadow's Fraunhofer integral, and against the energy it must carry (the
  shadow's area, by Parseval's theorem).
"""
import os

import numpy as np
import pytest
from scipy import special

M = 1.333
LAM = 0.6328
HERE = os.path.dirname(os.path.abspath(__file__))


def test_airy_on_the_negative_axis_matches_scipy(oracle):
    z = np.concatenate([np.linspace(0.0, 40.0, 801), [9.999, 10.0, 10.001, 100.0, 400.0]])
    for x in z:
        ai, aip = oracle.airy_neg(x)
        ref = special.airy(-x)
        scale = abs(ref[0]) + abs(ref[1]) * x ** -0.5 if x > 0 else 1.0
        assert abs(ai - ref[0]) < 1e-11 * scale, (x, ai, ref[0])
        assert abs(aip - ref[1]) < 1e-11 * (abs(ref[1]) + abs(ref[0]) * x ** 0.5 + 1e-300), (x, aip, ref[1])


def test_bessel_j1_matches_scipy(oracle):
    for x in np.concatenate([np.linspace(0.0, 80.0, 1601), [24.999, 25.0, 25.001, 1e3, 5e3 + 0.3, -7.5]]):
        assert abs(oracle.bessel_j1(x) - special.j1(x)) < 1e-14, x


def _golden_k0():
    rows = []
    with open(os.path.join(HERE, "golden", "table1_supernumerary_peaks.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                a, K, th = line.split()
                if int(K) == 0:
                    rows.append((float(a), float(th)))
    return rows


@pytest.mark.parametrize("a,N,step", [(50.0, 512, 0.005), (500.0, 1024, 0.002)])
def test_main_bow_of_table1(oracle, a, N, step):
    """The first maximum past the caustic band of the rainbow, perpendicular
    channel (x-polarised light in the plane phi = 90 deg), p = 2 only."""
    paper = dict(_golden_k0())[a]
    P = oracle.particle((a, a, a), (0, 0, 0), M)
    S = oracle.setup(LAM, 1, 2, 2, N, corrections=oracle.CAUSTIC)
    th = np.arange(137.0, 141.0, step)
    r = oracle.farfield(P, S, th, np.array([90.0]))
    I = (np.abs(r["field"][0]) ** 2).sum(0)[:, 0]
    ok = (r["flags"][:, 0] & 2) == 0
    first = np.argmax(ok & (th > 137.0) & (r["ncontrib"][:, 0] == 2))
    pk = [i for i in range(first + 1, I.size - 1) if I[i] > I[i - 1] and I[i] >= I[i + 1]]
    i = pk[0]
    t = np.linspace(th[i] - step, th[i] + step, 81)
    rr = oracle.farfield(P, S, t, np.array([90.0]))
    t_peak = t[np.argmax((np.abs(rr["field"][0]) ** 2).sum(0)[:, 0])]
    assert abs(t_peak - paper) < 0.02, (a, t_peak, paper)
    # geometric optics alone has no maximum there: its intensity only falls
    go = oracle.farfield(P, oracle.setup(LAM, 1, 2, 2, N), th[first:i + 20], np.array([90.0]))
    Ig = (np.abs(go["field"][0]) ** 2).sum(0)[:, 0]
    assert np.all(np.diff(Ig[: i - first + 10]) < 0)


def test_uniform_form_tends_to_the_ray_sum_far_from_the_fold(oracle):
    """The Airy form of a fold pair differs from the two-ray sum by terms of
    relative order 1 / Delta (Delta: half the pair's path-phase difference),
    so the difference falls as the node moves away from the rainbow."""
    P = oracle.particle((50.0, 50.0, 50.0), (0, 0, 0), M)
    th = np.arange(138.5, 165.0, 0.5)
    ph = np.array([90.0])
    go = oracle.farfield(P, oracle.setup(LAM, 1, 2, 2, 512), th, ph)["field"][0, :, :, 0]
    cf = oracle.farfield(P, oracle.setup(LAM, 1, 2, 2, 512, corrections=oracle.CAUSTIC), th, ph)["field"][0, :, :, 0]
    rel = np.abs(cf - go).max(0) / np.abs(go).max(0)
    near, far = rel[th < 140.0].max(), rel[th > 155.0].max()
    assert near > 1e-1 and far < 2e-2 and far < near / 10, (near, far)


def test_dark_side_of_the_fold_stays_empty(oracle):
    P = oracle.particle((50.0, 50.0, 50.0), (0, 0, 0), M)
    th = np.arange(130.0, 137.5, 0.25)
    r = oracle.farfield(P, oracle.setup(LAM, 2, 2, 2, 256, corrections=oracle.CAUSTIC), th, np.arange(0.0, 360, 30.0))
    assert np.abs(r["field"]).max() == 0.0


def _shadow(oracle, axes, euler):
    """x-y block of R diag(a^2, b^2, c^2) R^T, R from the oracle's rotation
    convention (Z-Y-Z, body -> lab), rebuilt here from the Euler angles."""
    al, be, ga = np.radians(euler)
    Rz = lambda t: np.array([[np.cos(t), -np.sin(t), 0], [np.sin(t), np.cos(t), 0], [0, 0, 1]])
    Ry = lambda t: np.array([[np.cos(t), 0, np.sin(t)], [0, 1, 0], [-np.sin(t), 0, np.cos(t)]])
    R = Rz(al) @ Ry(be) @ Rz(ga)
    S = R @ np.diag(np.square(axes)) @ R.T
    return S[:2, :2]


def _diffraction_only(oracle, axes, euler, th, ph, n_pol=2):
    """The diffraction term alone: the far field with the correction minus without."""
    P = oracle.particle(axes, euler, M)
    a = oracle.farfield(P, oracle.setup(LAM, n_pol, 0, 0, 16, corrections=oracle.DIFFRACTION), th, ph)["field"]
    b = oracle.farfield(P, oracle.setup(LAM, n_pol, 0, 0, 16), th, ph)["field"]
    return a - b


def test_diffraction_matches_a_quadrature_of_the_shadow(oracle):
    """Fraunhofer integral (i k / 2 pi) int_shadow exp(-i k n_t.rho) d^2 rho by
    brute force on a fine grid over the projected ellipse."""
    axes, euler = (6.0, 4.0, 3.0), (30.0, 50.0, 10.0)
    k = 2 * np.pi / LAM
    S2 = _shadow(oracle, axes, euler)
    Sinv = np.linalg.inv(S2)
    ext = np.sqrt(np.diag(S2))
    h = 0.01
    xs = np.arange(-ext[0], ext[0] + h, h)
    ys = np.arange(-ext[1], ext[1] + h, h)
    X, Y = np.meshgrid(xs, ys)
    inside = (Sinv[0, 0] * X * X + 2 * Sinv[0, 1] * X * Y + Sinv[1, 1] * Y * Y) <= 1.0
    xi, yi = X[inside], Y[inside]
    th = np.array([0.0, 2.0, 5.0, 9.0])
    ph = np.array([0.0, 40.0, 135.0])
    D = _diffraction_only(oracle, axes, euler, th, ph)
    for i, t in enumerate(np.radians(th)):
        for j, f in enumerate(np.radians(ph)):
            nx, ny = np.sin(t) * np.cos(f), np.sin(t) * np.sin(f)
            F = 1j * k / (2 * np.pi) * np.exp(-1j * k * (nx * xi + ny * yi)).sum() * h * h
            # the quadrature's pixelated rim errs by ~1e-3 of the forward amplitude
            tol = 2e-3 * k / (2 * np.pi) * inside.sum() * h * h
            # x polarisation (cos phi, -sin phi), y polarisation (sin phi, cos phi)
            assert np.allclose(D[0, :, i, j], F * np.array([np.cos(f), -np.sin(f)]), rtol=0, atol=tol), (t, f)
            assert np.allclose(D[1, :, i, j], F * np.array([np.sin(f), np.cos(f)]), rtol=0, atol=tol), (t, f)


def test_diffraction_carries_the_shadow_area(oracle):
    """Parseval: the diffracted power over all directions equals the shadow's
    area; for k a >> 1 it lies within a few degrees of forward."""
    axes, euler = (30.0, 25.0, 20.0), (10.0, 70.0, -40.0)
    S2 = _shadow(oracle, axes, euler)
    area = np.pi * np.sqrt(np.linalg.det(S2))
    th = np.arange(0.0, 8.0, 0.01)
    ph = np.arange(0.0, 360.0, 2.0)
    D = _diffraction_only(oracle, axes, euler, th, ph, n_pol=1)
    I = (np.abs(D[0]) ** 2).sum(0)
    dth, dph = np.radians(0.01), np.radians(2.0)
    power = (I * np.sin(np.radians(th))[:, None]).sum() * dth * dph
    assert abs(power / area - 1.0) < 0.02, power / area
    # forward amplitude: i k area / 2 pi, along the incident polarisation
    assert np.allclose(D[0, :, 0, 0], [1j * (2 * np.pi / LAM) * area / (2 * np.pi), 0.0], rtol=1e-12, atol=1e-9)
