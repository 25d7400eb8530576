"""Pins of the oracle's interface physics: Fresnel coefficients (Eq. 8) and
vector Snell (Eq. 4), against identities the paper's equations must satisfy.

None of these re-type the oracle's formulas: they check energy conservation,
Brewster's zero, the normal-incidence and grazing limits, and Snell's law on
the traced polyline using the ellipsoid normal.
"""
import numpy as np
import pytest


@pytest.mark.parametrize("m_rel", [1.333, 1.5, 1 / 1.333, 1 / 1.5, 2.4])
def test_fresnel_energy_conservation(oracle, m_rel):
    """R + T = 1 per polarisation with T = Re(k_rn)/k_in |t|^2 (Eq. 8)."""
    for ci in np.linspace(0.01, 1.0, 97):
        f = oracle.fresnel(m_rel, ci)
        ratio = f["krn_over_kin"]
        for r, t in ((f["r_perp"], f["t_perp"]), (f["r_par"], f["t_par"])):
            T = ratio.real * abs(t) ** 2
            assert abs(abs(r) ** 2 + T - 1.0) < 1e-14


@pytest.mark.parametrize("m_rel", [1.333, 1 / 1.333, 1.7])
def test_fresnel_brewster_zero_and_limits(oracle, m_rel):
    # Brewster: tan(theta_B) = m_rel  => r_par = 0 (Table 1 discussion: phase jump of the parallel channel)
    thb = np.arctan(m_rel)
    f = oracle.fresnel(m_rel, np.cos(thb))
    assert abs(f["r_par"]) < 1e-14
    # r_par changes sign across Brewster's angle
    f1 = oracle.fresnel(m_rel, np.cos(thb - 0.01))
    f2 = oracle.fresnel(m_rel, np.cos(thb + 0.01))
    assert np.sign(f1["r_par"].real) != np.sign(f2["r_par"].real)
    # normal incidence: r_perp = -r_par = (1 - m)/(1 + m), t_perp = t_par = 2/(1+m)
    f = oracle.fresnel(m_rel, 1.0)
    assert abs(f["r_perp"] - (1 - m_rel) / (1 + m_rel)) < 1e-15
    assert abs(f["r_par"] + f["r_perp"]) < 1e-15
    assert abs(f["t_perp"] - 2 / (1 + m_rel)) < 1e-15
    assert abs(f["t_par"] - 2 / (1 + m_rel)) < 1e-15
    if m_rel > 1:
        # grazing incidence on a denser medium: both reflect with -1
        f = oracle.fresnel(m_rel, 1e-9)
        assert abs(f["r_perp"] + 1) < 1e-8 and abs(f["r_par"] + 1) < 1e-8


def test_fresnel_total_internal_reflection(oracle):
    m_rel = 1 / 1.333
    crit = np.arcsin(m_rel)
    for th in np.linspace(crit + 1e-3, np.pi / 2 - 1e-3, 20):
        f = oracle.fresnel(m_rel, np.cos(th))
        assert abs(abs(f["r_perp"]) - 1) < 1e-14 and abs(abs(f["r_par"]) - 1) < 1e-14
        assert f["krn_over_kin"].real == 0.0 and f["krn_over_kin"].imag > 0  # evanescent, decaying


def test_snell_on_polyline(oracle):
    """Eq. 4 on every interaction of traced ellipsoid rays: tangential wave
    vectors are continuous, the reflected direction mirrors the incident one,
    and every direction is a unit vector."""
    from paper_2403_13856_amd.inputs import random_ellipsoid
    rng = np.random.default_rng(1)
    for trial in range(4):
        axes, euler, m = random_ellipsoid(rng)
        P = oracle.particle(axes, euler, m)
        S = oracle.setup(0.6328, 2, 0, 4, 16)
        L = oracle.grid_halfwidth(P)
        xy = rng.uniform(-L, L, size=(64, 2))
        rays = oracle.trace_rays(P, S, xy)
        Rm = _rotation(euler)
        A = np.diag(1.0 / np.array(axes) ** 2)
        for i in range(64):
            ray = rays[i]
            if not ray.active:
                continue
            hits = [np.array(ray.hit[q][:]) for q in range(ray.n_hits)]
            dirs = [np.array([0.0, 0.0, 1.0])] + [np.array(ray.dir_cont[q][:]) for q in range(ray.n_hits)]
            n_in = 1.0
            for q in range(ray.n_hits - 1):
                rb = Rm.T @ hits[q]
                assert abs(rb @ A @ rb - 1.0) < 1e-12  # the hit lies on the ellipsoid
                nb = A @ rb
                nl = Rm @ (nb / np.linalg.norm(nb))
                d_in, d_out = dirs[q], dirs[q + 1]
                assert abs(np.linalg.norm(d_out) - 1) < 1e-14
                # the continuing branch is refracted at q=0, reflected afterwards
                n_out = m if q == 0 else n_in
                tan_in = n_in * (d_in - np.dot(d_in, nl) * nl)
                tan_out = n_out * (d_out - np.dot(d_out, nl) * nl)
                assert np.linalg.norm(tan_in - tan_out) < 1e-13
                if q > 0:  # reflection: normal component flips
                    assert abs(np.dot(d_in, nl) + np.dot(d_out, nl)) < 1e-13
                # the next hit lies on the straight continuation
                seg = hits[q + 1] - hits[q]
                assert np.linalg.norm(np.cross(seg / np.linalg.norm(seg), d_out)) < 1e-12
                n_in = n_out
            # exit (transmitted) order p >= 1: check Snell on the last emission too
            for p in range(1, ray.n_hits):
                e = oracle.ray_emit(ray, p)
                if not e["valid"]:
                    continue
                rb = Rm.T @ e["rexit"]
                nb = A @ rb
                nl = Rm @ (nb / np.linalg.norm(nb))
                d_in = dirs[p]
                tan_in = m * (d_in - np.dot(d_in, nl) * nl)
                tan_out = e["dir"] - np.dot(e["dir"], nl) * nl
                assert np.linalg.norm(tan_in - tan_out) < 1e-13
                assert np.linalg.norm(e["rexit"] - hits[p]) < 1e-12


def _rotation(euler_deg):
    a, b, g = np.radians(euler_deg)
    Rz = lambda t: np.array([[np.cos(t), -np.sin(t), 0], [np.sin(t), np.cos(t), 0], [0, 0, 1]])
    Ry = lambda t: np.array([[np.cos(t), 0, np.sin(t)], [0, 1, 0], [-np.sin(t), 0, np.cos(t)]])
    return Rz(a) @ Ry(b) @ Rz(g)
