"""Pin of the oracle's weak absorption (reading R14: every internal segment of
length L scales the field by exp(-k m_im L); Snell and Eq. 8 use the real part).
On a sphere of radius a every internal chord of a ray of impact parameter b
has length 2 a cos(theta_r), sin(theta_r) = b / (a m), so order p's field is
that of the transparent sphere times exp(-k m_im p 2 a cos(theta_r)) exactly."""
import numpy as np

A, M, LAM = 50.0, 1.333, 0.6328


def test_sphere_orders_attenuate_by_their_chords(oracle):
    k = 2 * np.pi / LAM
    m_im = 2e-4
    b = np.array([0.05, 0.3, 0.6, 0.85, 0.97]) * A
    xy = np.stack([b * np.cos(0.7), b * np.sin(0.7)], 1)
    S = oracle.setup(LAM, 2, 0, 3, 16)
    clear = oracle.trace_rays(oracle.particle((A, A, A), (0, 0, 0), M), S, xy)
    lossy = oracle.trace_rays(oracle.particle((A, A, A), (0, 0, 0), M, m_im), S, xy)
    cos_r = np.sqrt(1.0 - (b / (A * M)) ** 2)
    for i in range(b.size):
        for p in range(4):
            f0 = np.array(clear[i].emit[p].field[:])
            f1 = np.array(lossy[i].emit[p].field[:])
            expect = np.exp(-k * m_im * p * 2 * A * cos_r[i])
            assert np.allclose(f1, expect * f0, rtol=1e-12, atol=1e-14 * np.abs(f0).max()), (i, p)
            # the divergence amplitude and the phase are those of the real index
            assert clear[i].emit[p].amp == lossy[i].emit[p].amp
            assert clear[i].emit[p].phase == lossy[i].emit[p].phase


def test_zero_absorption_is_the_transparent_particle(oracle):
    th, ph = np.arange(0.0, 181.0, 5.0), np.arange(0.0, 360.0, 15.0)
    S = oracle.setup(LAM, 2, 0, 3, 48)
    a = oracle.farfield(oracle.particle((40.0, 35.0, 30.0), (10, 20, 30), M), S, th, ph)["field"]
    b = oracle.farfield(oracle.particle((40.0, 35.0, 30.0), (10, 20, 30), M, 0.0), S, th, ph)["field"]
    assert np.array_equal(a, b)
