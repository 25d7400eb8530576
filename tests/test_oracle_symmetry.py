"""Symmetry and covariance pins of the oracle's per-ray trace (frames, body <->
lab rotations, basis independence of Eq. 3, Jones bookkeeping).

S1  Euler (a, b, g) == (a+180, -b, g+180) (same rotation) and == (a, b, g+180)
    (the ellipsoid is invariant under a half turn about its own z axis).
S2  axis-aligned ellipsoid: mirror y -> -y maps the ray at (x, y) onto the ray
    at (x, -y); the x-polarised field mirrors with it.
S3  spheroid with its symmetry axis along k: a quarter turn about z maps the
    x-polarised ray at xi onto the y-polarised ray at R xi.
S5  permuting the semi-axes with the compensating rotation changes nothing.
S6  scaling a, b, c, lambda by s scales the far-field amplitude by s and leaves
    directions, phases and focal-line counts unchanged.
"""
import numpy as np
import pytest

LAM = 0.6328


def _emits(oracle, P, S, xy, p_max):
    rays = oracle.trace_rays(P, S, xy)
    out = []
    for i in range(xy.shape[0]):
        out.append([oracle.ray_emit(rays[i], p) for p in range(p_max + 1)])
    return out


def _field_close(f1, f2, tol=1e-11):
    scale = max(np.abs(f1).max(), np.abs(f2).max(), 1e-300)
    return np.abs(f1 - f2).max() <= tol * scale


def _sample(L, n=60, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(-L, L, size=(n, 2))


@pytest.mark.parametrize("euler", [(30.0, 20.0, 10.0), (-70.0, 110.0, 45.0)])
def test_s1_euler_equivalences(oracle, euler):
    axes, m, p_max = (60.0, 50.0, 40.0), 1.333, 3
    S = oracle.setup(LAM, 2, 0, p_max, 16)
    P0 = oracle.particle(axes, euler, m)
    xy = _sample(oracle.grid_halfwidth(P0))
    ref = _emits(oracle, P0, S, xy, p_max)
    a, b, g = euler
    for alt in [(a + 180.0, -b, g + 180.0), (a, b, g + 180.0)]:
        got = _emits(oracle, oracle.particle(axes, alt, m), S, xy, p_max)
        for er, eg in zip(ref, got):
            for p in range(p_max + 1):
                assert er[p]["valid"] == eg[p]["valid"]
                if not er[p]["valid"]:
                    continue
                assert er[p]["nf"] == eg[p]["nf"]
                assert np.abs(er[p]["dir"] - eg[p]["dir"]).max() < 1e-12
                assert abs(er[p]["amp"] - eg[p]["amp"]) < 1e-10 * er[p]["amp"]
                assert abs(er[p]["phase"] - eg[p]["phase"]) < 1e-9
                assert _field_close(er[p]["field"], eg[p]["field"], 1e-9)


def test_s2_mirror_symmetry(oracle):
    axes, m, p_max = (60.0, 50.0, 40.0), 1.333, 3
    S = oracle.setup(LAM, 1, 0, p_max, 16)
    P = oracle.particle(axes, (0, 0, 0), m)
    xy = _sample(oracle.grid_halfwidth(P), seed=3)
    mir = xy * np.array([1.0, -1.0])
    e1 = _emits(oracle, P, S, xy, p_max)
    e2 = _emits(oracle, P, S, mir, p_max)
    Mm = np.diag([1.0, -1.0, 1.0])
    for a, b in zip(e1, e2):
        for p in range(p_max + 1):
            assert a[p]["valid"] == b[p]["valid"]
            if not a[p]["valid"]:
                continue
            assert np.abs(Mm @ a[p]["dir"] - b[p]["dir"]).max() < 1e-12
            assert a[p]["nf"] == b[p]["nf"]
            assert _field_close(Mm @ a[p]["field"][0], b[p]["field"][0])


def test_s3_polarisation_rotation_spheroid(oracle):
    axes, m, p_max = (55.0, 55.0, 45.0), 1.333, 3
    S = oracle.setup(LAM, 2, 0, p_max, 16)
    P = oracle.particle(axes, (0, 0, 0), m)
    xy = _sample(oracle.grid_halfwidth(P), seed=4)
    Rq = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])  # +90 deg about z
    rot = xy @ Rq[:2, :2].T
    e1 = _emits(oracle, P, S, xy, p_max)
    e2 = _emits(oracle, P, S, rot, p_max)
    for a, b in zip(e1, e2):
        for p in range(p_max + 1):
            if not a[p]["valid"]:
                assert not b[p]["valid"]
                continue
            assert np.abs(Rq @ a[p]["dir"] - b[p]["dir"]).max() < 1e-12
            # x-polarised at xi  ->  y-polarised at R xi
            assert _field_close(Rq @ a[p]["field"][0], b[p]["field"][1])


def test_s5_axis_permutation(oracle):
    m, p_max = 1.4, 3
    S = oracle.setup(LAM, 2, 0, p_max, 16)
    P1 = oracle.particle((60.0, 50.0, 40.0), (0, 0, 0), m)
    P2 = oracle.particle((50.0, 60.0, 40.0), (90.0, 0, 0), m)  # body x -> lab y
    xy = _sample(oracle.grid_halfwidth(P1), seed=5)
    assert abs(oracle.grid_halfwidth(P1) - oracle.grid_halfwidth(P2)) < 1e-12
    e1 = _emits(oracle, P1, S, xy, p_max)
    e2 = _emits(oracle, P2, S, xy, p_max)
    for a, b in zip(e1, e2):
        for p in range(p_max + 1):
            assert a[p]["valid"] == b[p]["valid"]
            if not a[p]["valid"]:
                continue
            assert np.abs(a[p]["dir"] - b[p]["dir"]).max() < 1e-12
            assert a[p]["nf"] == b[p]["nf"]
            assert _field_close(a[p]["field"], b[p]["field"], 1e-9)


def test_s6_size_scaling(oracle):
    m, p_max, s = 1.333, 3, 3.0
    axes = np.array([60.0, 50.0, 40.0])
    euler = (10.0, 40.0, -20.0)
    P1 = oracle.particle(axes, euler, m)
    P2 = oracle.particle(axes * s, euler, m)
    S1 = oracle.setup(LAM, 2, 0, p_max, 16)
    S2 = oracle.setup(LAM * s, 2, 0, p_max, 16)
    xy = _sample(oracle.grid_halfwidth(P1), seed=6)
    e1 = _emits(oracle, P1, S1, xy, p_max)
    e2 = _emits(oracle, P2, S2, xy * s, p_max)
    for a, b in zip(e1, e2):
        for p in range(p_max + 1):
            assert a[p]["valid"] == b[p]["valid"]
            if not a[p]["valid"]:
                continue
            assert np.abs(a[p]["dir"] - b[p]["dir"]).max() < 1e-12
            assert abs(b[p]["amp"] / a[p]["amp"] - s) < 1e-11 * s
            assert abs(a[p]["phase"] - b[p]["phase"]) < 1e-9
            assert _field_close(s * a[p]["field"], b[p]["field"], 1e-10)
