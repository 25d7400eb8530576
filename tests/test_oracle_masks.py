"""Pins of the oracle's comparison aids: the per-node size of the interpolated
terms before they cancel ("uncancelled"), and the sheet-edge mask (flag bit 3).

uncancelled = sum_b (sum_v |lambda_v| |F_v|)^2 over a node's triangle
contributions b and their three vertex terms, incoh = sum_b |f_b|^2 with
f_b = sum_v lambda_v F_v e^{i carry_v}.  By the triangle inequality
uncancelled >= incoh at every node; the two are equal where one weight is 1
(a node on a ray's own direction); and since the carry makes the three vertex
terms agree in phase to second order in the ray spacing h, their magnitudes'
sum exceeds the sum's magnitude by O(h^4).

The sheet edge of order p = 1 on a sphere has a closed form: a ray of impact
parameter b = a sin(theta_i) leaves deflected by 2 theta_i - 2 theta_r
(Snell, sin theta_r = sin theta_i / m), up to 180 - 2 arcsin(1 / m) at
grazing incidence.  The field of the grid ends at the images of its boundary
rays (those with a neighbour that misses the sphere, or on the grid's edge).
"""
import numpy as np
import pytest

A = 50.0
M = 1.333
LAM = 0.6328


def _sphere(oracle):
    return oracle.particle((A, A, A), (0, 0, 0), M)


def test_uncancelled_bounds_the_incoherent_sum_and_converges_at_fourth_order(oracle):
    th = np.arange(0.0, 181.0, 1.0)
    ph = np.arange(0.0, 360.0, 1.0)
    medians = []
    for N in (64, 128, 256, 512):
        r = oracle.farfield(_sphere(oracle), oracle.setup(LAM, 1, 0, 2, N), th, ph)
        inc, unc, nc = r["incoh"], r["uncancelled"], r["ncontrib"]
        assert np.all(unc >= inc * (1 - 1e-12)), N
        assert np.all((unc == 0) == (nc == 0)) and np.all((inc == 0) == (nc == 0)), N
        sel = (r["flags"] == 0) & (nc > 0)
        medians.append(np.median(unc[sel] / inc[sel] - 1.0))
    rates = [medians[i] / medians[i + 1] for i in range(3)]
    # fourth order: halving h divides the excess by ~16 (measured 15, 16, 15)
    assert all(q > 8.0 for q in rates), (medians, rates)
    assert medians[-1] < 1e-5


def test_uncancelled_bounds_the_incoherent_sum_on_an_ellipsoid(oracle):
    p = oracle.particle((60.0, 50.0, 40.0), (30.0, 20.0, 10.0), M)
    r = oracle.farfield(p, oracle.setup(LAM, 2, 0, 3, 96), np.arange(0.0, 181.0, 1.5), np.arange(0.0, 360.0, 2.0))
    assert r["ncontrib"].sum() > 0
    assert np.all(r["uncancelled"] >= r["incoh"] * (1 - 1e-12))


def test_uncancelled_equals_the_incoherent_sum_on_a_ray_direction(oracle):
    """A node next to a ray's exit direction (1e-10 of the way to the centroid of
    one of its triangles, so that exactly one triangle holds it) has weights
    (1, 0, 0) to 1e-10: both sums are that ray's |F|^2 to that order."""
    P = _sphere(oracle)
    N = 64
    S = oracle.setup(LAM, 1, 0, 0, N)
    h = 2 * A / N
    for ix, iy in ((10, 20), (33, 40), (50, 12), (5, 31)):
        xy = np.array([[ix, iy], [ix + 1, iy], [ix + 1, iy + 1]], float)
        rays = oracle.trace_rays(P, S, -A + (xy + 0.5) * h)
        d = np.array([rays[k].emit[0].dir[:] for k in range(3)])
        n = d[0] + 1e-10 * (d.mean(0) - d[0])
        n /= np.linalg.norm(n)
        th = np.degrees(np.arccos(n[2]))
        ph = np.degrees(np.arctan2(n[1], n[0])) % 360.0
        r = oracle.farfield(P, S, np.array([th]), np.array([ph]))
        assert r["ncontrib"][0, 0] == 1, (ix, iy)
        inc, unc = r["incoh"][0, 0], r["uncancelled"][0, 0]
        assert inc > 0 and abs(unc / inc - 1.0) < 1e-9, (ix, iy, unc / inc - 1.0)


def _boundary_deflections(N):
    """Closed-form p = 1 deflections (deg) of the grid rays that bound the lit
    disc: inside it, with a grid neighbour outside it or no neighbour at all."""
    h = 2 * A / N
    c = -A + (np.arange(N) + 0.5) * h
    X, Y = np.meshgrid(c, c)
    inside = X ** 2 + Y ** 2 < A * A
    pad = np.pad(inside, 1)
    nb_out = np.zeros_like(inside)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            nb_out |= ~pad[1 + dy:1 + dy + N, 1 + dx:1 + dx + N]
    b = np.sqrt(X[inside & nb_out] ** 2 + Y[inside & nb_out] ** 2) / A
    ti, tr = np.arcsin(b), np.arcsin(b / M)
    return np.degrees(2 * ti - 2 * tr)


@pytest.mark.parametrize("N", [64, 256, 1024])
def test_sheet_edge_mask_hugs_the_sheet_edge(oracle, N):
    band = 0.1
    grazing = 180.0 - 2.0 * np.degrees(np.arcsin(1.0 / M))  # 82.787 deg
    th = np.arange(0.0, 180.001, 0.05)
    ph = np.array([0.0, 17.0, 45.0, 90.0, 133.0])
    r = oracle.farfield(_sphere(oracle), oracle.setup(LAM, 1, 1, 1, N), th, ph, band_deg=band)
    fl, nc = r["flags"], r["ncontrib"]
    tt = np.broadcast_to(th[:, None], fl.shape)
    edge = (fl & 8) != 0
    defl = _boundary_deflections(N)
    lo, hi = defl.min(), defl.max()
    assert lo < hi < grazing
    # flagged nodes lie within the band of the boundary rays' images
    assert edge.any()
    assert tt[edge].min() >= lo - band - 1e-6 and tt[edge].max() <= hi + band + 1e-6
    # wherever a theta column's coverage starts or stops, the node is flagged
    change = (nc[1:] > 0) != (nc[:-1] > 0)
    trans = np.zeros_like(edge)
    trans[1:] |= change
    trans[:-1] |= change
    trans &= (tt > band) & (tt < 180.0 - band)
    assert trans.sum() >= ph.size and np.all(edge[trans])
    # inside the sheet: covered once and unflagged; beyond it: empty and unflagged
    inner = (tt > band + 0.05) & (tt < lo - band)
    outer = (tt > hi + band) & (tt < 180.0 - band)
    # (tie nodes, bit 0, lie on the symmetry lines phi = 0, 45, 90 deg of the grid)
    assert np.all(nc[inner] == 1) and np.all((fl[inner] & ~1) == 0)
    assert np.all(nc[outer] == 0) and np.all(fl[outer] == 0)
    # the mask follows the grid's rim toward the grazing edge as N grows
    if N == 1024:
        assert grazing - hi < 0.5


def test_narrow_sheet_edge_band_keeps_the_caustic_band(oracle):
    """The sheet-edge band has its own width: narrowing it leaves the caustic
    (bit 1) and pole (bit 2) bands and the field itself unchanged."""
    p = oracle.particle((60.0, 50.0, 40.0), (30.0, 20.0, 10.0), M)
    S = oracle.setup(LAM, 2, 0, 3, 64)
    th, ph = np.arange(0.0, 181.0, 1.0), np.arange(0.0, 360.0, 2.0)
    wide = oracle.farfield(p, S, th, ph)
    narrow = oracle.farfield(p, S, th, ph, edge_band_deg=1e-4)
    assert np.array_equal(wide["field"], narrow["field"])
    assert np.array_equal(wide["flags"] & 7, narrow["flags"] & 7)
    assert ((narrow["flags"] & 8) != 0).sum() < ((wide["flags"] & 8) != 0).sum()
