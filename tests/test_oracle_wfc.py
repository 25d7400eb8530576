"""Pins of the oracle's wavefront-curvature machinery (Eq. 3 at every
interaction, free propagation, Eq. 6 divergence factor, focal-line count).

The reference is the classical ray-tube construction the paper contrasts its
method with (a bundle of neighbouring rays): three rays per axis, central
differences in the incident position xi.  Along any straight segment the
transverse offset of a neighbouring ray, measured in the plane normal to the
central ray, is X(s) = A + s B (first order in h).  Then

* the WFC right after the interaction is Q = B A^{-1}  (d(dir_perp) = Q d(r_perp));
* a focal line is a zero of det(A + s B) on the segment (s in (0, L), or
  s > 0 on the far-field leg);
* energy along the tube: S^2 |det B_far| = prod over refractions of
  (n_out cos theta_out)/(n_in cos theta_in), S the far-field amplitude.

Synge's relations (Eqs. 1-2) pin the special case of incidence in a symmetry
plane.
"""
import numpy as np
import pytest

from paper_2403_13856_amd.inputs import random_ellipsoid

LAM = 0.6328


def _rotation(euler_deg):
    a, b, g = np.radians(euler_deg)
    Rz = lambda t: np.array([[np.cos(t), -np.sin(t), 0], [np.sin(t), np.cos(t), 0], [0, 0, 1]])
    Ry = lambda t: np.array([[np.cos(t), 0, np.sin(t)], [0, 1, 0], [-np.sin(t), 0, np.cos(t)]])
    return Rz(a) @ Ry(b) @ Rz(g)


def _segments(ray, p):
    """(start point, direction, basis e1, length) for the internal segments
    leading to order p and for its far-field leg."""
    segs = []
    for q in range(p):  # continuing branch after interactions 1..p
        P0 = np.array(ray.hit[q][:])
        d0 = np.array(ray.dir_cont[q][:])
        e1 = np.array(ray.eperp_cont[q][:])
        L = np.linalg.norm(np.array(ray.hit[q + 1][:]) - P0)
        segs.append((P0, d0, e1, L))
    e = ray.emit[p]
    segs.append((np.array(e.rexit[:]), np.array(e.dir[:]), np.array(e.eperp[:]), np.inf))
    return segs


def _tube(rays_c, rays_px, rays_mx, rays_py, rays_my, p, h):
    """Per segment: (A, B, L, basis) from central differences."""
    out = []
    sc = _segments(rays_c, p)
    nbr = [_segments(r, p) for r in (rays_px, rays_mx, rays_py, rays_my)]
    for k, (C0, d0, e1, L) in enumerate(sc):
        e2 = np.cross(d0, e1)
        E = np.stack([e1, e2])

        def ab(seg):
            Pn, dn = seg[k][0], seg[k][1]
            t0 = (C0 - Pn) @ d0 / (dn @ d0)
            alpha = Pn + t0 * dn - C0
            beta = dn / (dn @ d0) - d0
            return E @ alpha, E @ beta
        (apx, bpx), (amx, bmx), (apy, bpy), (amy, bmy) = [ab(s) for s in nbr]
        A = np.stack([(apx - amx) / (2 * h), (apy - amy) / (2 * h)], 1)
        B = np.stack([(bpx - bmx) / (2 * h), (bpy - bmy) / (2 * h)], 1)
        out.append((A, B, L))
    return out


def _roots_in(A, B, L):
    """Zeros of det(A + s B) for s in (0, L) and their distance to the ends."""
    c2 = np.linalg.det(B)
    c0 = np.linalg.det(A)
    c1 = A[0, 0] * B[1, 1] + B[0, 0] * A[1, 1] - A[0, 1] * B[1, 0] - B[0, 1] * A[1, 0]
    roots = np.roots([c2, c1, c0]) if abs(c2) > 1e-300 else np.roots([c1, c0])
    roots = [r.real for r in roots if abs(r.imag) < 1e-9 * (1 + abs(r.real))]
    inside = [r for r in roots if 0 < r < L]
    margin = min([abs(r) for r in roots] + [abs(r - L) for r in roots if np.isfinite(L)] + [np.inf])
    return len(inside), margin


def _trace_tubes(oracle, P, S, xy, h):
    offs = np.array([[0, 0], [h, 0], [-h, 0], [0, h], [0, -h]])
    pts = (xy[:, None, :] + offs[None, :, :]).reshape(-1, 2)
    rays = oracle.trace_rays(P, S, pts)
    return [[rays[5 * i + j] for j in range(5)] for i in range(xy.shape[0])]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_wfc_matches_finite_difference_ray_tubes(oracle, seed):
    rng = np.random.default_rng(100 + seed)
    axes, euler, m = random_ellipsoid(rng)
    P = oracle.particle(axes, euler, m)
    p_max = 3
    S = oracle.setup(LAM, 1, 0, p_max, 16)
    L = oracle.grid_halfwidth(P)
    xy = rng.uniform(-L, L, size=(80, 2))
    h = 1e-5 * min(axes)
    tubes = _trace_tubes(oracle, P, S, xy, h)
    tubes2 = _trace_tubes(oracle, P, S, xy, 2 * h)
    Rm = _rotation(euler)
    Amat = np.diag(1.0 / np.array(axes) ** 2)
    checked = 0
    for rc, rc2 in zip(tubes, tubes2):
        if not all(r.active for r in rc + rc2):
            continue
        for p in range(p_max + 1):
            if not all(r.emit[p].valid for r in rc + rc2):
                continue
            tube_h = _tube(*rc, p, h)
            tube_2h = _tube(*rc2, p, 2 * h)
            # Richardson extrapolation of the central differences (error O(h^4))
            tube = [((4 * A1 - A2) / 3, (4 * B1 - B2) / 3, L1) for (A1, B1, L1), (A2, B2, _) in zip(tube_h, tube_2h)]
            # skip rays near a caustic: the first-order tube is ill-conditioned there
            conds = [np.linalg.cond(Am) for Am, _, _ in tube]
            if max(conds) > 1e4:
                continue
            # WFC right after each interaction, and at the exit
            for k, (Am, Bm, Lk) in enumerate(tube):
                Qfd = Bm @ np.linalg.inv(Am)
                if k < p:
                    qo = np.array(rc[0].q_cont[k][:])
                else:
                    qo = np.array(rc[0].emit[p].q[:])
                Qo = np.array([[qo[0], qo[1]], [qo[1], qo[2]]])
                scale = np.abs(Qo).max()
                assert np.abs(Qfd - Qo).max() < 1e-6 * scale, (p, k, Qfd, Qo)
            # focal lines: zeros of the tube cross-section
            nf = 0
            margins = []
            for Am, Bm, Lk in tube:
                n, mg = _roots_in(Am, Bm, Lk)
                nf += n
                margins.append(mg)
            if min(margins) > 1e-3 * min(axes):
                assert nf == rc[0].emit[p].nf, (p, nf, rc[0].emit[p].nf)
            # power along the tube (Eq. 5-6 amplitude vs ray-tube energy)
            e = rc[0].emit[p]
            Bfar = tube[-1][1]
            ratio = 1.0
            if p >= 1:
                hits = [np.array(rc[0].hit[0][:]), np.array(e.rexit[:])]
                dins = [np.array([0, 0, 1.0]), np.array(rc[0].dir_cont[p - 1][:])]
                douts = [np.array(rc[0].dir_cont[0][:]), np.array(e.dir[:])]
                nins, nouts = [1.0, m], [m, 1.0]
                for hpt, di, do, ni, no in zip(hits, dins, douts, nins, nouts):
                    rb = Rm.T @ hpt
                    nb = Amat @ rb
                    nl = Rm @ (nb / np.linalg.norm(nb))
                    ratio *= (no * abs(do @ nl)) / (ni * abs(di @ nl))
            lhs = e.amp ** 2 * abs(np.linalg.det(Bfar))
            assert abs(lhs / ratio - 1) < 1e-6, (p, lhs, ratio)
            checked += 1
    assert checked > 80


@pytest.mark.parametrize("axes", [(60.0, 50.0, 40.0), (40.0, 55.0, 70.0)])
def test_synge_relations_symmetric_plane(oracle, axes):
    """Eqs. 1-2: for incidence in the symmetry plane y = 0 of an axis-aligned
    ellipsoid, the refracted principal WFCs follow
      k_r/R_r1 = k_i/R_i1 + (k_rn - k_in)/rho_1,
      k_rn^2/(k_r R_r2) = k_in^2/(k_i R_i2) + (k_rn - k_in)/rho_2,
    with a plane incident wave (1/R_i = 0) and rho = -1/kappa for a surface
    convex towards the outward normal (index 1: perpendicular to the incidence
    plane, 2: in it).  The reflected wave follows with k_rn -> -k_in."""
    a, b, c = axes
    m = 1.333
    k = 2 * np.pi / LAM
    P = oracle.particle(axes, (0, 0, 0), m)
    S = oracle.setup(LAM, 1, 0, 1, 16)
    xs = np.linspace(-0.95, 0.95, 38) * a  # even count: no exact normal incidence (incidence plane undefined)
    rays = oracle.trace_rays(P, S, np.stack([xs, np.zeros_like(xs)], 1))
    for i, x0 in enumerate(xs):
        z0 = -c * np.sqrt(1 - (x0 / a) ** 2)
        t = np.arctan2(z0 / c, x0 / a)
        # in-plane curvature of the ellipse section (parametric formula)
        kap_par = a * c / (a * a * np.sin(t) ** 2 + c * c * np.cos(t) ** 2) ** 1.5
        # out-of-plane normal curvature via Meusnier's theorem on the section x = x0
        s = 1 - (x0 / a) ** 2
        bp, cp = b * np.sqrt(s), c * np.sqrt(s)
        nvec = np.array([x0 / a ** 2, 0.0, z0 / c ** 2])
        nhat = nvec / np.linalg.norm(nvec)
        kap_perp = (cp / bp ** 2) * abs(nhat[2])
        ci = abs(nhat[2])
        ct = np.sqrt(1 - (1 - ci * ci) / m ** 2)
        kin, krn, kr = k * ci, m * k * ct, m * k
        q_t = np.array(rays[i].q_cont[0][:])
        assert abs(q_t[1]) < 1e-12 * np.abs(q_t).max()
        assert abs(q_t[0] - (-(krn - kin) * kap_perp / kr)) < 1e-12 * abs(q_t[0])
        assert abs(q_t[2] - (-(krn - kin) * kap_par * kr / krn ** 2)) < 1e-12 * abs(q_t[2])
        q_r = np.array(rays[i].emit[0].q[:])
        assert abs(q_r[0] - 2 * ci * kap_perp) < 1e-12 * abs(q_r[0])
        assert abs(q_r[2] - 2 * kap_par / ci) < 1e-12 * abs(q_r[2])
