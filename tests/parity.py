"""Comparison of the HIP path's far fields and ray records with the FP64
oracle's, shared by the GPU parity tests.

Mixed path (FP32 wave quantities, FP64 polyline and phase):
  * intensity |I_gpu - I_ref| / sum_b |f_b|^2 < 1e-4, the denominator being the
    node's incoherent sum over its triangle contributions (the metric of the
    near-zero-safe reading of the mixed bar); the ratio of the oracle's
    uncancelled size sum_b (sum_v |lambda_v| |F_v|)^2 to it is reported;
  * phase < 1e-3 rad where |F| >= 0.1 sqrt(sum_b |f_b|^2);
  * every node is compared except those within 0.1 deg of a dropped fold
    triangle (caustics, flag bit 1) or of theta = 0 / 180 deg (bit 2), and
    those within EDGE_BAND_MIXED of the edge of an order's ray sheet (bit 3):
    FP32 rounding of the directions and edge normals, a few 1e-7 rad, decides
    there whether a node belongs to the sheet's last triangle.  Tie nodes
    (bit 0) are compared: either owner gives the same value.
FP64 path:
  * every node outside the caustic and pole bands, sheet edges and ties
    included, within `tol` relative to sqrt(sum_b |f_b|^2), with the same
    contribution count; nodes the oracle leaves empty stay empty;
  * where a contributing ray is ill-conditioned, its field is defined in FP64
    only to its conditioning times eps: the divergence factor to cond[0] eps (a
    focal line close to an interface: the cancellation in det(I + L Q) of
    Eq. 6), its exit point -- hence the phase carried to a node, k n.r -- to
    drift x |r| eps with drift = cond[1], the growth of a direction perturbation
    along the ray.  A node within reach of such a ray is held to
    max(tol, COND_C eps (cond[0] + k |r_exit| cond[1])), from the GPU's own
    per-ray records (rtw_trace cond).
"""
import numpy as np

EDGE_BAND_MIXED = 1e-4  # deg
EPS64 = 2.0 ** -53
COND_C = 16.0  # measured: a ray's amplitude differs by up to ~2.4 eps cond


def _say(msg):
    print(msg, flush=True)


def oracle_farfield(oracle, op, os_, th, ph, mixed):
    """The oracle's far field with the sheet-edge band the comparison needs."""
    return oracle.farfield(op, os_, th, ph, edge_band_deg=EDGE_BAND_MIXED if mixed else 0.1)


def compare_mixed(ref, F, int_tol=1e-4, ph_tol=1e-3, say=_say, tag="", denominator="incoherent", extra_incoh=None):
    """Assert the mixed-path bars; returns (intensity errors, phase errors) of the compared nodes.
    denominator="uncancelled" divides by max(uncancelled, incoherent) instead: for
    grids so coarse that a triangle's interpolated terms cancel (the ratio of the
    two reaches ~100 at 24^2 rays), where FP32 rounding scales with the terms.
    extra_incoh: a further term's |F|^2 per node (the diffraction term), counted
    as one more contribution of the incoherent sum."""
    assert ref["edge_band_deg"] <= EDGE_BAND_MIXED, "oracle run with a wide sheet-edge band"
    fl = ref["flags"]
    inc = ref["incoh"] if extra_incoh is None else ref["incoh"] + extra_incoh
    sel = ((fl & 6) == 0) & (((fl & 8) == 0)) & (inc > 0)
    I_ref = (np.abs(ref["field"]) ** 2).sum(axis=(0, 1))
    I_got = (np.abs(F) ** 2).sum(axis=(0, 1))
    ratio = np.maximum(ref["uncancelled"], inc)[sel] / inc[sel]
    rel = np.abs(I_got - I_ref)[sel] / inc[sel]
    if denominator == "uncancelled":
        rel = rel / ratio
    else:
        assert denominator == "incoherent"
    big = (np.abs(ref["field"]) >= 0.1 * np.sqrt(inc)[None, None]) & sel[None, None]
    dph = np.abs(np.angle(F[big] * np.conj(ref["field"][big])))
    say(f"   {tag}mixed ({denominator}): {sel.sum()} of {sel.size} nodes compared ({((fl & 1) != 0).sum()} ties); intensity max "
        f"{rel.max(initial=0.0):.3e}; phase max {dph.max(initial=0.0):.3e}; uncancelled/incoherent max "
        f"{ratio.max(initial=1.0):.4f}")
    assert rel.max(initial=0.0) < int_tol, rel.max(initial=0.0)
    assert dph.max(initial=0.0) < ph_tol, dph.max(initial=0.0)
    return rel, dph


def node_dirs(th_deg, ph_deg):
    t = np.radians(np.asarray(th_deg, float))[:, None]
    p = np.radians(np.asarray(ph_deg, float))[None, :]
    return np.stack(np.broadcast_arrays(np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)), -1).reshape(-1, 3)


def ray_conditioning(rec, k):
    """Per-ray FP64 conditioning cond[0] + k |r_exit| cond[1] (see above)."""
    return rec["cond"][:, 0, :] + k * np.sqrt((rec["rexit"] ** 2).sum(1)) * rec["cond"][:, 1, :]


def cond_allowance(rec, N, th_deg, ph_deg, tol, robs=0.0, k=2 * np.pi / 0.6328):
    """Per-node bound max(tol, COND_C eps cond) from the GPU's FP64 per-ray
    records `rec` (flags, dir, rexit, cond of rtw_trace; cond as in
    ray_conditioning), over the rays whose triangles can hold the node: a ray
    reaches the nodes within the largest angle between its node-space
    direction and those of its eight grid neighbours (every triangle it is a
    vertex of lies inside that cap)."""
    from scipy.spatial import cKDTree
    n_t, n_p = len(th_deg), len(ph_deg)
    allow = np.full(n_t * n_p, tol)
    cond = ray_conditioning(rec, k)
    valid = (rec["flags"] & 1) == 1
    thr = tol / (COND_C * EPS64)
    bad = np.argwhere(valid & (cond > thr))
    if bad.size == 0:
        return allow.reshape(n_t, n_p), 0
    d = rec["dir"]
    if robs > 0.0:  # node-space direction: toward the point M on the sphere of radius R
        r = rec["rexit"]
        dr = (d * r).sum(1)
        dM = -dr + np.sqrt(np.maximum(robs ** 2 - (r * r).sum(1) + dr ** 2, 0.0))
        d = (r + dM[:, None, :] * d) / robs
    tree = cKDTree(node_dirs(th_deg, ph_deg))
    for o, i in bad:
        iy, ix = divmod(int(i), N)
        dv = d[o, :, i]
        rho = 0.0
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                jx, jy = ix + dx, iy + dy
                if (dx or dy) and 0 <= jx < N and 0 <= jy < N and valid[o, jy * N + jx]:
                    rho = max(rho, np.linalg.norm(d[o, :, jy * N + jx] - dv))
        idx = tree.query_ball_point(dv, 1.05 * rho + 1e-12)
        if idx:
            allow[idx] = np.maximum(allow[idx], COND_C * EPS64 * cond[o, i])
    return allow.reshape(n_t, n_p), len(bad)


def compare_fp64(ref, F, nc, tol=1e-10, allow=None, say=_say, tag="", extra_incoh=None):
    """Assert the FP64 bars; allow (per node) replaces tol where a contributing
    ray is ill-conditioned (cond_allowance).  Returns the fraction compared."""
    fl = ref["flags"]
    inc = np.sqrt(ref["incoh"] if extra_incoh is None else ref["incoh"] + extra_incoh)
    comp = (fl & 6) == 0
    bound = np.full(inc.shape, tol) if allow is None else np.maximum(allow, tol)
    err = np.abs(F - ref["field"]).max(axis=(0, 1)) / np.maximum(inc, 1e-300)
    sel = comp & (inc > 0)
    ties = sel & ((fl & 1) != 0)
    over = sel & (err >= tol)
    say(f"   {tag}fp64: {sel.sum()} of {sel.size} nodes compared ({ties.sum()} ties, worst there "
        f"{err[ties].max(initial=0.0):.2e}); worst {err[sel].max(initial=0.0):.3e}; {over.sum()} above {tol:.1e}, "
        f"largest allowance used {(err[over] / tol).max(initial=0.0):.1f} x tol")
    assert np.all(err[sel] < bound[sel]), (err[sel] / bound[sel]).max()
    assert np.array_equal(nc[comp], ref["ncontrib"][comp]), "contribution counts differ"
    assert np.abs(F[..., comp & (inc == 0)]).max(initial=0.0) == 0.0
    return comp.mean()
