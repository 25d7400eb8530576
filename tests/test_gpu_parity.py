"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element
by element, on seeded inputs.

Bars (written per test; the far-field comparisons are tests/parity.py's):
* FP64 path: per-ray records within 1e-10 relative, or within COND_C eps cond
  where the GPU's own conditioning record cond says the divergence factor is
  defined no better; far fields within 1e-10 relative on every node outside
  the caustic and pole bands, tie nodes and sheet edges included; integer
  results (which orders are emitted, focal-line counts, contributions per
  node) identical.
* Mixed path (FP32 wave quantities, FP64 phase): far-field intensity within
  1e-4 of the node's incoherent sum sum_b |f_b|^2, phase within 1e-3 rad
  where |F| >= 0.1 sqrt(sum_b |f_b|^2), on every node outside the 0.1 deg
  caustic and pole bands and 1e-4 deg of a sheet edge.
"""
import sys

import numpy as np
import pytest

import parity as PAR
from paper_2403_13856_amd import inputs as I

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_13856_amd import rtw
    rtw.load()
    return rtw


def _oracle_pair(oracle, R, axes, euler, m, lam, n_pol, p_min, p_max, N, precision):
    op = oracle.particle(axes, euler, m)
    os_ = oracle.setup(lam, n_pol, p_min, p_max, N)
    gp = R.make_particle(axes, euler, m)
    gi = R.make_incident(lam, n_pol)
    go = R.make_opts(p_min, p_max, N, precision)
    return op, os_, gp, gi, go


TRACE_CASES = [
    ("sphere", (50.0, 50.0, 50.0), (0.0, 0.0, 0.0), 1.333, 1, 0, 3, 64),
    ("ellipsoid_60_50_40", (60.0, 50.0, 40.0), (30.0, 20.0, 10.0), 1.333, 2, 0, 3, 48),
    ("random_0", None, None, None, 2, 0, 5, 40),
    ("random_1", None, None, None, 2, 1, 4, 33),
    ("dense_m_below_1", (30.0, 35.0, 40.0), (5.0, 60.0, -20.0), 0.75, 2, 0, 3, 40),
]


def _case_params(case, seed):
    name, axes, euler, m, n_pol, p_min, p_max, N = case
    if axes is None:
        axes, euler, m = I.random_ellipsoid(np.random.default_rng(seed))
    return name, axes, euler, m, n_pol, p_min, p_max, N


@pytest.mark.parametrize("ci", range(len(TRACE_CASES)))
def test_trace_fp64_matches_oracle(oracle, R, ci):
    name, axes, euler, m, n_pol, p_min, p_max, N = _case_params(TRACE_CASES[ci], 10 + ci)
    say(f"[trace fp64] {name} axes={axes} euler={euler} m={m} N={N} p={p_min}..{p_max}")
    op, os_, gp, gi, go = _oracle_pair(oracle, R, axes, euler, m, 0.6328, n_pol, p_min, p_max, N, R.FP64)
    ref = oracle.trace_grid(op, os_)
    got = {k: v.cpu().numpy() for k, v in R.trace(gp, gi, go).items()}
    torch.cuda.synchronize()
    assert np.array_equal(got["flags"], ref["flags"]), "emitted orders / focal-line counts differ"
    v = (ref["flags"] & 1).astype(bool)
    assert v.sum() > 0
    scale = max(axes)
    assert np.abs(got["dir"] - ref["dir"]).max() < 1e-12
    assert np.abs(got["rexit"] - ref["rexit"]).max() < 1e-10 * scale
    assert np.abs(got["phase"] - ref["phase"]).max() < 1e-10 * max(1.0, np.abs(ref["phase"]).max())
    # per ray: 1e-10, or the ray's FP64 conditioning (divergence factor, exit point)
    bound = np.maximum(1e-10, PAR.COND_C * PAR.EPS64 * PAR.ray_conditioning(got, 2 * np.pi / 0.6328))
    amp_rel = np.abs(got["amp"][v] - ref["amp"][v]) / ref["amp"][v]
    say(f"   amp worst {amp_rel.max():.2e}; {(amp_rel >= 1e-10).sum()} rays above 1e-10 "
        f"(cond up to {got['cond'][:, 0][v].max():.2e})")
    assert np.all(amp_rel < bound[v]), (amp_rel / bound[v]).max()
    F = ref["field"][..., 0, :] + 1j * ref["field"][..., 1, :]
    Fg = got["field"][..., 0, :] + 1j * got["field"][..., 1, :]
    mag = np.sqrt((np.abs(F) ** 2).sum(axis=(1, 2), keepdims=True))
    err = (np.abs(Fg - F) / np.maximum(mag, 1e-300)).max(axis=(1, 2))
    assert np.all(err[v] < bound[v]), (err[v] / bound[v]).max()


@pytest.mark.parametrize("ci", range(len(TRACE_CASES)))
def test_trace_mixed_matches_oracle(oracle, R, ci):
    name, axes, euler, m, n_pol, p_min, p_max, N = _case_params(TRACE_CASES[ci], 10 + ci)
    say(f"[trace mixed] {name} N={N}")
    op, os_, gp, gi, go = _oracle_pair(oracle, R, axes, euler, m, 0.6328, n_pol, p_min, p_max, N, R.MIXED)
    ref = oracle.trace_grid(op, os_)
    got = {k: v.cpu().numpy() for k, v in R.trace(gp, gi, go).items()}
    same = got["flags"] == ref["flags"]
    assert same.mean() > 0.999, same.mean()       # focal counts may flip within rounding of a caustic
    v = ((ref["flags"] & 1) == 1) & same
    ddir = np.abs(got["dir"] - ref["dir"]).max(axis=1)[v]
    assert np.quantile(ddir, 0.999) < 2e-5 and ddir.max() < 1e-3, (np.quantile(ddir, 0.999), ddir.max())
    # The far field uses each ray's phase carried to a node direction n as
    # phase + k r.(dir - n); comparing at n = oracle direction removes the
    # (harmless) difference of the FP32 exit direction.
    k = 2 * np.pi / 0.6328
    carried = got["phase"] + k * (got["rexit"] * (got["dir"] - ref["dir"])).sum(axis=1)
    dphi = np.abs(np.angle(np.exp(1j * (carried - ref["phase"]))))[v]
    amp_rel = (np.abs(got["amp"] - ref["amp"]) / np.maximum(ref["amp"], 1e-300))[v]
    say(f"   phase q99.9 {np.quantile(dphi, 0.999):.2e} max {dphi.max():.2e}; "
        f"amp q99.9 {np.quantile(amp_rel, 0.999):.2e} max {amp_rel.max():.2e}")
    assert np.quantile(dphi, 0.999) < 1e-4 and dphi.max() < 1e-3
    assert np.quantile(amp_rel, 0.999) < 2e-5 and amp_rel.max() < 1e-3


def _farfield_gpu(R, gp, gi, go, theta, phi, hits_per_node=6.0):
    ff = R.FarField(gp, gi, go, theta, phi, hits_per_node=hits_per_node)
    F = ff().cpu().numpy()
    nc = ff.ncontrib.cpu().numpy()
    return F, nc, ff


def _compare_fp64(ref, F, nc, tol=1e-10):
    return PAR.compare_fp64(ref, F, nc, tol)


def test_farfield_fp64_sphere(oracle, R):
    w = I.sphere_fp64()
    for N in (128, 512):
        say(f"[farfield fp64] sphere N={N} nodes={w.theta_deg.size}x{w.phi_deg.size}")
        op, os_, gp, gi, go = _oracle_pair(oracle, R, w.semi_axes, w.euler_deg, w.m, w.wavelength, w.n_pol,
                                          w.p_min, w.p_max, N, R.FP64)
        ref = oracle.farfield(op, os_, w.theta_deg, w.phi_deg)
        F, nc, _ = _farfield_gpu(R, gp, gi, go, w.theta_deg, w.phi_deg)
        frac = _compare_fp64(ref, F, nc)
        assert frac > 0.95


@pytest.mark.parametrize("N", [96, 2048])
def test_farfield_fp64_ellipsoid(oracle, R, N):
    """N = 2048 is the benchmark workload at its full size (the FP64 leg bench.py times)."""
    w = I.ellipsoid_mixed()
    say(f"[farfield fp64] ellipsoid N={N} full node grid")
    op, os_, gp, gi, go = _oracle_pair(oracle, R, w.semi_axes, w.euler_deg, w.m, w.wavelength, w.n_pol,
                                      w.p_min, w.p_max, N, R.FP64)
    ref = oracle.farfield(op, os_, w.theta_deg, w.phi_deg)
    F, nc, _ = _farfield_gpu(R, gp, gi, go, w.theta_deg, w.phi_deg)
    frac = _compare_fp64(ref, F, nc)
    assert frac > 0.9


def _compare_mixed(ref, F, int_tol=1e-4, ph_tol=1e-3):
    return PAR.compare_mixed(ref, F, int_tol, ph_tol, say)


@pytest.mark.parametrize("N", [256, 2048])
def test_farfield_mixed_ellipsoid(oracle, R, N):
    """The benchmark workload (N=2048 is its full size) and a smaller grid."""
    w = I.ellipsoid_mixed()
    say(f"[farfield mixed] ellipsoid N={N} nodes={w.n_nodes}")
    op, os_, gp, gi, go = _oracle_pair(oracle, R, w.semi_axes, w.euler_deg, w.m, w.wavelength, w.n_pol,
                                      w.p_min, w.p_max, N, R.MIXED)
    ref = PAR.oracle_farfield(oracle, op, os_, w.theta_deg, w.phi_deg, mixed=True)
    F, nc, ff = _farfield_gpu(R, gp, gi, go, w.theta_deg, w.phi_deg)
    hits, fp64 = ff.stats()
    rel, dph = _compare_mixed(ref, F)
    say(f"   intensity rel p99.99 {np.quantile(rel, 0.9999):.3e}; hits {hits}; rays re-traced in FP64 {fp64} "
        f"of {N * N}")
    assert rel.size > 0.95 * w.n_nodes


def test_farfield_deterministic(R):
    w = I.ellipsoid_mixed()
    say("[determinism] ellipsoid N=256 mixed, two runs")
    gp = R.make_particle(w.semi_axes, w.euler_deg, w.m)
    gi = R.make_incident(w.wavelength, 2)
    go = R.make_opts(0, 3, 256, R.MIXED)
    ff = R.FarField(gp, gi, go, w.theta_deg, w.phi_deg)
    a = ff().clone()
    b = ff().clone()
    assert torch.equal(torch.view_as_real(a), torch.view_as_real(b))


def test_farfield_graph_replay_equals_eager(R):
    # rtw_farfield queues kernels only (no allocation, copy, fill or sync), so
    # a caller can capture it into a HIP graph; every replay, with eager work
    # on the same workspace between replays, must give the eager result.
    w = I.ellipsoid_mixed()
    say("[graph] ellipsoid N=256 mixed: captured far field replayed three times")
    for prec in (R.MIXED, R.FP64):
        ff = R.FarField(R.make_particle(w.semi_axes, w.euler_deg, w.m), R.make_incident(w.wavelength, 2),
                        R.make_opts(0, 3, 256, prec), w.theta_deg, w.phi_deg)
        ref = torch.view_as_real(ff()).clone()
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            ff.launch(stream=s, with_counts=False)
        torch.cuda.synchronize()
        for _ in range(3):
            ff.out.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(torch.view_as_real(ff.field()), ref)
            ff.launch(with_counts=False)  # eager work between replays
            torch.cuda.synchronize()
            assert torch.equal(torch.view_as_real(ff.field()), ref)


def test_farfield_edge_cases(oracle, R):
    # a single quad (N = 2), one node row, a lone order, both precisions
    say("[edge] N=2, tiny grids, lone orders")
    for prec in (R.FP64, R.MIXED):
        for (N, th, ph, pmin, pmax) in [(2, [90.0, 150.0, 180.0], [0.0, 90.0, 270.0], 0, 2),
                                        (16, [180.0], [0.0], 0, 0),
                                        (24, [0.0, 20.0], [0.0, 45.0, 359.0], 1, 1),
                                        (31, np.arange(0, 181, 3.0), np.arange(0, 360, 7.0), 3, 3)]:
            th = np.asarray(th, float)
            ph = np.asarray(ph, float)
            op, os_, gp, gi, go = _oracle_pair(oracle, R, (40.0, 35.0, 30.0), (15.0, 25.0, 35.0), 1.333, 0.6328, 2,
                                              pmin, pmax, N, prec)
            ref = PAR.oracle_farfield(oracle, op, os_, th, ph, mixed=prec == R.MIXED)
            F, nc, _ = _farfield_gpu(R, gp, gi, go, th, ph)
            say(f"   precision={prec} N={N} nodes={th.size}x{ph.size} p={pmin}..{pmax}")
            if prec == R.FP64:
                _compare_fp64(ref, F, nc)
            else:
                _compare_mixed(ref, F)


def test_workspace_overflow_is_reported_and_recovered(oracle, R):
    w = I.sphere_fp64()
    # a 0.25 deg node grid (1 M nodes, 1.7 M hits) against the smallest pool
    # (256 slots in each of the 1024 partitions): the pool must overflow
    th = I.uniform_angles(0.0, 180.0, 0.25)
    ph = I.uniform_angles(0.0, 359.75, 0.25)
    say(f"[overflow] sphere N=128, {th.size}x{ph.size} nodes, with a deliberately small hit pool")
    gp = R.make_particle(w.semi_axes, w.euler_deg, w.m)
    gi = R.make_incident(w.wavelength, 1)
    go = R.make_opts(0, 2, 128, R.FP64)
    ff = R.FarField(gp, gi, go, th, ph, hits_per_node=0.01)
    small = ff.ws_bytes
    ff.launch()
    rc, need = ff.status()
    assert rc == R.RTW_ERR_WORKSPACE and need > small
    F = ff().cpu().numpy()  # grows the workspace and re-runs
    assert ff.ws_bytes >= need
    op = oracle.particle(w.semi_axes, w.euler_deg, w.m)
    ref = oracle.farfield(op, oracle.setup(w.wavelength, 1, 0, 2, 128), th, ph)
    _compare_fp64(ref, F, ff.ncontrib.cpu().numpy())


def test_uniform_axis_boxes_match_segment_tables(R):
    # Boxes on a uniform node axis use FP32 index arithmetic, on any other axis
    # the segment tables; boxes only prune, so adding one off-grid node (which
    # makes the axis non-uniform) must leave every shared node bitwise alike.
    w = I.ellipsoid_mixed()
    th_u = I.uniform_angles(0.0, 180.0, 0.25)
    ph_u = I.uniform_angles(0.0, 359.0, 1.0)
    for prec in (R.MIXED, R.FP64):
        gp = R.make_particle(w.semi_axes, w.euler_deg, w.m)
        gi = R.make_incident(w.wavelength, 2)
        go = R.make_opts(0, 3, 512, prec)
        F_u, nc_u, _ = _farfield_gpu(R, gp, gi, go, th_u, ph_u)
        for axis in ("theta", "phi"):
            th, ph = th_u, ph_u
            if axis == "theta":
                th = np.sort(np.append(th_u, 33.3))
            else:
                ph = np.sort(np.append(ph_u, 200.5))
            F, nc, _ = _farfield_gpu(R, gp, gi, go, th, ph)
            it = np.searchsorted(th, th_u)
            ip = np.searchsorted(ph, ph_u)
            assert np.array_equal(th[it], th_u) and np.array_equal(ph[ip], ph_u)
            say(f"[uniform axis] precision={prec} extra node on {axis}: "
                f"{int(nc_u.sum())} contributions on the uniform grid")
            assert np.array_equal(nc[np.ix_(it, ip)], nc_u)
            assert np.array_equal(F[:, :, it][:, :, :, ip], F_u)


def test_node_ranges_of_a_large_grid_match_its_halves(R):
    # The node ranges come from a scan of the node counts whose block sums are
    # added up by the final pass itself up to 4096 scan blocks of 2048 nodes,
    # and scanned by a kernel of their own beyond.  A 3601 x 3600 node grid
    # (13 M nodes) takes the second way, each of its two theta halves the
    # first; every node's sum depends only on its own hits, so the halves
    # must reproduce the whole grid bitwise.
    w = I.ellipsoid_mixed()
    th = I.uniform_angles(0.0, 180.0, 0.05)
    ph = I.uniform_angles(0.0, 359.9, 0.1)
    assert th.size * ph.size > 4096 * 2048 and (th.size // 2) * ph.size <= 4096 * 2048
    half = th.size // 2
    gp = R.make_particle(w.semi_axes, w.euler_deg, w.m)
    gi = R.make_incident(w.wavelength, 2)
    go = R.make_opts(0, 3, 256, R.MIXED)
    say(f"[node ranges] ellipsoid N=256 mixed on {th.size}x{ph.size} nodes and on its two theta halves")
    F, nc, _ = _farfield_gpu(R, gp, gi, go, th, ph)
    Fa, nca, _ = _farfield_gpu(R, gp, gi, go, th[:half], ph)
    Fb, ncb, _ = _farfield_gpu(R, gp, gi, go, th[half:], ph)
    say(f"   {int(nc.sum())} contributions on the whole grid")
    assert nc.sum() > 0 and nca.sum() > 0 and ncb.sum() > 0
    assert np.array_equal(nc[:half], nca) and np.array_equal(nc[half:], ncb)
    assert np.array_equal(F[:, :, :half], Fa) and np.array_equal(F[:, :, half:], Fb)


def test_three_run_axis_boxes_match_segment_tables(R):
    # An axis of three uniform runs (a refined band, as on the large
    # workload's theta grid) and the same axis with one off-grid node more
    # (five runs) index their boxes through the segment tables with different
    # runs.  Boxes only prune, so every shared node must come out bitwise alike.
    w = I.ellipsoid_mixed()
    th_3 = np.concatenate([I.uniform_angles(0.0, 119.5, 0.5), I.uniform_angles(120.0, 140.0, 0.02),
                           I.uniform_angles(140.5, 180.0, 0.5)])
    ph_u = I.uniform_angles(0.0, 359.0, 1.0)
    th_x = np.sort(np.append(th_3, 60.3))
    it = np.searchsorted(th_x, th_3)
    assert np.array_equal(th_x[it], th_3)
    for prec in (R.MIXED, R.FP64):
        gp = R.make_particle(w.semi_axes, w.euler_deg, w.m)
        gi = R.make_incident(w.wavelength, 2)
        go = R.make_opts(0, 3, 512, prec)
        F3, nc3, _ = _farfield_gpu(R, gp, gi, go, th_3, ph_u)
        Fx, ncx, _ = _farfield_gpu(R, gp, gi, go, th_x, ph_u)
        say(f"[three-run axis] precision={prec}: {int(nc3.sum())} contributions")
        assert nc3.sum() > 0
        assert np.array_equal(ncx[it], nc3)
        assert np.array_equal(Fx[:, :, it], F3)


def test_paper_spheroid_strips_match_oracle(oracle, R):
    """The paper's spheroid (a=b=100, c=90 um, incidence along its x axis) at its
    full ray count and the paper's 0.01 deg node spacing, on strips across the
    primary rainbow and the forward lobe: mixed path against the oracle."""
    w = I.paper_spheroid()
    ph = I.uniform_angles(0.0, 90.0, 45.0)
    op, os_, gp, gi, go = _oracle_pair(oracle, R, w.semi_axes, w.euler_deg, w.m, w.wavelength, w.n_pol, w.p_min,
                                      w.p_max, w.grid_n, R.MIXED)
    for th in (I.uniform_angles(136.0, 140.0, 0.01), I.uniform_angles(5.0, 6.0, 0.01)):
        say(f"[paper spheroid] N={w.grid_n}, theta {th[0]:.2f}..{th[-1]:.2f} step 0.01 x phi {ph.tolist()}")
        ref = PAR.oracle_farfield(oracle, op, os_, th, ph, mixed=True)
        F, nc, _ = _farfield_gpu(R, gp, gi, go, th, ph)
        rel, dph = _compare_mixed(ref, F)
        assert rel.size > 0.5 * th.size * ph.size
