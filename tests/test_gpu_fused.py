"""GPU checks of the fused mixed-precision kernel (k_fused: trace, rasterisation
and hit contributions per ray tile, no per-ray records in HBM) against the
staged pipeline (the default) and the FP64 oracle; rtw_batch_opts.fused asks for it.

Bars:
* the same set of node hits as the staged pipeline: equal contribution counts
  at every node and equal hit totals;
* the oracle's mixed bars (tests/parity.py) on the same inputs;
* fused and staged far fields within 1e-4 of the node's incoherent sum of each
  other (they differ only where a ray re-traced in FP64 emitted an order before
  its divergence factor became ill-conditioned: the fused kernel keeps that
  order's FP32 record, the staged one the FP64 re-trace's);
* bitwise the same result for any tile height and persistence (every ray's
  records, every hit and the per-node summation order are independent of the
  tiling).
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


def _run(R, part, N, n_pol, p_min, p_max, th, ph, staged, tune=None, robs=0.0):
    inc = R.make_incident(0.6328, n_pol, observation_radius=robs)
    b = R.Batch([part], [N], inc, R.make_opts(p_min, p_max, N, R.MIXED), th, ph, fused=not staged, tune=tune,
                incoherent=True)
    F = b().clone()
    hits, fp64 = b.stats()
    return F[0].cpu().numpy(), b.ncontrib[0].cpu().numpy(), b.incoh[0].cpu().numpy(), hits, fp64


CASES = [
    # (label, particle, N, n_pol, p_min, p_max, node grid stride, oracle comparison)
    ("c2", None, 320, 2, 0, 3, (5, 2), True),
    ("tile-edge", None, 65, 2, 0, 3, (3, 1), True),
    ("p1-3 one pol", None, 130, 1, 1, 3, (4, 2), True),
    # orders 4 and 5 fold everywhere at this ray density: every node lies in
    # the oracle's 0.1 deg caustic band, so only fused against staged here
    ("p0-5", None, 200, 2, 0, 5, (4, 2), False),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused_matches_staged_and_oracle(R, oracle, case):
    label, part, N, n_pol, p_min, p_max, (st, sp), vs_oracle = case
    w = I.ellipsoid_mixed()
    if part is None:
        part = (w.semi_axes, w.euler_deg, w.m)
    th, ph = w.theta_deg[::st], w.phi_deg[::sp]
    say(f"[fused {label}] N={N} n_pol={n_pol} p={p_min}..{p_max} nodes={len(th)}x{len(ph)}")
    Ff, ncf, incf, hf, ff = _run(R, part, N, n_pol, p_min, p_max, th, ph, staged=False)
    Fs, ncs, incs, hs, fs = _run(R, part, N, n_pol, p_min, p_max, th, ph, staged=True)
    say(f"   hits fused {hf} staged {hs}; FP64 re-traced rays fused {ff} staged {fs}")
    assert hf == hs
    assert np.array_equal(ncf, ncs), "fused and staged hit different nodes"
    inc = incs.sum(axis=0).reshape(len(th), len(ph))
    I_f = (np.abs(Ff) ** 2).sum(axis=(0, 1))
    I_s = (np.abs(Fs) ** 2).sum(axis=(0, 1))
    sel = inc > 0
    d = np.abs(I_f - I_s)[sel] / inc[sel]
    say(f"   fused vs staged: intensity max {d.max(initial=0.0):.2e} over {sel.sum()} nodes")
    assert d.max(initial=0.0) < 1e-4
    if not vs_oracle:
        return
    op = oracle.particle(*part)
    ref = PAR.oracle_farfield(oracle, op, oracle.setup(0.6328, n_pol, p_min, p_max, N), th, ph, mixed=True)
    rel, _ = PAR.compare_mixed(ref, Ff, say=say, tag="fused ")
    assert rel.size > 0.5 * len(th) * len(ph)


def test_fused_tiling_does_not_change_results(R):
    w = I.ellipsoid_mixed()
    part = (w.semi_axes, w.euler_deg, w.m)
    th, ph = w.theta_deg[::6], w.phi_deg[::3]
    ref, ncr, _, hr, fr = _run(R, part, 300, 2, 0, 3, th, ph, staged=False)
    for t in [(256, 1, 0), (1024, 2, 0), (4096, 8, 0), (768, 2, 0)]:
        say(f"[fused tiling] tile_rays={t[0]} blocks_per_cu={t[1]}")
        got, nc, _, h, f = _run(R, part, 300, 2, 0, 3, th, ph, staged=False, tune=R.Tune(*t))
        assert np.array_equal(got.view(np.float32), ref.view(np.float32)), t
        # (the count of FP64 re-traced rays grows with the rays that
        # neighbouring tiles share, so it is not compared)
        assert np.array_equal(nc, ncr) and h == hr, t


def test_fused_finite_radius_matches_staged(R):
    """The general instance (observation at a finite radius) against the staged pipeline."""
    w = I.ellipsoid_mixed()
    part = (w.semi_axes, w.euler_deg, w.m)
    th, ph = w.theta_deg[::6], w.phi_deg[::3]
    Ff, ncf, _, hf, _ = _run(R, part, 200, 2, 0, 3, th, ph, staged=False, robs=150.0)
    Fs, ncs, incs, hs, _ = _run(R, part, 200, 2, 0, 3, th, ph, staged=True, robs=150.0)
    say(f"[fused R=150] hits fused {hf} staged {hs}")
    assert hf == hs and np.array_equal(ncf, ncs)
    inc = incs.sum(axis=0).reshape(len(th), len(ph))
    sel = inc > 0
    d = np.abs((np.abs(Ff) ** 2).sum(axis=(0, 1)) - (np.abs(Fs) ** 2).sum(axis=(0, 1)))[sel] / inc[sel]
    say(f"   fused vs staged: intensity max {d.max(initial=0.0):.2e}")
    assert d.max(initial=0.0) < 1e-4


def test_fused_batch_equals_single_fused_calls(R):
    """A batch of uneven particles through the fused kernel, in one chunk and
    one particle per chunk: every far field bitwise equal to the particle's
    own fused call (keys are per particle, the tiles are the particle's own)."""
    rng = np.random.default_rng(5)
    parts = [I.random_ellipsoid(rng, 15.0, 60.0) for _ in range(6)]
    sides = [48, 130, 65, 96, 40, 200]
    th, ph = I.batch_node_grid()
    inc = R.make_incident(0.6328, 2)
    singles = []
    for part, N in zip(parts, sides):
        b = R.Batch([part], [N], inc, R.make_opts(0, 3, 2, R.MIXED), th, ph, fused=True)
        singles.append((torch.view_as_real(b()[0]).clone(), b.ncontrib[0].clone()))
    for rays_per_chunk in (0, 1):
        say(f"[fused batch] n={len(parts)} sides={sides} rays_per_chunk={rays_per_chunk}")
        b = R.Batch(parts, sides, inc, R.make_opts(0, 3, 2, R.MIXED), th, ph, fused=True,
                    rays_per_chunk=rays_per_chunk)
        F = torch.view_as_real(b()).clone()
        for i, (Fs, ncs) in enumerate(singles):
            assert torch.equal(F[i], Fs), f"particle {i} differs"
            assert torch.equal(b.ncontrib[i], ncs), i
