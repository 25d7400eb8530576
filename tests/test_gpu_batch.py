"""GPU parity of the batched path (rtw_batch): many particles of uneven size in
one call, chunked and traced by the persistent kernel.

Bars:
* Bitwise: every particle's far field and contribution counts equal those of
  rtw_farfield on that particle alone (same kernels, same per-node summation
  order), for any chunking and any tuning.
* Against the FP64 oracle (tests/parity.py): FP64 within 1e-10 relative --
  or, for the large particles of the batch (size parameter up to ~5000),
  within the FP64 rounding of the phase itself (fp64_tol), and near rays whose
  divergence factor is ill-conditioned within COND_C eps cond of the GPU's own
  record -- and mixed within 1e-4 intensity / 1e-3 rad.
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


def _small_batch(seed, n, sides):
    rng = np.random.default_rng(seed)
    parts = [I.random_ellipsoid(rng, 15.0, 60.0) for _ in range(n)]
    return parts, [sides[i % len(sides)] for i in range(n)]


def _single(R, part, N, n_pol, p_min, p_max, prec, th, ph):
    ff = R.FarField(R.make_particle(*part), R.make_incident(0.6328, n_pol), R.make_opts(p_min, p_max, N, prec), th, ph)
    F = ff().clone()
    return F, ff.ncontrib.clone()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_equals_single_particle_calls(R, prec):
    P = R.FP64 if prec == "fp64" else R.MIXED
    th, ph = I.batch_node_grid()
    parts, sides = _small_batch(7, 7, [40, 64, 33, 80, 48])
    for rays_per_chunk in (1, 9000, 0):  # one particle per chunk, a few per chunk, all in one chunk
        say(f"[batch {prec}] n={len(parts)} sides={sides} rays_per_chunk={rays_per_chunk}")
        b = R.Batch(parts, sides, R.make_incident(0.6328, 2), R.make_opts(0, 3, 2, P), th, ph,
                    rays_per_chunk=rays_per_chunk)
        F = b().clone()
        nc = b.ncontrib.clone()
        for i, (part, N) in enumerate(zip(parts, sides)):
            Fs, ncs = _single(R, part, N, 2, 0, 3, P, th, ph)
            assert torch.equal(torch.view_as_real(F[i]), torch.view_as_real(Fs)), f"particle {i} differs"
            assert torch.equal(nc[i], ncs)


def test_batch_tuning_does_not_change_results(R):
    th, ph = I.batch_node_grid()
    parts, sides = _small_batch(11, 5, [56, 40, 72])
    say(f"[batch tuning] sides={sides}")
    b = R.Batch(parts, sides, R.make_incident(0.6328, 2), R.make_opts(0, 3, 2, R.MIXED), th, ph)
    ref = torch.view_as_real(b().clone())
    for t in [(256, 4, 8), (2048, 16, 128), (512, 1, 1)]:
        b.tune = R.Tune(*t)
        got = torch.view_as_real(b().clone())
        assert torch.equal(got, ref), t
    best = b.autotune()
    say(f"   autotune -> tile {best.tile_rays} blocks/CU {best.blocks_per_cu} cand_inline {best.cand_inline}")
    assert best.tile_rays % 256 == 0 and best.blocks_per_cu > 0 and best.cand_inline > 0
    assert torch.equal(torch.view_as_real(b().clone()), ref)


def fp64_tol(axes, m, p_max, k=2 * np.pi / 0.6328):
    """1e-10 relative, or the FP64 rounding of the phase itself when that is
    larger: both sides evaluate a phase of up to Phi = k m 2 (p_max + 1) a_max
    radians, whose last bits differ with the operation order, so fields agree
    to about 50 eps Phi (eps = 2.2e-16).  Above size parameter ~10^3 this
    exceeds 1e-10."""
    phi = k * max(m, 1.0) * 2 * (p_max + 1) * max(axes)
    return max(1e-10, 50 * 2.22e-16 * phi)


def _fp64_allowance(R, part, N, th, ph, tol):
    """Per-node FP64 bound from the GPU's own per-ray conditioning records."""
    rec = R.trace(R.make_particle(*part), R.make_incident(0.6328, 2), R.make_opts(0, 3, N, R.FP64),
                  records=("flags", "dir", "rexit", "cond"))
    rec = {k: v.cpu().numpy() for k, v in rec.items()}
    return PAR.cond_allowance(rec, N, th, ph, tol)


@pytest.mark.parametrize("part_set", range(4))
def test_batch_of_seeded_particles_matches_oracle(oracle, R, part_set):
    """The first 64 particles of the seeded 4096-particle workload (seed 0) at
    their own sizes, 16 per test: each batch call bitwise equal to single calls,
    and every particle against the oracle in both precisions."""
    th, ph = I.batch_node_grid()
    bp = I.batch_particles(4096, seed=0)[16 * part_set:16 * (part_set + 1)]
    parts = [(p.semi_axes, p.euler_deg, p.m) for p in bp]
    sides = [p.grid_n for p in bp]
    say(f"[seeded batch] particles {16 * part_set}..{16 * part_set + 15}, sides {min(sides)}..{max(sides)}")
    got = {}
    for prec, P in (("fp64", R.FP64), ("mixed", R.MIXED)):
        b = R.Batch(parts, sides, R.make_incident(0.6328, 2), R.make_opts(0, 3, 2, P), th, ph,
                    rays_per_chunk=1 << 22)
        F = b().cpu().numpy()
        nc = b.ncontrib.cpu().numpy()
        for i in range(len(parts)):
            Fs, ncs = _single(R, parts[i], sides[i], 2, 0, 3, P, th, ph)
            assert np.array_equal(F[i], Fs.cpu().numpy()), (prec, i)
            assert np.array_equal(nc[i], ncs.cpu().numpy()), (prec, i)
        got[prec] = (F, nc)
        del b
    for i in range(len(parts)):
        ref = PAR.oracle_farfield(oracle, oracle.particle(*parts[i]), oracle.setup(0.6328, 2, 0, 3, sides[i]), th, ph,
                                  mixed=True)
        tol = fp64_tol(parts[i][0], parts[i][2], 3)
        allow, n_ill = _fp64_allowance(R, parts[i], sides[i], th, ph, tol)
        tag = f"particle {16 * part_set + i} N={sides[i]} a_max={max(parts[i][0]):.0f} ({n_ill} ill-conditioned rays) "
        PAR.compare_fp64(ref, got["fp64"][0][i], got["fp64"][1][i], tol, allow, say, tag)
        PAR.compare_mixed(ref, got["mixed"][0][i], say=say, tag=tag)


def test_batch_argument_errors(R):
    th, ph = I.batch_node_grid()
    with pytest.raises(R.RTWError):
        R.Batch([((10.0, 10.0, 10.0), (0, 0, 0), 1.0)], [32], R.make_incident(0.6328, 1),
                R.make_opts(0, 2, 2, R.MIXED), th, ph)  # m = 1
    b = R.Batch([((10.0, 11.0, 12.0), (0, 0, 0), 1.33)], [32], R.make_incident(0.6328, 1),
                R.make_opts(0, 2, 2, R.MIXED), th, ph)
    b.tune = R.Tune(300, 8, 32)  # not a multiple of 256
    with pytest.raises(R.RTWError):
        b.launch()


def test_batch_incoherent_intensity_matches_oracle(oracle, R):
    """Per-node incoherent intensity sum_b |f_b|^2 (the surrogate's training
    quantity) against the oracle's, summed over the two polarisations."""
    th, ph = I.batch_node_grid()
    parts, sides = _small_batch(21, 3, [48, 64, 40])
    for prec, P, tol in (("fp64", R.FP64, 1e-10), ("mixed", R.MIXED, 1e-4)):
        b = R.Batch(parts, sides, R.make_incident(0.6328, 2), R.make_opts(0, 3, 2, P), th, ph, incoherent=True)
        b()
        inc = b.incoh.cpu().numpy().sum(axis=1).reshape(len(parts), th.size, ph.size)
        for i in range(len(parts)):
            ref = PAR.oracle_farfield(oracle, oracle.particle(*parts[i]), oracle.setup(0.6328, 2, 0, 3, sides[i]), th,
                                      ph, mixed=True)
            # FP64 keeps the sheet edges (bit 3); the mixed path drops the nodes within 1e-4 deg of one
            clean = (ref["flags"] & (6 if prec == "fp64" else 14)) == 0
            rel = np.abs(inc[i] - ref["incoh"])[clean] / np.maximum(ref["incoh"][clean], 1e-300)
            rel = rel[ref["incoh"][clean] > 0]
            say(f"[incoherent {prec}] particle {i}: max relative difference {rel.max(initial=0):.2e}")
            assert rel.max(initial=0) < tol
