"""Seeded synthetic inputs shared by the HIP path, its tests and the oracle tests.

This module holds input generation only -- particle parameters, observation
grids and the batched-particle sampler.  It contains none of the method's
arithmetic.  All workloads are analytic ellipsoids, so no dataset is needed.

Workloads (sizes of the ray and node grids, orders, polarisations):

* ``sphere_fp64``      sphere a=b=c=50 um, m=1.333, lambda=0.6328 um, x-polarised,
  p=0..2, 512x512 rays, nodes theta 0..180 step 1 deg x phi 0..359 step 1 deg.
* ``ellipsoid_mixed``  ellipsoid 60/50/40 um, ZYZ Euler (30,20,10) deg, m=1.333,
  p=0..3, 2048x2048 rays, nodes theta 0..180 step 0.1 deg x phi 0..359.5 step
  0.5 deg, x and y polarisations.
* ``large_ellipsoid``  ellipsoid 1000/950/900 um, Euler (0,0,0), m=1.333, p=0..5,
  8192x8192 rays, theta 0..119.5 step 0.5, 120..170 step 0.02, 170.5..180 step
  0.5 deg, phi 0..359.5 step 0.5 deg, x-polarised.
* ``paper_spheroid``   the paper's own spheroid: a=b=100, c=90 um, m=1.333,
  plane wave along the particle's x axis (Euler (0, 90, 180): lab z = body x,
  lab x = body z), x-polarised, p=0..3, 3456x3456 rays (the ray density of
  ``ellipsoid_mixed``), nodes theta 0..180 x phi 0..359.99 step 0.01 deg
  (18001 x 36000, the paper's 0.01 deg angular resolution).
* ``batch``            4096 ellipsoids drawn with SplitMix64 from seed 0
  (``batch_particles``), p=0..3, ray-grid side proportional to size, nodes
  theta 0..180 step 0.5 x phi 0..358 step 2 deg, x and y polarisations.
"""
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

WAVELENGTH = 0.6328  # um, He-Ne, in the surrounding medium


@dataclass
class Workload:
    name: str
    semi_axes: Tuple[float, float, float]
    euler_deg: Tuple[float, float, float]
    m: float
    wavelength: float
    p_min: int
    p_max: int
    grid_n: int
    n_pol: int
    theta_deg: np.ndarray = field(repr=False)
    phi_deg: np.ndarray = field(repr=False)

    @property
    def n_nodes(self) -> int:
        return int(self.theta_deg.size * self.phi_deg.size)


def uniform_angles(start: float, stop: float, step: float) -> np.ndarray:
    """start, start+step, ... <= stop (inclusive), each value i*step + start."""
    n = int(round((stop - start) / step)) + 1
    return start + step * np.arange(n, dtype=np.float64)


def sphere_fp64(grid_n: int = 512) -> Workload:
    return Workload("sphere_fp64", (50.0, 50.0, 50.0), (0.0, 0.0, 0.0), 1.333, WAVELENGTH, 0, 2, grid_n, 1,
                    uniform_angles(0.0, 180.0, 1.0), uniform_angles(0.0, 359.0, 1.0))


def ellipsoid_mixed(grid_n: int = 2048) -> Workload:
    return Workload("ellipsoid_mixed", (60.0, 50.0, 40.0), (30.0, 20.0, 10.0), 1.333, WAVELENGTH, 0, 3, grid_n, 2,
                    uniform_angles(0.0, 180.0, 0.1), uniform_angles(0.0, 359.5, 0.5))


def large_theta_grid() -> np.ndarray:
    return np.concatenate([uniform_angles(0.0, 119.5, 0.5), uniform_angles(120.0, 170.0, 0.02),
                           uniform_angles(170.5, 180.0, 0.5)])


def large_ellipsoid(grid_n: int = 8192) -> Workload:
    return Workload("large_ellipsoid", (1000.0, 950.0, 900.0), (0.0, 0.0, 0.0), 1.333, WAVELENGTH, 0, 5, grid_n, 1,
                    large_theta_grid(), uniform_angles(0.0, 359.5, 0.5))


def paper_spheroid(grid_n: int = 3456) -> Workload:
    return Workload("paper_spheroid", (100.0, 100.0, 90.0), (0.0, 90.0, 180.0), 1.333, WAVELENGTH, 0, 3, grid_n, 1,
                    uniform_angles(0.0, 180.0, 0.01), uniform_angles(0.0, 359.99, 0.01))


def batch_node_grid() -> Tuple[np.ndarray, np.ndarray]:
    return uniform_angles(0.0, 180.0, 0.5), uniform_angles(0.0, 358.0, 2.0)


# --------------------------------------------------------------------------
# SplitMix64 (Steele, Lea, Flood 2014) -- the batched-particle sampler
# --------------------------------------------------------------------------
_MASK = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """53-bit uniform in [0, 1)."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def _quat_to_zyz_deg(q) -> Tuple[float, float, float]:
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                  [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                  [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    beta = np.arccos(np.clip(R[2, 2], -1.0, 1.0))
    alpha = np.arctan2(R[1, 2], R[0, 2])
    gamma = np.arctan2(R[2, 1], -R[2, 0])
    return tuple(float(np.degrees(v)) for v in (alpha, beta, gamma))


@dataclass
class BatchParticle:
    semi_axes: Tuple[float, float, float]
    euler_deg: Tuple[float, float, float]
    m: float
    grid_n: int
    mean_radius: float


def batch_particles(n: int = 4096, seed: int = 0) -> List[BatchParticle]:
    """Ellipsoids with volume-equivalent radius U[20,500] um, axis ratios b/a,
    c/a ~ U[0.8,1.2], orientation uniform on SO(3) (Shoemake's uniform
    quaternion), m ~ U[1.30,1.50]; ray-grid side N = clamp(64 round(4.096
    rbar / 64), 256, 2048).  Draw order per particle: rbar, b/a, c/a, u1, u2,
    u3, m."""
    rng = SplitMix64(seed)
    out = []
    for _ in range(n):
        rbar = 20.0 + 480.0 * rng.uniform()
        ba = 0.8 + 0.4 * rng.uniform()
        ca = 0.8 + 0.4 * rng.uniform()
        u1, u2, u3 = rng.uniform(), rng.uniform(), rng.uniform()
        m = 1.30 + 0.20 * rng.uniform()
        a = rbar / (ba * ca) ** (1.0 / 3.0)
        q = (np.sqrt(1 - u1) * np.sin(2 * np.pi * u2), np.sqrt(1 - u1) * np.cos(2 * np.pi * u2),
             np.sqrt(u1) * np.sin(2 * np.pi * u3), np.sqrt(u1) * np.cos(2 * np.pi * u3))
        q = (q[3], q[0], q[1], q[2])  # (w, x, y, z)
        n_side = int(min(2048, max(256, 64 * round(4.096 * rbar / 64.0))))
        out.append(BatchParticle((a, ba * a, ca * a), _quat_to_zyz_deg(q), m, n_side, rbar))
    return out


def random_ellipsoid(rng: np.random.Generator, r_lo=20.0, r_hi=80.0):
    """A random small ellipsoid for parity tests: (semi_axes, euler_deg, m)."""
    r = rng.uniform(r_lo, r_hi)
    ratios = rng.uniform(0.8, 1.2, size=3)
    axes = tuple(float(v) for v in r * ratios)
    euler = tuple(float(v) for v in rng.uniform(-180.0, 180.0, size=3))
    m = float(rng.uniform(1.30, 1.50))
    return axes, euler, m
