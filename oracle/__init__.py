"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never does.

Every routine follows the paper (Ren et al., Ray Theory of Waves): the ray
trace applies Eq. 4 (vector Snell), Eq. 8 (Fresnel), Eq. 3 (wavefront
equation) at each interaction, Eq. 6 for the divergence factor and Eqs. 9-10
for the phase; the far field applies the interpolation of the RTW-strategy
section.  See ``rtw_oracle.c`` for the readings taken where the paper is
silent.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

MAX_ORDER = 15


class Particle(ctypes.Structure):
    _fields_ = [("semi_axes", ctypes.c_double * 3), ("euler_deg", ctypes.c_double * 3), ("m", ctypes.c_double),
                ("m_im", ctypes.c_double)]


class Setup(ctypes.Structure):
    _fields_ = [("wavelength", ctypes.c_double), ("n_pol", ctypes.c_int), ("p_min", ctypes.c_int),
                ("p_max", ctypes.c_int), ("grid_n", ctypes.c_int), ("source_distance", ctypes.c_double),
                ("observation_radius", ctypes.c_double), ("corrections", ctypes.c_int)]


CAUSTIC = 1      # uniform Airy form across fold caustics (reading R12)
DIFFRACTION = 2  # forward Fraunhofer diffraction of the shadow (reading R13)


class Emit(ctypes.Structure):
    _fields_ = [("valid", ctypes.c_int), ("nf", ctypes.c_int), ("det_neg", ctypes.c_int), ("tir_any", ctypes.c_int),
                ("dir", ctypes.c_double * 3), ("rexit", ctypes.c_double * 3), ("opl", ctypes.c_double),
                ("phase", ctypes.c_double), ("amp", ctypes.c_double), ("D", ctypes.c_double),
                ("q", ctypes.c_double * 3), ("eperp", ctypes.c_double * 3), ("epar", ctypes.c_double * 3),
                ("jones", ctypes.c_double * 8), ("field", ctypes.c_double * 12), ("obs", ctypes.c_double * 3)]


class Ray(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int), ("n_hits", ctypes.c_int),
                ("hit", (ctypes.c_double * 3) * (MAX_ORDER + 2)),
                ("q_cont", (ctypes.c_double * 3) * (MAX_ORDER + 2)),
                ("eperp_cont", (ctypes.c_double * 3) * (MAX_ORDER + 2)),
                ("dir_cont", (ctypes.c_double * 3) * (MAX_ORDER + 2)),
                ("emit", Emit * (MAX_ORDER + 1))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        ip = P(ctypes.c_int)
        _lib.rtwo_trace_rays.argtypes = [P(Particle), P(Setup), ctypes.c_int, dp, P(Ray)]
        _lib.rtwo_trace_grid.argtypes = [P(Particle), P(Setup), ip, dp, dp, dp, dp, dp]
        _lib.rtwo_farfield.argtypes = [P(Particle), P(Setup), ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_double,
                                       ctypes.c_double, dp, dp, ip, ip, dp]
        _lib.rtwo_grid_halfwidth.argtypes = [P(Particle)]
        _lib.rtwo_grid_halfwidth.restype = ctypes.c_double
        _lib.rtwo_grid_halfwidth_source.argtypes = [P(Particle), ctypes.c_double]
        _lib.rtwo_grid_halfwidth_source.restype = ctypes.c_double
        _lib.rtwo_fresnel.argtypes = [ctypes.c_double, ctypes.c_double, dp]
        _lib.rtwo_set_threads.argtypes = [ctypes.c_int]
        _lib.rtwo_airy_neg.argtypes = [ctypes.c_double, dp, dp]
        _lib.rtwo_bessel_j1.argtypes = [ctypes.c_double]
        _lib.rtwo_bessel_j1.restype = ctypes.c_double
        _lib.rtwo_get_threads.restype = ctypes.c_int
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if a is not None else None


def particle(semi_axes, euler_deg=(0.0, 0.0, 0.0), m=1.333, m_im=0.0):
    """m: real part of the index; m_im >= 0 its imaginary part (weak absorption, reading R14)."""
    p = Particle()
    p.m_im = float(m_im)
    p.semi_axes[:] = [float(v) for v in semi_axes]
    p.euler_deg[:] = [float(v) for v in euler_deg]
    p.m = float(m)
    return p


def setup(wavelength=0.6328, n_pol=1, p_min=0, p_max=2, grid_n=64, source_distance=0.0, observation_radius=0.0,
          corrections=0):
    """Trace settings; source_distance > 0 puts a point source at lab (0, 0, -source_distance);
    observation_radius > 0 observes on the sphere of that radius instead of the far field;
    corrections: CAUSTIC | DIFFRACTION."""
    s = Setup()
    s.corrections = int(corrections)
    s.source_distance = float(source_distance)
    s.observation_radius = float(observation_radius)
    s.wavelength = float(wavelength)
    s.n_pol = int(n_pol)
    s.p_min = int(p_min)
    s.p_max = int(p_max)
    s.grid_n = int(grid_n)
    return s


def set_threads(n):
    lib().rtwo_set_threads(int(n))


def get_threads():
    return lib().rtwo_get_threads()


def grid_halfwidth(part, source_distance=0.0):
    """Half-width of the incident grid (um), widened for a point source."""
    return lib().rtwo_grid_halfwidth_source(ctypes.byref(part), float(source_distance))


def trace_rays(part, st, xy):
    """Trace rays entering at lab points xy[i] = (x, y).  Returns a ctypes array of Ray."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    n = xy.shape[0]
    out = (Ray * max(n, 1))()
    rc = lib().rtwo_trace_rays(ctypes.byref(part), ctypes.byref(st), n, _dp(xy), out)
    if rc != 0:
        raise ValueError("rtwo_trace_rays rejected its arguments")
    return out


def airy_neg(z):
    """(Ai(-z), Ai'(-z)) for z >= 0."""
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().rtwo_airy_neg(float(z), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def bessel_j1(x):
    return lib().rtwo_bessel_j1(float(x))


def fresnel(m_rel, ci):
    out = np.zeros(10)
    lib().rtwo_fresnel(float(m_rel), float(ci), _dp(out))
    c = out[0::2] + 1j * out[1::2]
    return dict(r_perp=c[0], r_par=c[1], t_perp=c[2], t_par=c[3], krn_over_kin=c[4])


def trace_grid(part, st):
    """Per-ray records on the full cell-centred grid (see rtwo_trace_grid)."""
    N = st.grid_n
    n_ord = st.p_max - st.p_min + 1
    NN = N * N
    flags = np.zeros((n_ord, NN), np.int32)
    d = np.zeros((n_ord, 3, NN))
    r = np.zeros((n_ord, 3, NN))
    ph = np.zeros((n_ord, NN))
    amp = np.zeros((n_ord, NN))
    field = np.zeros((n_ord, st.n_pol, 3, 2, NN))
    rc = lib().rtwo_trace_grid(ctypes.byref(part), ctypes.byref(st), _ip(flags), _dp(d), _dp(r), _dp(ph), _dp(amp),
                               _dp(field))
    if rc != 0:
        raise ValueError("rtwo_trace_grid rejected its arguments")
    return dict(flags=flags, dir=d, rexit=r, phase=ph, amp=amp, field=field)


def farfield(part, st, theta_deg, phi_deg, band_deg=0.1, edge_band_deg=None):
    """Far field F(theta, phi) (um): complex array [n_pol, 2 (theta, phi), n_theta, n_phi],
    plus per-node incoherent sums, flags and contribution counts.  band_deg is the
    width of the caustic and pole bands (flag bits 1, 2), edge_band_deg that of
    the sheet-edge band (bit 3; None: band_deg)."""
    if edge_band_deg is None:
        edge_band_deg = band_deg
    th = np.ascontiguousarray(theta_deg, dtype=np.float64)
    ph = np.ascontiguousarray(phi_deg, dtype=np.float64)
    nt, nphi = th.size, ph.size
    field = np.zeros((st.n_pol, 2, nt, nphi, 2))
    incoh = np.zeros(nt * nphi)
    nflags = np.zeros(nt * nphi, np.int32)
    ncon = np.zeros(nt * nphi, np.int32)
    unc = np.zeros(nt * nphi)
    rc = lib().rtwo_farfield(ctypes.byref(part), ctypes.byref(st), nt, _dp(th), nphi, _dp(ph), float(band_deg),
                             float(edge_band_deg), _dp(field), _dp(incoh), _ip(nflags), _ip(ncon), _dp(unc))
    if rc != 0:
        raise ValueError("rtwo_farfield rejected its arguments")
    F = field[..., 0] + 1j * field[..., 1]
    return dict(field=F, incoh=incoh.reshape(nt, nphi), flags=nflags.reshape(nt, nphi),
                ncontrib=ncon.reshape(nt, nphi), uncancelled=unc.reshape(nt, nphi), band_deg=float(band_deg),
                edge_band_deg=float(edge_band_deg))


def ray_emit(ray, p):
    """Python view of one emitted order of a traced ray."""
    e = ray.emit[p]
    j = np.array(e.jones[:]).reshape(2, 2, 2)
    f = np.array(e.field[:]).reshape(2, 3, 2)
    return dict(valid=bool(e.valid), nf=e.nf, det_neg=bool(e.det_neg), tir_any=bool(e.tir_any),
                dir=np.array(e.dir[:]), rexit=np.array(e.rexit[:]), opl=e.opl, phase=e.phase, amp=e.amp, D=e.D,
                q=np.array(e.q[:]), eperp=np.array(e.eperp[:]), epar=np.array(e.epar[:]),
                jones=j[..., 0] + 1j * j[..., 1], field=f[..., 0] + 1j * f[..., 1])
