"""Thin ctypes binding of librtw.so (include/rtw.h).

Argument marshalling only: PyTorch tensors provide device memory and the HIP
stream; every step of the method runs in the library's kernels.  If the built
library is missing, loading raises -- there is no fallback.
"""
import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

from . import build as _build

RTW_OK = 0
RTW_ERR_INVALID_ARG = -1
RTW_ERR_UNSUPPORTED = -2
RTW_ERR_WORKSPACE = -3
RTW_ERR_DEVICE = -4
FP64 = 0
MIXED = 1
MAX_ORDER = 15


class Particle(ctypes.Structure):
    _fields_ = [("semi_axes", ctypes.c_double * 3), ("euler_deg", ctypes.c_double * 3), ("m", ctypes.c_double),
                ("m_im", ctypes.c_double)]


class Incident(ctypes.Structure):
    _fields_ = [("wavelength", ctypes.c_double), ("n_pol", ctypes.c_int), ("source_distance", ctypes.c_double),
                ("observation_radius", ctypes.c_double)]


class TraceOpts(ctypes.Structure):
    _fields_ = [("p_min", ctypes.c_int), ("p_max", ctypes.c_int), ("grid_n", ctypes.c_int),
                ("precision", ctypes.c_int), ("corrections", ctypes.c_int)]


CAUSTIC = 1      # uniform Airy form at fold caustics
DIFFRACTION = 2  # forward Fraunhofer diffraction of the shadow


class Grid(ctypes.Structure):
    _fields_ = [("n_theta", ctypes.c_int), ("theta_deg", ctypes.c_void_p), ("n_phi", ctypes.c_int),
                ("phi_deg", ctypes.c_void_p)]


class RayRecords(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_void_p), ("dir", ctypes.c_void_p), ("rexit", ctypes.c_void_p),
                ("phase", ctypes.c_void_p), ("amp", ctypes.c_void_p), ("field", ctypes.c_void_p),
                ("cond", ctypes.c_void_p)]


class Tune(ctypes.Structure):
    _fields_ = [("tile_rays", ctypes.c_int), ("blocks_per_cu", ctypes.c_int), ("cand_inline", ctypes.c_int)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("rays_per_chunk", ctypes.c_longlong), ("hits_per_node", ctypes.c_double), ("fused", ctypes.c_int)]


EXPORTED = ["rtw_trace", "rtw_farfield_workspace_size", "rtw_farfield", "rtw_farfield_static", "rtw_farfield_status",
            "rtw_farfield_stats", "rtw_batch_workspace_size", "rtw_batch", "rtw_batch_autotune",
            "rtw_profile_enable", "rtw_profile_read", "rtw_profile_only", "rtw_last_error", "rtw_version"]

_lib = None


class RTWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rtw error {code}: {msg}")
        self.code = code


def lib_path() -> str:
    return _build.LIB


def load():
    """Load librtw.so (built in-tree by paper_2403_13856_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"librtw.so not built ({path}); run `python -m paper_2403_13856_amd.build`")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.rtw_trace.argtypes = [P(Particle), P(Incident), P(TraceOpts), P(RayRecords), ctypes.c_void_p]
    L.rtw_farfield_workspace_size.argtypes = [P(Particle), P(Incident), P(TraceOpts), P(Grid), ctypes.c_double,
                                              P(ctypes.c_size_t)]
    L.rtw_farfield.argtypes = [P(Particle), P(Incident), P(TraceOpts), P(Grid), ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    L.rtw_farfield_static.argtypes = [P(Particle), P(Incident), P(TraceOpts), P(Grid), ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.rtw_farfield_status.argtypes = [ctypes.c_void_p, ctypes.c_void_p, P(ctypes.c_size_t)]
    L.rtw_batch_workspace_size.argtypes = [ctypes.c_int, P(Particle), P(ctypes.c_int), P(Incident), P(TraceOpts),
                                           P(Grid), P(BatchOpts), P(ctypes.c_size_t)]
    L.rtw_batch.argtypes = [ctypes.c_int, P(Particle), P(ctypes.c_int), P(Incident), P(TraceOpts), P(Grid),
                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, P(Tune), P(BatchOpts), ctypes.c_void_p,
                            ctypes.c_size_t, ctypes.c_void_p]
    L.rtw_batch_autotune.argtypes = [ctypes.c_int, P(Particle), P(ctypes.c_int), P(Incident), P(TraceOpts),
                                     P(Grid), P(BatchOpts), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p, P(Tune)]
    L.rtw_farfield_stats.argtypes = [ctypes.c_void_p, ctypes.c_void_p, P(ctypes.c_uint64), P(ctypes.c_uint64)]
    L.rtw_profile_enable.argtypes = [ctypes.c_int]
    L.rtw_profile_only.argtypes = [ctypes.c_char_p]
    L.rtw_profile_read.argtypes = [ctypes.c_int, ctypes.c_char_p, P(ctypes.c_double), P(ctypes.c_int),
                                   P(ctypes.c_int)]
    L.rtw_last_error.restype = ctypes.c_char_p
    L.rtw_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != RTW_OK:
        raise RTWError(rc, load().rtw_last_error().decode())


def profile_enable(on: bool = True):
    """Bracket every library kernel with HIP events on its stream (for benchmarks)."""
    _check(load().rtw_profile_enable(1 if on else 0))


def profile_only(name=None):
    """Record events only for the kernel reported under this name (None: every kernel)."""
    _check(load().rtw_profile_only(name.encode() if name else None))


def profile_read(max_kernels: int = 32):
    """{kernel name: (total ms, launches)} of the kernels recorded since the last read."""
    names = ctypes.create_string_buffer(64 * max_kernels)
    ms = (ctypes.c_double * max_kernels)()
    cnt = (ctypes.c_int * max_kernels)()
    n = ctypes.c_int(0)
    _check(load().rtw_profile_read(max_kernels, names, ms, cnt, ctypes.byref(n)))
    out = {}
    for i in range(min(n.value, max_kernels)):
        nm = names.raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode()
        out[nm] = (ms[i], cnt[i])
    return out


def make_particle(semi_axes: Sequence[float], euler_deg: Sequence[float] = (0, 0, 0), m: float = 1.333,
                  m_im: float = 0.0):
    """m: real part of the index; m_im >= 0 its imaginary part (weak absorption)."""
    p = Particle()
    p.m_im = float(m_im)
    p.semi_axes[:] = [float(v) for v in semi_axes]
    p.euler_deg[:] = [float(v) for v in euler_deg]
    p.m = float(m)
    return p


def make_incident(wavelength: float = 0.6328, n_pol: int = 1, source_distance: float = 0.0,
                  observation_radius: float = 0.0):
    """Incident wave: a plane wave along +z, or (source_distance > 0) a point source at lab (0, 0, -source_distance);
    observation_radius > 0 puts the nodes on the sphere of that radius instead of the far field."""
    inc = Incident()
    inc.wavelength = float(wavelength)
    inc.n_pol = int(n_pol)
    inc.source_distance = float(source_distance)
    inc.observation_radius = float(observation_radius)
    return inc


def make_opts(p_min=0, p_max=2, grid_n=64, precision=FP64, corrections=0):
    o = TraceOpts()
    o.p_min, o.p_max, o.grid_n, o.precision = int(p_min), int(p_max), int(grid_n), int(precision)
    o.corrections = int(corrections)
    return o


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


RECORD_NAMES = ("flags", "dir", "rexit", "phase", "amp", "field", "cond")


def trace(part, inc, opts, device="cuda", stream=None, records=RECORD_NAMES):
    """Per-ray records of every emitted order (rtw_trace); FP64 tensors on the
    device, for the record names listed (the others are not written)."""
    import torch
    N = opts.grid_n
    n_ord = opts.p_max - opts.p_min + 1
    NN = N * N
    shapes = dict(flags=(n_ord, NN), dir=(n_ord, 3, NN), rexit=(n_ord, 3, NN), phase=(n_ord, NN), amp=(n_ord, NN),
                  field=(n_ord, inc.n_pol, 3, 2, NN), cond=(n_ord, 2, NN))
    out = {k: torch.empty(shapes[k], dtype=torch.int32 if k == "flags" else torch.float64, device=device)
           for k in RECORD_NAMES if k in records}
    rec = RayRecords(*[_ptr(out.get(k)) for k in RECORD_NAMES])
    _check(load().rtw_trace(ctypes.byref(part), ctypes.byref(inc), ctypes.byref(opts), ctypes.byref(rec),
                            _stream_ptr(stream)))
    return out


@dataclass
class FarField:
    """Reusable far-field evaluator: owns the node-angle tensors and the workspace."""
    part: Particle
    inc: Incident
    opts: TraceOpts
    theta_deg: "object"
    phi_deg: "object"
    hits_per_node: float = 6.0
    device: str = "cuda"

    def __post_init__(self):
        import torch
        self.theta = torch.as_tensor(self.theta_deg, dtype=torch.float64, device=self.device).contiguous()
        self.phi = torch.as_tensor(self.phi_deg, dtype=torch.float64, device=self.device).contiguous()
        self.grid = Grid(self.theta.numel(), self.theta.data_ptr(), self.phi.numel(), self.phi.data_ptr())
        n = ctypes.c_size_t(0)
        _check(load().rtw_farfield_workspace_size(ctypes.byref(self.part), ctypes.byref(self.inc),
                                                  ctypes.byref(self.opts), ctypes.byref(self.grid),
                                                  float(self.hits_per_node), ctypes.byref(n)))
        self._alloc(n.value)
        dt = torch.float64 if self.opts.precision == FP64 else torch.float32
        self.out = torch.empty((self.inc.n_pol, 2, self.theta.numel(), self.phi.numel(), 2), dtype=dt,
                               device=self.device)
        self.ncontrib = torch.empty((self.theta.numel(), self.phi.numel()), dtype=torch.int32, device=self.device)

    def _alloc(self, nbytes):
        import torch
        self.ws_bytes = int(nbytes)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255

    def launch(self, stream=None, with_counts=True):
        """Enqueue one far-field evaluation (asynchronous)."""
        _check(load().rtw_farfield(ctypes.byref(self.part), ctypes.byref(self.inc), ctypes.byref(self.opts),
                                   ctypes.byref(self.grid), _ptr(self.out),
                                   _ptr(self.ncontrib) if with_counts else None,
                                   ctypes.c_void_p(self.ws_ptr), ctypes.c_size_t(self.ws_bytes),
                                   _stream_ptr(stream)))

    def status(self, stream=None):
        """RTW_OK or RTW_ERR_WORKSPACE (synchronises the stream); returns (code, bytes_needed)."""
        need = ctypes.c_size_t(0)
        rc = load().rtw_farfield_status(ctypes.c_void_p(self.ws_ptr), _stream_ptr(stream), ctypes.byref(need))
        if rc not in (RTW_OK, RTW_ERR_WORKSPACE):
            _check(rc)
        return rc, need.value

    def stats(self, stream=None):
        """(node contributions, rays re-traced in FP64) of the last evaluation (synchronises)."""
        hits, fp64 = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(load().rtw_farfield_stats(ctypes.c_void_p(self.ws_ptr), _stream_ptr(stream), ctypes.byref(hits),
                                         ctypes.byref(fp64)))
        return hits.value, fp64.value

    def __call__(self, stream=None, with_counts=True):
        """Evaluate, growing the workspace and re-running if the hit pool overflowed."""
        for _ in range(4):
            self.launch(stream, with_counts)
            rc, need = self.status(stream)
            if rc == RTW_OK:
                return self.field()
            self._alloc(max(need, 2 * self.ws_bytes))
        raise RTWError(RTW_ERR_WORKSPACE, "hit pool kept overflowing")

    def field(self):
        """Complex view [n_pol, 2 (theta, phi), n_theta, n_phi]."""
        import torch
        return torch.view_as_complex(self.out)


def farfield_static(part, inc, opts, theta, phi, out, ncontrib=None, status=None, stream=None):
    """rtw_farfield_static: the far field with the library's static workspace
    (no device allocation).  theta, phi: device float64 node angles (deg); out:
    device [n_pol, 2, n_theta, n_phi, 2] (float64 for FP64, float32 for MIXED);
    ncontrib: device int32 [n_theta, n_phi] or None; status: device int32 [1]
    or None (RTW_OK, or RTW_ERR_WORKSPACE on hit-pool overflow)."""
    grid = Grid(theta.numel(), theta.data_ptr(), phi.numel(), phi.data_ptr())
    _check(load().rtw_farfield_static(ctypes.byref(part), ctypes.byref(inc), ctypes.byref(opts), ctypes.byref(grid),
                                      _ptr(out), _ptr(ncontrib), _ptr(status), _stream_ptr(stream)))


@dataclass
class Batch:
    """Far fields of many particles in one rtw_batch call (device output
    [n, n_pol, 2, n_theta, n_phi] complex).  particles: (semi_axes, euler_deg,
    m) triples; grid_n: ray-grid side of each."""
    particles: Sequence
    grid_n: Sequence[int]
    inc: Incident
    opts: TraceOpts
    theta_deg: "object"
    phi_deg: "object"
    rays_per_chunk: int = 0
    hits_per_node: float = 0.0
    tune: Optional[Tune] = None
    device: str = "cuda"
    allocate: bool = True  # False: describe the particles only (no workspace or output)
    incoherent: bool = False  # also return per-node incoherent intensities (self.incoh)
    m_im: Optional[Sequence[float]] = None  # imaginary parts of the indices (None: all 0)
    fused: bool = False  # the fused kernel where it applies (mixed, <= 6 orders, no caustic correction)

    def __post_init__(self):
        import torch
        n = len(self.particles)
        self.n = n
        mi = [0.0] * n if self.m_im is None else [float(x) for x in self.m_im]
        self.parts = (Particle * n)(*[make_particle(a, e, m, mi[i]) for i, (a, e, m) in enumerate(self.particles)])
        self.gn = (ctypes.c_int * n)(*[int(g) for g in self.grid_n])
        self.bopts = BatchOpts(int(self.rays_per_chunk), float(self.hits_per_node), 1 if self.fused else 0)
        self.theta = torch.as_tensor(self.theta_deg, dtype=torch.float64, device=self.device).contiguous()
        self.phi = torch.as_tensor(self.phi_deg, dtype=torch.float64, device=self.device).contiguous()
        self.grid = Grid(self.theta.numel(), self.theta.data_ptr(), self.phi.numel(), self.phi.data_ptr())
        if not self.allocate:
            return
        nb = ctypes.c_size_t(0)
        _check(load().rtw_batch_workspace_size(n, self.parts, self.gn, ctypes.byref(self.inc), ctypes.byref(self.opts),
                                               ctypes.byref(self.grid), ctypes.byref(self.bopts), ctypes.byref(nb)))
        self._alloc(nb.value)
        dt = torch.float64 if self.opts.precision == FP64 else torch.float32
        self.out = torch.empty((n, self.inc.n_pol, 2, self.theta.numel(), self.phi.numel(), 2), dtype=dt,
                               device=self.device)
        self.ncontrib = torch.empty((n, self.theta.numel(), self.phi.numel()), dtype=torch.int32, device=self.device)
        self.incoh = torch.empty((n, self.inc.n_pol, self.theta.numel() * self.phi.numel()), dtype=dt,
                                 device=self.device) if self.incoherent else None

    def _alloc(self, nbytes):
        import torch
        self.ws_bytes = int(nbytes)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) & ~255

    def launch(self, stream=None, with_counts=True):
        _check(load().rtw_batch(self.n, self.parts, self.gn, ctypes.byref(self.inc), ctypes.byref(self.opts),
                                ctypes.byref(self.grid), _ptr(self.out), _ptr(self.ncontrib) if with_counts else None,
                                _ptr(self.incoh), ctypes.byref(self.tune) if self.tune is not None else None,
                                ctypes.byref(self.bopts),
                                ctypes.c_void_p(self.ws_ptr), ctypes.c_size_t(self.ws_bytes), _stream_ptr(stream)))

    def autotune(self, stream=None):
        """Run the library's autotuner on this batch and keep its choice."""
        best = Tune()
        _check(load().rtw_batch_autotune(self.n, self.parts, self.gn, ctypes.byref(self.inc), ctypes.byref(self.opts),
                                         ctypes.byref(self.grid), ctypes.byref(self.bopts), _ptr(self.out),
                                         ctypes.c_void_p(self.ws_ptr), ctypes.c_size_t(self.ws_bytes),
                                         _stream_ptr(stream), ctypes.byref(best)))
        self.tune = best
        return best

    def status(self, stream=None):
        need = ctypes.c_size_t(0)
        rc = load().rtw_farfield_status(ctypes.c_void_p(self.ws_ptr), _stream_ptr(stream), ctypes.byref(need))
        if rc not in (RTW_OK, RTW_ERR_WORKSPACE):
            _check(rc)
        return rc, need.value

    def stats(self, stream=None):
        hits, fp64 = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(load().rtw_farfield_stats(ctypes.c_void_p(self.ws_ptr), _stream_ptr(stream), ctypes.byref(hits),
                                         ctypes.byref(fp64)))
        return hits.value, fp64.value

    def __call__(self, stream=None, with_counts=True):
        for _ in range(4):
            self.launch(stream, with_counts)
            rc, need = self.status(stream)
            if rc == RTW_OK:
                return self.field()
            self._alloc(max(need, 2 * self.ws_bytes))
        raise RTWError(RTW_ERR_WORKSPACE, "hit pool kept overflowing")

    def field(self):
        import torch
        return torch.view_as_complex(self.out)


# ---------------------------------------------------------------------------
# learned surrogate (include/rtw_surrogate.h)
# ---------------------------------------------------------------------------
SURROGATE_EXPORTED = ["rtw_surrogate_last_error", "rtw_surrogate_param_count", "rtw_surrogate_create",
                      "rtw_surrogate_destroy", "rtw_surrogate_set_normalization", "rtw_surrogate_get_params",
                      "rtw_surrogate_set_params", "rtw_surrogate_forward", "rtw_surrogate_forward_layered",
                      "rtw_surrogate_grad",
                      "rtw_surrogate_get_grads", "rtw_surrogate_train_step", "rtw_surrogate_features",
                      "rtw_cell_log_intensity", "rtw_surrogate_query_scratch_size", "rtw_surrogate_query"]
EXPORTED = EXPORTED + SURROGATE_EXPORTED
N_FEATURES, WIDTH, DEPTH = 9, 512, 6


class Cells(ctypes.Structure):
    _fields_ = [("n_theta_cells", ctypes.c_int), ("theta0_deg", ctypes.c_double), ("dtheta_deg", ctypes.c_double),
                ("n_phi_cells", ctypes.c_int), ("phi0_deg", ctypes.c_double), ("dphi_deg", ctypes.c_double)]

    def centres(self):
        import numpy as np
        tc = self.theta0_deg + (np.arange(self.n_theta_cells) + 0.5) * self.dtheta_deg
        pc = self.phi0_deg + (np.arange(self.n_phi_cells) + 0.5) * self.dphi_deg
        T, P = np.meshgrid(tc, pc, indexing="ij")
        return T.ravel(), P.ravel()


_slib = None


def sload():
    global _slib
    if _slib is not None:
        return _slib
    L = load()
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.rtw_surrogate_last_error.restype = ctypes.c_char_p
    L.rtw_surrogate_param_count.argtypes = [P(ctypes.c_size_t)]
    L.rtw_surrogate_create.argtypes = [ctypes.c_uint64, ctypes.c_int, P(vp)]
    L.rtw_surrogate_destroy.argtypes = [vp]
    L.rtw_surrogate_set_normalization.argtypes = [vp, P(ctypes.c_float), P(ctypes.c_float), P(ctypes.c_float),
                                                  P(ctypes.c_float)]
    L.rtw_surrogate_get_params.argtypes = [vp, P(ctypes.c_float), ctypes.c_size_t]
    L.rtw_surrogate_set_params.argtypes = [vp, P(ctypes.c_float), ctypes.c_size_t]
    L.rtw_surrogate_get_grads.argtypes = [vp, P(ctypes.c_float), ctypes.c_size_t]
    L.rtw_surrogate_save.argtypes = [vp, ctypes.c_char_p]
    L.rtw_surrogate_load.argtypes = [vp, ctypes.c_char_p]
    L.rtw_surrogate_forward.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.rtw_surrogate_forward_layered.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.rtw_surrogate_grad.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.rtw_surrogate_train_step.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_float, vp, vp]
    L.rtw_surrogate_features.argtypes = [ctypes.c_int, P(Particle), P(Incident), ctypes.c_int, P(ctypes.c_double),
                                         P(ctypes.c_double), P(ctypes.c_float)]
    L.rtw_cell_log_intensity.argtypes = [ctypes.c_int, vp, ctypes.c_int, P(Grid), P(Cells), vp, vp]
    L.rtw_surrogate_query_scratch_size.argtypes = [ctypes.c_int, P(Particle), P(ctypes.c_int), P(Incident),
                                                   P(TraceOpts), P(Grid), P(Cells), P(ctypes.c_size_t)]
    L.rtw_surrogate_query.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_float, ctypes.c_int, P(Particle),
                                      P(ctypes.c_int), P(Incident), P(TraceOpts), P(Grid), P(Cells), P(Tune), vp, vp,
                                      vp, vp, ctypes.c_size_t, P(ctypes.c_int), vp]
    _slib = L
    return L


def _scheck(rc):
    if rc != RTW_OK:
        raise RTWError(rc, sload().rtw_surrogate_last_error().decode())


def param_count():
    n = ctypes.c_size_t(0)
    _scheck(sload().rtw_surrogate_param_count(ctypes.byref(n)))
    return n.value


def surrogate_features(particles, inc, cells):
    """Host features [n_part * n_cells, 9] (float32) of every (particle, cell)."""
    import numpy as np
    n = len(particles)
    parts = (Particle * n)(*[make_particle(a, e, m) for (a, e, m) in particles])
    tc, pc = cells.centres()
    tc = np.ascontiguousarray(tc, dtype=np.float64)
    pc = np.ascontiguousarray(pc, dtype=np.float64)
    out = np.empty((n, tc.size, N_FEATURES), dtype=np.float32)
    _scheck(sload().rtw_surrogate_features(n, parts, ctypes.byref(inc), tc.size,
                                           tc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           pc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out.reshape(-1, N_FEATURES)


def cell_log_intensity(batch, cells, stream=None):
    """ln cell-mean incoherent intensity [n_part, n_cells, n_pol] of a computed
    Batch made with incoherent=True (mixed precision)."""
    import torch
    if batch.incoh is None or batch.incoh.dtype != torch.float32:
        raise ValueError("needs a mixed-precision Batch with incoherent=True")
    n_cells = cells.n_theta_cells * cells.n_phi_cells
    out = torch.empty((batch.n, n_cells, batch.inc.n_pol), dtype=torch.float32, device=batch.device)
    _scheck(sload().rtw_cell_log_intensity(batch.n, _ptr(batch.incoh), batch.inc.n_pol, ctypes.byref(batch.grid),
                                           ctypes.byref(cells), _ptr(out), _stream_ptr(stream)))
    return out


class Surrogate:
    """Handle of the BF16 MLP surrogate (rtw_surrogate_*)."""

    def __init__(self, seed=0, max_rows=65536):
        self.h = ctypes.c_void_p(0)
        _scheck(sload().rtw_surrogate_create(int(seed), int(max_rows), ctypes.byref(self.h)))
        self.max_rows = max_rows

    def close(self):
        if self.h:
            sload().rtw_surrogate_destroy(self.h)
            self.h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_normalization(self, feat_shift, feat_scale, target_shift, target_scale):
        import numpy as np
        a = [np.ascontiguousarray(v, dtype=np.float32) for v in (feat_shift, feat_scale, target_shift, target_scale)]
        fp = [x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) for x in a]
        _scheck(sload().rtw_surrogate_set_normalization(self.h, *fp))

    def get_params(self):
        import numpy as np
        out = np.empty(param_count(), dtype=np.float32)
        _scheck(sload().rtw_surrogate_get_params(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), out.size))
        return out

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        _scheck(sload().rtw_surrogate_set_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size))

    def save(self, path):
        """Write the trained network (parameters and normalisation) to a file."""
        _scheck(sload().rtw_surrogate_save(self.h, str(path).encode()))

    def load(self, path):
        """Read a network written by save()."""
        _scheck(sload().rtw_surrogate_load(self.h, str(path).encode()))

    def get_grads(self):
        import numpy as np
        out = np.empty(param_count(), dtype=np.float32)
        _scheck(sload().rtw_surrogate_get_grads(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), out.size))
        return out

    def forward(self, feats, stream=None, layered=False):
        """feats: device float32 [n, 9] -> device [n, 4] (ln I_x, ln I_y, ln sigma_x, ln sigma_y).
        layered: through the per-layer products of training (rtw_surrogate_forward_layered)."""
        import torch
        n = feats.shape[0]
        out = torch.empty((n, 4), dtype=torch.float32, device=feats.device)
        fn = sload().rtw_surrogate_forward_layered if layered else sload().rtw_surrogate_forward
        for a in range(0, n, self.max_rows):
            b = min(n, a + self.max_rows)
            _scheck(fn(self.h, b - a, _ptr(feats[a:b]), _ptr(out[a:b]), _stream_ptr(stream)))
        return out

    def grad(self, feats, targets, stream=None):
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        _scheck(sload().rtw_surrogate_grad(self.h, feats.shape[0], _ptr(feats), _ptr(targets), _ptr(loss),
                                           _stream_ptr(stream)))
        return loss

    def train_step(self, feats, targets, lr, stream=None):
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        _scheck(sload().rtw_surrogate_train_step(self.h, feats.shape[0], _ptr(feats), _ptr(targets), float(lr),
                                                 _ptr(loss), _stream_ptr(stream)))
        return loss

    def query(self, feats, q_part, q_cell, tau, batch, cells, tune=None, stream=None):
        """Answers with RTW fallback; batch: a Batch describing the queries'
        particles (its workspace and output are not used).  Returns (answer
        [n, 2], pred [n, 4], used_fallback [n], particles re-computed)."""
        import torch
        n = feats.shape[0]
        dev = feats.device
        pred = torch.empty((n, 4), dtype=torch.float32, device=dev)
        ans = torch.empty((n, 2), dtype=torch.float32, device=dev)
        used = torch.empty(n, dtype=torch.int32, device=dev)
        nb = ctypes.c_size_t(0)
        L = sload()
        _scheck(L.rtw_surrogate_query_scratch_size(batch.n, batch.parts, batch.gn, ctypes.byref(batch.inc),
                                                   ctypes.byref(batch.opts), ctypes.byref(batch.grid),
                                                   ctypes.byref(cells), ctypes.byref(nb)))
        if getattr(self, "_scratch", None) is None or self._scratch.numel() < nb.value:
            self._scratch = None
            torch.cuda.empty_cache()
            self._scratch = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        nrec = ctypes.c_int(0)
        _scheck(L.rtw_surrogate_query(self.h, n, _ptr(feats), _ptr(q_part), _ptr(q_cell), float(tau), batch.n,
                                      batch.parts, batch.gn, ctypes.byref(batch.inc), ctypes.byref(batch.opts),
                                      ctypes.byref(batch.grid), ctypes.byref(cells),
                                      ctypes.byref(tune) if tune is not None else None, _ptr(pred), _ptr(ans),
                                      _ptr(used), _ptr(self._scratch), ctypes.c_size_t(self._scratch.numel()),
                                      ctypes.byref(nrec), _stream_ptr(stream)))
        return ans, pred, used, nrec.value
