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
    _fields_ = [("semi_axes", ctypes.c_double * 3), ("euler_deg", ctypes.c_double * 3), ("m", ctypes.c_double)]


class Incident(ctypes.Structure):
    _fields_ = [("wavelength", ctypes.c_double), ("n_pol", ctypes.c_int)]


class TraceOpts(ctypes.Structure):
    _fields_ = [("p_min", ctypes.c_int), ("p_max", ctypes.c_int), ("grid_n", ctypes.c_int),
                ("precision", ctypes.c_int)]


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
    _fields_ = [("rays_per_chunk", ctypes.c_longlong), ("hits_per_node", ctypes.c_double)]


EXPORTED = ["rtw_trace", "rtw_farfield_workspace_size", "rtw_farfield", "rtw_farfield_status",
            "rtw_farfield_stats", "rtw_batch_workspace_size", "rtw_batch", "rtw_batch_autotune",
            "rtw_profile_enable", "rtw_profile_read", "rtw_last_error", "rtw_version"]

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
    L.rtw_farfield_status.argtypes = [ctypes.c_void_p, ctypes.c_void_p, P(ctypes.c_size_t)]
    L.rtw_batch_workspace_size.argtypes = [ctypes.c_int, P(Particle), P(ctypes.c_int), P(Incident), P(TraceOpts),
                                           P(Grid), P(BatchOpts), P(ctypes.c_size_t)]
    L.rtw_batch.argtypes = [ctypes.c_int, P(Particle), P(ctypes.c_int), P(Incident), P(TraceOpts), P(Grid),
                            ctypes.c_void_p, ctypes.c_void_p, P(Tune), P(BatchOpts), ctypes.c_void_p, ctypes.c_size_t,
                            ctypes.c_void_p]
    L.rtw_batch_autotune.argtypes = [ctypes.c_int, P(Particle), P(ctypes.c_int), P(Incident), P(TraceOpts),
                                     P(Grid), P(BatchOpts), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p, P(Tune)]
    L.rtw_farfield_stats.argtypes = [ctypes.c_void_p, ctypes.c_void_p, P(ctypes.c_uint64), P(ctypes.c_uint64)]
    L.rtw_profile_enable.argtypes = [ctypes.c_int]
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


def make_particle(semi_axes: Sequence[float], euler_deg: Sequence[float] = (0, 0, 0), m: float = 1.333):
    p = Particle()
    p.semi_axes[:] = [float(v) for v in semi_axes]
    p.euler_deg[:] = [float(v) for v in euler_deg]
    p.m = float(m)
    return p


def make_incident(wavelength: float = 0.6328, n_pol: int = 1):
    inc = Incident()
    inc.wavelength = float(wavelength)
    inc.n_pol = int(n_pol)
    return inc


def make_opts(p_min=0, p_max=2, grid_n=64, precision=FP64):
    o = TraceOpts()
    o.p_min, o.p_max, o.grid_n, o.precision = int(p_min), int(p_max), int(grid_n), int(precision)
    return o


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def trace(part, inc, opts, device="cuda", stream=None):
    """Per-ray records of every emitted order (rtw_trace); FP64 tensors on the device."""
    import torch
    N = opts.grid_n
    n_ord = opts.p_max - opts.p_min + 1
    NN = N * N
    out = dict(flags=torch.empty((n_ord, NN), dtype=torch.int32, device=device),
               dir=torch.empty((n_ord, 3, NN), dtype=torch.float64, device=device),
               rexit=torch.empty((n_ord, 3, NN), dtype=torch.float64, device=device),
               phase=torch.empty((n_ord, NN), dtype=torch.float64, device=device),
               amp=torch.empty((n_ord, NN), dtype=torch.float64, device=device),
               field=torch.empty((n_ord, inc.n_pol, 3, 2, NN), dtype=torch.float64, device=device),
               cond=torch.empty((n_ord, 2, NN), dtype=torch.float64, device=device))
    rec = RayRecords(*[_ptr(out[k]) for k in ("flags", "dir", "rexit", "phase", "amp", "field", "cond")])
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

    def __post_init__(self):
        import torch
        n = len(self.particles)
        self.n = n
        self.parts = (Particle * n)(*[make_particle(a, e, m) for (a, e, m) in self.particles])
        self.gn = (ctypes.c_int * n)(*[int(g) for g in self.grid_n])
        self.bopts = BatchOpts(int(self.rays_per_chunk), float(self.hits_per_node))
        self.theta = torch.as_tensor(self.theta_deg, dtype=torch.float64, device=self.device).contiguous()
        self.phi = torch.as_tensor(self.phi_deg, dtype=torch.float64, device=self.device).contiguous()
        self.grid = Grid(self.theta.numel(), self.theta.data_ptr(), self.phi.numel(), self.phi.data_ptr())
        nb = ctypes.c_size_t(0)
        _check(load().rtw_batch_workspace_size(n, self.parts, self.gn, ctypes.byref(self.inc), ctypes.byref(self.opts),
                                               ctypes.byref(self.grid), ctypes.byref(self.bopts), ctypes.byref(nb)))
        self._alloc(nb.value)
        dt = torch.float64 if self.opts.precision == FP64 else torch.float32
        self.out = torch.empty((n, self.inc.n_pol, 2, self.theta.numel(), self.phi.numel(), 2), dtype=dt,
                               device=self.device)
        self.ncontrib = torch.empty((n, self.theta.numel(), self.phi.numel()), dtype=torch.int32, device=self.device)

    def _alloc(self, nbytes):
        import torch
        self.ws_bytes = int(nbytes)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) & ~255

    def launch(self, stream=None, with_counts=True):
        _check(load().rtw_batch(self.n, self.parts, self.gn, ctypes.byref(self.inc), ctypes.byref(self.opts),
                                ctypes.byref(self.grid), _ptr(self.out), _ptr(self.ncontrib) if with_counts else None,
                                ctypes.byref(self.tune) if self.tune is not None else None, ctypes.byref(self.bopts),
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
