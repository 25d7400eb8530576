// rtw_lib.hip -- librtw.so: the C ABI of include/rtw.h over the gfx950 kernels.
//
// rtw_farfield runs, on the caller's stream:
//   k_setup       node tables (sin/cos of the node angles) and pool reset
//   k_trace<G>    one thread per incident ray: Eqs. 3-10, emission records (SoA)
//   k_raster<G>   one thread per (order, grid quad): triangle -> node hits
//   k_node_sum<G> one thread per node: ordered sum of its hits -> far field
// G = double (RTW_FP64) or float (RTW_MIXED, with FP64 path/phase/Jacobian).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rtw.h"
#include "rtw_device.hpp"
#include "rtw_raster.hpp"

using namespace rtw;

namespace {

thread_local std::string g_err;

// Optional per-kernel timing: HIP events recorded on the caller's stream around
// every launch while enabled (rtw_profile_enable), read by rtw_profile_read.
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
bool g_prof_on = false;

struct ProfScope {
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(const char* n, hipStream_t s) : name(n), st(s) {
    if (!g_prof_on) return;
    hipEventCreate(&a);
    hipEventCreate(&b);
    hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a) return;
    hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back({name, a, b});
  }
};

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

constexpr double PI_H = 3.14159265358979323846;
constexpr unsigned WS_MAGIC = 0x52545746u;  // "RTWF"

// Header at the start of a far-field workspace (written by k_setup).
struct WsHeader {
  unsigned magic;
  int cap_part;
  int n_part;
  int pad;
  unsigned long long bytes_per_hit;
  unsigned long long fixed_bytes;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int check_particle(const rtw_particle* p, const rtw_incident* inc, const rtw_trace_opts* o) {
  if (!p || !inc || !o) return fail(RTW_ERR_INVALID_ARG, "NULL argument struct");
  for (int i = 0; i < 3; ++i)
    if (!(p->semi_axes[i] > 0.0) || !std::isfinite(p->semi_axes[i]))
      return fail(RTW_ERR_INVALID_ARG, "semi-axis %d must be positive and finite", i);
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(p->euler_deg[i])) return fail(RTW_ERR_INVALID_ARG, "Euler angle %d is not finite", i);
  if (!(p->m > 0.0) || !std::isfinite(p->m)) return fail(RTW_ERR_INVALID_ARG, "refractive index must be positive");
  if (p->m == 1.0) return fail(RTW_ERR_UNSUPPORTED, "m = 1: no interface");
  if (!(inc->wavelength > 0.0) || !std::isfinite(inc->wavelength))
    return fail(RTW_ERR_INVALID_ARG, "wavelength must be positive");
  if (inc->n_pol != 1 && inc->n_pol != 2) return fail(RTW_ERR_INVALID_ARG, "n_pol must be 1 or 2");
  if (o->p_min < 0 || o->p_max < o->p_min) return fail(RTW_ERR_INVALID_ARG, "need 0 <= p_min <= p_max");
  if (o->p_max > RTW_MAX_ORDER) return fail(RTW_ERR_UNSUPPORTED, "p_max > %d", RTW_MAX_ORDER);
  if (o->grid_n < 2 || o->grid_n > 16384) return fail(RTW_ERR_INVALID_ARG, "grid_n must be in [2, 16384]");
  if (o->precision != RTW_FP64 && o->precision != RTW_MIXED)
    return fail(RTW_ERR_INVALID_ARG, "precision must be RTW_FP64 or RTW_MIXED");
  return RTW_OK;
}

// Body -> lab rotation R = Rz(alpha) Ry(beta) Rz(gamma), row-major.
void rotation_zyz(const double* deg, double* R) {
  double a = deg[0] * PI_H / 180.0, b = deg[1] * PI_H / 180.0, g = deg[2] * PI_H / 180.0;
  double ca = cos(a), sa = sin(a), cb = cos(b), sb = sin(b), cg = cos(g), sg = sin(g);
  R[0] = ca * cb * cg - sa * sg; R[1] = -ca * cb * sg - sa * cg; R[2] = ca * sb;
  R[3] = sa * cb * cg + ca * sg; R[4] = -sa * cb * sg + ca * cg; R[5] = sa * sb;
  R[6] = -sb * cg;               R[7] = sb * sg;                 R[8] = cb;
}

ParticleConst make_const(const rtw_particle* p, const rtw_incident* inc, const rtw_trace_opts* o) {
  ParticleConst P;
  for (int i = 0; i < 3; ++i) P.A[i] = 1.0 / (p->semi_axes[i] * p->semi_axes[i]);
  rotation_zyz(p->euler_deg, P.R);
  double sxx = 0, syy = 0;
  for (int k = 0; k < 3; ++k) {
    double s2 = p->semi_axes[k] * p->semi_axes[k];
    sxx += P.R[k] * P.R[k] * s2;
    syy += P.R[3 + k] * P.R[3 + k] * s2;
  }
  P.L = std::max(std::sqrt(sxx), std::sqrt(syy));
  P.N = o->grid_n;
  P.h = 2.0 * P.L / P.N;
  P.k = 2.0 * PI_H / inc->wavelength;
  P.m = p->m;
  P.p_min = o->p_min;
  P.p_max = o->p_max;
  P.n_pol = inc->n_pol;
  P.amplif_limit = 32.0;
  return P;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <typename G>
__global__ void __launch_bounds__(256) k_trace(const ParticleConst P, const Records<G> rec) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= rec.NN) return;
  const int n_ord = P.p_max - P.p_min + 1;
  for (int o = 0; o < n_ord; ++o) rec.flags[o * rec.NN + id] = 0;
  RecordSink<G> sink{rec, id, P.k, P.amplif_limit, false};
  const int iy = (int)(id / P.N), ix = (int)(id - (long)iy * P.N);
  trace_ray<G>(P, ix, iy, sink);
  if (sizeof(G) == 4) {
    // Rays whose divergence factor is ill-conditioned in FP32 are listed for the
    // FP64 pass (one append per wave).
    const bool redo = sink.need64;
    const unsigned long long mask = __ballot(redo);
    if (mask) {
      const int lane = threadIdx.x & 63, leader = __ffsll((long long)mask) - 1;
      unsigned base = 0;
      if (lane == leader) base = atomicAdd(rec.n_fp64, (unsigned)__popcll(mask));
      base = __shfl(base, leader);
      if (redo) rec.redo_list[base + __popcll(mask & ((1ull << lane) - 1ull))] = (int)id;
    }
  }
}

// FP64 re-trace of the listed rays, writing into the FP32 records.  A fixed
// grid strides over the list, whose length is only known on the device.
__global__ void __launch_bounds__(256) k_retrace64(const ParticleConst P, const Records<float> rec) {
  const unsigned n = *rec.n_fp64;
  const int n_ord = P.p_max - P.p_min + 1;
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const long id = rec.redo_list[i];
    for (int o = 0; o < n_ord; ++o) rec.flags[o * rec.NN + id] = 0;
    RecordSink<float> sink{rec, id, P.k, 0.0, false};
    const int iy = (int)(id / P.N), ix = (int)(id - (long)iy * P.N);
    trace_ray<double>(P, ix, iy, sink);
  }
}

// Sink of rtw_trace: FP64 diagnostic records.
template <typename G>
struct DiagSink {
  rtw_ray_records out;
  long id, NN;
  int n_pol;
  double amplif_limit;
  bool need64;
  template <typename E>
  __device__ void emit(const Emission<E>& e) {
    if (sizeof(E) == 4 && e.amplif > amplif_limit) need64 = true;
    const long o = e.slot;
    if (out.flags) out.flags[o * NN + id] = 1 | (e.nf << 1) | (e.det_neg << 8);
    if (out.dir) {
      out.dir[(o * 3 + 0) * NN + id] = (double)e.dir.x;
      out.dir[(o * 3 + 1) * NN + id] = (double)e.dir.y;
      out.dir[(o * 3 + 2) * NN + id] = (double)e.dir.z;
    }
    if (out.rexit) {
      out.rexit[(o * 3 + 0) * NN + id] = e.rexit.x;
      out.rexit[(o * 3 + 1) * NN + id] = e.rexit.y;
      out.rexit[(o * 3 + 2) * NN + id] = e.rexit.z;
    }
    if (out.phase) out.phase[o * NN + id] = e.phase;
    if (out.amp) out.amp[o * NN + id] = e.amp;
    if (out.cond) {
      out.cond[(o * 2 + 0) * NN + id] = e.amplif;
      out.cond[(o * 2 + 1) * NN + id] = e.drift;
    }
    if (out.field)
      for (int p = 0; p < n_pol; ++p)
        for (int x = 0; x < 3; ++x) {
          out.field[(((o * n_pol + p) * 3 + x) * 2 + 0) * NN + id] = (double)e.f[p][x].re;
          out.field[(((o * n_pol + p) * 3 + x) * 2 + 1) * NN + id] = (double)e.f[p][x].im;
        }
  }
};

template <typename G>
__global__ void __launch_bounds__(256) k_trace_diag(const ParticleConst P, const rtw_ray_records out) {
  const long NN = (long)P.N * P.N;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= NN) return;
  const int n_ord = P.p_max - P.p_min + 1;
  for (long o = 0; o < n_ord; ++o) {
    if (out.flags) out.flags[o * NN + id] = 0;
    if (out.phase) out.phase[o * NN + id] = 0.0;
    if (out.amp) out.amp[o * NN + id] = 0.0;
    if (out.cond) out.cond[(o * 2 + 0) * NN + id] = out.cond[(o * 2 + 1) * NN + id] = 0.0;
    for (int x = 0; x < 3; ++x) {
      if (out.dir) out.dir[(o * 3 + x) * NN + id] = 0.0;
      if (out.rexit) out.rexit[(o * 3 + x) * NN + id] = 0.0;
    }
    if (out.field)
      for (int j = 0; j < P.n_pol * 6; ++j) out.field[(o * P.n_pol * 6 + j) * NN + id] = 0.0;
  }
  DiagSink<G> sink{out, id, NN, P.n_pol, P.amplif_limit, false};
  const int iy = (int)(id / P.N), ix = (int)(id - (long)iy * P.N);
  trace_ray<G>(P, ix, iy, sink);
  if (sizeof(G) == 4 && sink.need64) {
    for (long o = 0; o < n_ord; ++o)
      if (out.flags) out.flags[o * NN + id] = 0;
    trace_ray<double>(P, ix, iy, sink);
  }
}

// Node tables from the degree lists, reset of the hit pool, workspace header.
__global__ void k_setup(int n_theta, const double* theta_deg, int n_phi, const double* phi_deg, double* th,
                        double* ph, double* sth, double* cth, double* sph, double* cph, int* head, int n_nodes,
                        unsigned* counter, WsHeader* hdr, WsHeader hv) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const double D2R = 3.14159265358979323846 / 180.0;
  if (i < n_theta) {
    double t = theta_deg[i] * D2R;
    th[i] = t;
    sth[i] = sin(t);
    cth[i] = cos(t);
  }
  if (i < n_phi) {
    double p = phi_deg[i] * D2R;
    ph[i] = p;
    sph[i] = sin(p);
    cph[i] = cos(p);
  }
  if (i < n_nodes) head[i] = -1;
  if (i <= NPART + 1) counter[i] = 0u;
  if (i == 0) *hdr = hv;
}

constexpr int ROWS_CAP = 1 << 24;  // (triangle, row) items of large triangles

// Split each node-angle list into uniformly spaced runs (block 0: theta,
// block 1: phi).  A "break" is an index where the spacing changes; more than
// MAXSEG - 1 breaks leaves the list to binary search, and so does a run whose
// nodes deviate from its arithmetic model by more than 1e-10 of its step
// (the lookups allow 1e-9).
__global__ void __launch_bounds__(256) k_axis_segments(const double* th, int n_t, const double* ph, int n_p,
                                                       AxisSeg* seg_t, AxisSeg* seg_p) {
  const double* v = blockIdx.x == 0 ? th : ph;
  const int n = blockIdx.x == 0 ? n_t : n_p;
  AxisSeg* out = blockIdx.x == 0 ? seg_t : seg_p;
  __shared__ int nbreak, bad;
  __shared__ int brk[MAXSEG];
  __shared__ AxisSeg sg;
  if (threadIdx.x == 0) { nbreak = 0; bad = 0; }
  __syncthreads();
  for (int i = 1 + (int)threadIdx.x; i < n - 1; i += blockDim.x) {
    const double d0 = v[i] - v[i - 1], d1 = v[i + 1] - v[i];
    if (fabs(d1 - d0) > 1e-7 * fmax(fabs(d0), fabs(d1))) {
      const int k = atomicAdd(&nbreak, 1);
      if (k < MAXSEG) brk[k] = i;
    }
  }
  __syncthreads();
  const int nb = nbreak;
  if (n < 2 || nb > MAXSEG - 1) {
    if (threadIdx.x == 0) out->nseg = 0;
    return;
  }
  if (threadIdx.x == 0) {
    for (int a = 1; a < nb; ++a) {  // sort the few break indices
      int x = brk[a], b = a;
      while (b > 0 && brk[b - 1] > x) { brk[b] = brk[b - 1]; --b; }
      brk[b] = x;
    }
    int lo = 0;
    for (int k = 0; k <= nb; ++k) {
      const int hi = k < nb ? brk[k] : n - 1;
      sg.start[k] = lo;
      sg.end[k] = hi;
      sg.v0[k] = v[lo];
      sg.vend[k] = v[hi];
      sg.step[k] = (v[hi] - v[lo]) / (double)(hi - lo);
      sg.inv_step[k] = 1.0 / sg.step[k];
      lo = hi;
    }
    sg.nseg = nb + 1;
  }
  __syncthreads();
  for (int k = 0; k < sg.nseg; ++k)
    for (int i = sg.start[k] + (int)threadIdx.x; i <= sg.end[k]; i += blockDim.x) {
      const double model = sg.v0[k] + (double)(i - sg.start[k]) * sg.step[k];
      if (!(fabs(v[i] - model) <= 1e-10 * sg.step[k])) bad = 1;
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (bad) sg.nseg = 0;
    *out = sg;
  }
}

// Workspace layout of rtw_farfield.
struct Layout {
  size_t hdr, counter, th, ph, sth, cth, sph, cph, seg, flags, rr, ang, head, redo, rows, link, contrib, total;
  size_t fixed;          // everything except the hit pool
  size_t bytes_per_hit;  // link + contrib
};

Layout layout(const ParticleConst& P, int precision, int n_theta, int n_phi, long cap_total) {
  Layout L;
  const size_t gs = precision == RTW_FP64 ? 8 : 4;
  const long NN = (long)P.N * P.N;
  const int n_ord = P.p_max - P.p_min + 1;
  const long n_nodes = (long)n_theta * n_phi;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
  L.hdr = take(sizeof(WsHeader));
  L.counter = take(sizeof(unsigned) * (NPART + 2));  // hit-pool partitions, FP64 re-trace count, row-list count
  L.th = take(8 * n_theta); L.ph = take(8 * n_phi);
  L.sth = take(8 * n_theta); L.cth = take(8 * n_theta);
  L.sph = take(8 * n_phi); L.cph = take(8 * n_phi);
  L.seg = take(2 * sizeof(AxisSeg));
  L.flags = take(4 * (size_t)n_ord * NN);
  L.rr = take((precision == RTW_FP64 ? sizeof(RayRec<double>) : sizeof(RayRec<float>)) * (size_t)n_ord * NN);
  L.ang = take(sizeof(float2) * (size_t)n_ord * NN);
  L.head = take(4 * (size_t)n_nodes);
  L.redo = take(precision == RTW_FP64 ? 4 : 4 * (size_t)NN);
  L.rows = take(sizeof(int2) * (size_t)ROWS_CAP);
  L.fixed = off;
  L.bytes_per_hit = sizeof(int2) + gs * 4 * P.n_pol;
  L.link = take(sizeof(int2) * (size_t)cap_total);
  L.contrib = take(gs * 4 * P.n_pol * (size_t)cap_total);
  L.total = off;
  return L;
}

long cap_from_bytes(const Layout& base, size_t bytes) {
  // largest per-partition capacity whose pool fits in `bytes`
  if (bytes < base.fixed + 2 * 256) return 0;
  size_t avail = bytes - base.fixed - 2 * 256;
  long per = (long)(avail / (base.bytes_per_hit * NPART));
  return per;
}

// Triangle keys (order slot, quad, half) are 32-bit: 2 n_ord (N-1)^2 < 2^31.
int check_keys(const rtw_trace_opts* o) {
  const long nq = (long)(o->grid_n - 1) * (o->grid_n - 1);
  if (2L * (o->p_max - o->p_min + 1) * nq >= (1L << 31))
    return fail(RTW_ERR_UNSUPPORTED, "far field needs 2 (p_max - p_min + 1) (grid_n - 1)^2 < 2^31");
  return RTW_OK;
}

int check_grid(const rtw_grid* g) {
  if (!g) return fail(RTW_ERR_INVALID_ARG, "NULL grid");
  if (g->n_theta < 1 || g->n_phi < 1 || !g->theta_deg || !g->phi_deg)
    return fail(RTW_ERR_INVALID_ARG, "empty node grid");
  if ((long)g->n_theta * g->n_phi > (1L << 30)) return fail(RTW_ERR_INVALID_ARG, "node grid too large");
  return RTW_OK;
}

template <typename G>
int launch_farfield(const ParticleConst& P, int precision, const rtw_grid* grid, void* out, int32_t* ncontrib,
                    char* ws, size_t ws_bytes, hipStream_t st) {
  const long NN = (long)P.N * P.N;
  const int n_ord = P.p_max - P.p_min + 1;
  const int n_nodes = grid->n_theta * grid->n_phi;
  Layout base = layout(P, precision, grid->n_theta, grid->n_phi, 0);
  long cap_part = cap_from_bytes(base, ws_bytes);
  if (cap_part < 1) return fail(RTW_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu-byte minimum",
                                ws_bytes, base.fixed + base.bytes_per_hit * NPART + 512);
  if (cap_part > (1L << 30) / NPART) cap_part = (1L << 30) / NPART;
  Layout L = layout(P, precision, grid->n_theta, grid->n_phi, cap_part * NPART);
  if (L.total > ws_bytes) return fail(RTW_ERR_WORKSPACE, "internal layout exceeds workspace");

  WsHeader hv;
  hv.magic = WS_MAGIC;
  hv.cap_part = (int)cap_part;
  hv.n_part = NPART;
  hv.pad = 0;
  hv.bytes_per_hit = L.bytes_per_hit;
  hv.fixed_bytes = L.fixed + 512;

  NodeGrid ng;
  ng.n_theta = grid->n_theta; ng.n_phi = grid->n_phi;
  ng.th = (double*)(ws + L.th); ng.ph = (double*)(ws + L.ph);
  ng.sth = (double*)(ws + L.sth); ng.cth = (double*)(ws + L.cth);
  ng.sph = (double*)(ws + L.sph); ng.cph = (double*)(ws + L.cph);
  ng.seg_t = (const AxisSeg*)(ws + L.seg);
  ng.seg_p = (const AxisSeg*)(ws + L.seg) + 1;
  Records<G> rec;
  rec.flags = (int32_t*)(ws + L.flags);
  rec.rr = (RayRec<G>*)(ws + L.rr);
  rec.ang = (float2*)(ws + L.ang);
  rec.NN = NN;
  rec.n_pol = P.n_pol;
  rec.n_fp64 = (unsigned*)(ws + L.counter) + NPART;
  rec.redo_list = (int*)(ws + L.redo);
  HitPool<G> pool;
  pool.head = (int*)(ws + L.head);
  pool.link = (int2*)(ws + L.link);
  pool.contrib = (G*)(ws + L.contrib);
  pool.counter = (unsigned*)(ws + L.counter);
  pool.cap_part = (int)cap_part;
  pool.rows = (int2*)(ws + L.rows);
  pool.n_rows = (unsigned*)(ws + L.counter) + NPART + 1;
  pool.rows_cap = ROWS_CAP;

  long setup_n = std::max<long>({(long)n_nodes, (long)grid->n_theta, (long)grid->n_phi, (long)NPART + 2});
  { ProfScope ps("k_setup", st);
  hipLaunchKernelGGL(k_setup, dim3((unsigned)((setup_n + 255) / 256)), dim3(256), 0, st, grid->n_theta,
                     grid->theta_deg, grid->n_phi, grid->phi_deg, (double*)ng.th, (double*)ng.ph, (double*)ng.sth,
                     (double*)ng.cth, (double*)ng.sph, (double*)ng.cph, pool.head, n_nodes, pool.counter,
                     (WsHeader*)(ws + L.hdr), hv);
  hipLaunchKernelGGL(k_axis_segments, dim3(2), dim3(256), 0, st, ng.th, ng.n_theta, ng.ph, ng.n_phi,
                     (AxisSeg*)(ws + L.seg), (AxisSeg*)(ws + L.seg) + 1); }
  { ProfScope ps(precision == RTW_FP64 ? "k_trace_fp64" : "k_trace_mixed", st);
  hipLaunchKernelGGL(k_trace<G>, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, st, P, rec); }
  if (precision == RTW_MIXED) {
    ProfScope ps("k_retrace64", st);
    hipLaunchKernelGGL(k_retrace64, dim3((unsigned)std::min<long>(2048, (NN + 255) / 256)), dim3(256), 0, st, P,
                       *reinterpret_cast<Records<float>*>(&rec));
  }
  const long nquad = (long)(P.N - 1) * (P.N - 1);
  { ProfScope ps(precision == RTW_FP64 ? "k_raster_fp64" : "k_raster_mixed", st);
  hipLaunchKernelGGL(k_raster<G>, dim3((unsigned)((nquad + 255) / 256), n_ord), dim3(256), 0, st, P, rec, ng, pool,
                     BOX_MARGIN); }
  { ProfScope ps(precision == RTW_FP64 ? "k_raster_rows_fp64" : "k_raster_rows_mixed", st);
  hipLaunchKernelGGL(k_raster_rows<G>, dim3(1024), dim3(256), 0, st, P, rec, ng, pool, BOX_MARGIN); }
  { ProfScope ps(precision == RTW_FP64 ? "k_node_sum_fp64" : "k_node_sum_mixed", st);
  hipLaunchKernelGGL(k_node_sum<G>, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, st, pool, n_nodes,
                     P.n_pol, (G*)out, ncontrib); }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return RTW_OK;
}

}  // namespace

extern "C" {

const char* rtw_last_error(void) { return g_err.c_str(); }

int rtw_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return RTW_OK;
}

int rtw_profile_read(int max_kernels, char* names, double* total_ms, int* launches, int* n_kernels) {
  if (max_kernels < 0 || !n_kernels) return fail(RTW_ERR_INVALID_ARG, "bad profile buffers");
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs.swap(g_prof);
  }
  std::vector<std::string> nm;
  std::vector<double> ms;
  std::vector<int> cnt;
  int rc = RTW_OK;
  for (auto& r : recs) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) rc = fail(RTW_ERR_DEVICE, "event read failed: %s", hipGetErrorString(e));
    size_t i = 0;
    while (i < nm.size() && nm[i] != r.name) ++i;
    if (i == nm.size()) { nm.push_back(r.name); ms.push_back(0.0); cnt.push_back(0); }
    ms[i] += t;
    cnt[i] += 1;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  *n_kernels = (int)nm.size();
  for (int i = 0; i < (int)nm.size() && i < max_kernels; ++i) {
    if (names) { std::strncpy(names + 64 * i, nm[i].c_str(), 63); names[64 * i + 63] = 0; }
    if (total_ms) total_ms[i] = ms[i];
    if (launches) launches[i] = cnt[i];
  }
  return rc;
}

const char* rtw_version(void) { return "rtw-mi355x 0.1 (gfx950)"; }

int rtw_trace(const rtw_particle* part, const rtw_incident* inc, const rtw_trace_opts* opts,
              const rtw_ray_records* out, void* hip_stream) {
  int rc = check_particle(part, inc, opts);
  if (rc) return rc;
  if (!out) return fail(RTW_ERR_INVALID_ARG, "NULL output records");
  ParticleConst P = make_const(part, inc, opts);
  const long NN = (long)P.N * P.N;
  hipStream_t st = (hipStream_t)hip_stream;
  if (opts->precision == RTW_FP64)
    hipLaunchKernelGGL(k_trace_diag<double>, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, st, P, *out);
  else
    hipLaunchKernelGGL(k_trace_diag<float>, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, st, P, *out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return RTW_OK;
}

int rtw_farfield_workspace_size(const rtw_particle* part, const rtw_incident* inc, const rtw_trace_opts* opts,
                                const rtw_grid* grid, double hits_per_node, size_t* bytes) {
  int rc = check_particle(part, inc, opts);
  if (rc) return rc;
  if (!bytes) return fail(RTW_ERR_INVALID_ARG, "NULL bytes");
  if (!grid || grid->n_theta < 1 || grid->n_phi < 1) return fail(RTW_ERR_INVALID_ARG, "empty node grid");
  rc = check_keys(opts);
  if (rc) return rc;
  if (!(hits_per_node > 0.0)) hits_per_node = 6.0;
  ParticleConst P = make_const(part, inc, opts);
  const long n_nodes = (long)grid->n_theta * grid->n_phi;
  long cap_part = (long)std::ceil(hits_per_node * (double)n_nodes / NPART) + 256;
  Layout L = layout(P, opts->precision, grid->n_theta, grid->n_phi, cap_part * NPART);
  *bytes = L.total + 512;
  return RTW_OK;
}

int rtw_farfield(const rtw_particle* part, const rtw_incident* inc, const rtw_trace_opts* opts,
                 const rtw_grid* grid, void* out_field, int32_t* ncontrib, void* workspace, size_t workspace_bytes,
                 void* hip_stream) {
  int rc = check_particle(part, inc, opts);
  if (rc) return rc;
  rc = check_grid(grid);
  if (rc) return rc;
  rc = check_keys(opts);
  if (rc) return rc;
  if (!out_field || !workspace) return fail(RTW_ERR_INVALID_ARG, "NULL output or workspace");
  if (((uintptr_t)workspace & 255) != 0) return fail(RTW_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  ParticleConst P = make_const(part, inc, opts);
  hipStream_t st = (hipStream_t)hip_stream;
  if (opts->precision == RTW_FP64)
    return launch_farfield<double>(P, RTW_FP64, grid, out_field, ncontrib, (char*)workspace, workspace_bytes, st);
  return launch_farfield<float>(P, RTW_MIXED, grid, out_field, ncontrib, (char*)workspace, workspace_bytes, st);
}

int rtw_farfield_stats(const void* workspace, void* hip_stream, uint64_t* hits, uint64_t* fp64_rays) {
  if (!workspace) return fail(RTW_ERR_INVALID_ARG, "NULL workspace");
  hipStream_t st = (hipStream_t)hip_stream;
  WsHeader h;
  unsigned cnt[NPART + 2];
  hipError_t e = hipMemcpyAsync(&h, workspace, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cnt, (const char*)workspace + align256(sizeof(WsHeader)), sizeof(cnt), hipMemcpyDeviceToHost,
                       st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "stats read failed: %s", hipGetErrorString(e));
  if (h.magic != WS_MAGIC) return fail(RTW_ERR_INVALID_ARG, "workspace was not used by rtw_farfield");
  uint64_t tot = 0;
  for (int i = 0; i < NPART; ++i) tot += cnt[i];
  if (hits) *hits = tot;
  if (fp64_rays) *fp64_rays = cnt[NPART];
  return RTW_OK;
}

int rtw_farfield_status(const void* workspace, void* hip_stream, size_t* bytes_needed) {
  if (!workspace) return fail(RTW_ERR_INVALID_ARG, "NULL workspace");
  hipStream_t st = (hipStream_t)hip_stream;
  WsHeader h;
  unsigned cnt[NPART];
  hipError_t e = hipMemcpyAsync(&h, workspace, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "status read failed: %s", hipGetErrorString(e));
  if (h.magic != WS_MAGIC) return fail(RTW_ERR_INVALID_ARG, "workspace was not used by rtw_farfield");
  // the counters follow the header at the next 256-byte boundary
  e = hipMemcpyAsync(cnt, (const char*)workspace + align256(sizeof(WsHeader)), sizeof(cnt), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "status read failed: %s", hipGetErrorString(e));
  unsigned mx = 0;
  for (int i = 0; i < NPART; ++i) mx = std::max(mx, cnt[i]);
  if (bytes_needed) {
    size_t per = (size_t)mx + (mx >> 2) + 64;
    *bytes_needed = (size_t)h.fixed_bytes + per * NPART * h.bytes_per_hit + 1024;
  }
  if ((long)mx > h.cap_part)
    return fail(RTW_ERR_WORKSPACE, "hit pool overflow: %u hits in the fullest partition, capacity %d", mx, h.cap_part);
  return RTW_OK;
}

}  // extern "C"
