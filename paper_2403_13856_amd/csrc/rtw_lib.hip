// rtw_lib.hip -- librtw.so: the C ABI of include/rtw.h over the gfx950 kernels.
//
// rtw_farfield runs, on the caller's stream:
//   k_setup         node tables (sin/cos of the node angles), uniform runs of
//                   the angle lists, counter and first-chunk node-count reset
//   k_trace_tiles   persistent, one thread per incident ray: Eqs. 3-10, emission records
//   k_retrace64     (mixed) FP64 re-trace of the rays ill-conditioned in FP32
//   k_raster<G>     one thread per (order, grid quad): triangle -> node hits
//   k_scan          node counts -> node ranges; the chunk's hit totals
//   k_store_hits<G> one thread per hit: interpolated contribution, in node order
//   k_node_sum<G>   one thread per node: ordered sum of its hits -> far field
// G = double (RTW_FP64) or float (RTW_MIXED, with FP64 path/phase/Jacobian).
// rtw_batch with rtw_batch_opts.fused replaces trace to hit store by k_fused
// (rtw_fused.hpp), then k_scan, k_scatter and k_node_sum.
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
#include "rtw_fused.hpp"

using namespace rtw;

// Workspace of rtw_farfield_static: library-owned device memory, one copy per
// GPU (each at its own address), held until the process ends.  Host code
// never passes this name to a kernel: it is a host-side stand-in there.  The
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t STATIC_WS_BYTES = (size_t)RTW_STATIC_WORKSPACE_MIB << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

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
std::string g_prof_only;  // record only the kernels of this name (empty: every kernel)
thread_local bool g_prof_off = false;  // set while a call must not create events

struct ProfScope {
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(const char* n, hipStream_t s) : name(n), st(s) {
    if (!g_prof_on || g_prof_off) return;
    {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      if (!g_prof_only.empty() && g_prof_only != name) return;
    }
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
  if (!(p->m_im >= 0.0) || !std::isfinite(p->m_im))
    return fail(RTW_ERR_INVALID_ARG, "imaginary part of the index must be finite and >= 0");
  if (p->m == 1.0) return fail(RTW_ERR_UNSUPPORTED, "m = 1: no interface");
  if (!(inc->wavelength > 0.0) || !std::isfinite(inc->wavelength))
    return fail(RTW_ERR_INVALID_ARG, "wavelength must be positive");
  if (inc->n_pol != 1 && inc->n_pol != 2) return fail(RTW_ERR_INVALID_ARG, "n_pol must be 1 or 2");
  const double amax = std::max(p->semi_axes[0], std::max(p->semi_axes[1], p->semi_axes[2]));
  if (!(inc->source_distance == 0.0 || (inc->source_distance > amax && std::isfinite(inc->source_distance))))
    return fail(RTW_ERR_INVALID_ARG, "source_distance must be 0 (plane wave) or beyond the largest semi-axis");
  if (!(inc->observation_radius == 0.0 ||
        (inc->observation_radius > amax && std::isfinite(inc->observation_radius))))
    return fail(RTW_ERR_INVALID_ARG, "observation_radius must be 0 (far field) or beyond the largest semi-axis");
  if (o->p_min < 0 || o->p_max < o->p_min) return fail(RTW_ERR_INVALID_ARG, "need 0 <= p_min <= p_max");
  if (o->p_max > RTW_MAX_ORDER) return fail(RTW_ERR_UNSUPPORTED, "p_max > %d", RTW_MAX_ORDER);
  if (o->grid_n < 2 || o->grid_n > 16384) return fail(RTW_ERR_INVALID_ARG, "grid_n must be in [2, 16384]");
  if (o->precision != RTW_FP64 && o->precision != RTW_MIXED)
    return fail(RTW_ERR_INVALID_ARG, "precision must be RTW_FP64 or RTW_MIXED");
  if (o->corrections & ~(RTW_CAUSTIC | RTW_DIFFRACTION))
    return fail(RTW_ERR_INVALID_ARG, "corrections must be a combination of RTW_CAUSTIC and RTW_DIFFRACTION");
  if ((o->corrections & RTW_DIFFRACTION) && (inc->source_distance != 0.0 || inc->observation_radius != 0.0))
    return fail(RTW_ERR_UNSUPPORTED, "RTW_DIFFRACTION is the Fraunhofer term of a plane wave in the far field");
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
  P.zs = inc->source_distance;
  P.robs = inc->observation_radius;
  if (P.zs > 0.0) {
    // Point source S = (0, 0, -zs): the grid spans the particle's tangent cone
    // from S on the plane z = 0.  With D = X - S the cone is D^T K D = 0,
    // K = zs^2 (m m^T - m_z M) + M for the lab matrix M = R diag(1/a^2) R^T
    // and m = M e_z (the tangency condition (D^T M S)^2 = (D^T M D)(S^T M S - 1));
    // its extreme x (or y) on z = 0, where D = (x, y, zs), is the double-root
    // condition of the conic's quadratic in the other coordinate.
    const double zs = P.zs;
    double M[3][3], K[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += P.R[3 * i + k] * P.R[3 * j + k] * P.A[k];
        M[i][j] = acc;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) K[i][j] = zs * zs * (M[i][2] * M[j][2] - M[2][2] * M[i][j]) + M[i][j];
    double L = 0.0;
    for (int i = 0; i < 2; ++i) {
      const int j = 1 - i;
      const double a = K[i][j] * K[i][j] - K[j][j] * K[i][i];
      const double b = 2.0 * zs * (K[i][j] * K[j][2] - K[j][j] * K[i][2]);
      const double c = zs * zs * (K[j][2] * K[j][2] - K[j][j] * K[2][2]);
      const double sq = std::sqrt(b * b - 4.0 * a * c);
      L = std::max(L, std::max(std::fabs((-b + sq) / (2.0 * a)), std::fabs((-b - sq) / (2.0 * a))));
    }
    P.L = L;
  }
  P.N = o->grid_n;
  P.h = 2.0 * P.L / P.N;
  P.k = 2.0 * PI_H / inc->wavelength;
  P.m = p->m;
  P.m_im = p->m_im;
  P.p_min = o->p_min;
  P.p_max = o->p_max;
  P.n_pol = inc->n_pol;
  // FP64 re-trace above this amplification.  The wavefront curvature and the
  // divergence product are FP64 in both paths, so the amplified rounding is
  // FP64's: ~8 x amplif x 2^-53 relative in the divergence factor, and a
  // node's intensity error relative to its incoherent sum up to 2 n_b times
  // that for n_b contributions in phase; at 1e9 that stays below 1e-5.  (With
  // the curvature in FP32 the same bound, 8 x amplif x 2^-24, needed a limit
  // of 32, and 15% of the rays were re-traced.)
  P.amplif_limit = 1e9;
  return P;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Counters after the workspace header (unsigned): the NPART hit-pool partition
// fills, then per-chunk and per-call counters.
enum : int {
  C_REDO = NPART,  // rays listed for the FP64 re-trace in the current chunk
  C_ROWS,          // row-list items of the current chunk
  C_QUEUE,         // trace work items taken in the current chunk (plain particles)
  C_QUEUE_GEN,     // the same for the particles that need the general trace
  C_NEED,          // fullest hit-pool partition over the chunks of the call
  C_FP64_TOTAL,    // rays re-traced in FP64 over the call
  C_HITS,          // node hits over the call (64-bit, two slots: must be 8-byte aligned)
  C_HITS_HI,
  C_FUSED_HITS,    // hits of the current chunk on the fused path (its pool counters count slots)
  C_COUNT
};
static_assert(C_HITS % 2 == 0, "the 64-bit hit total needs an 8-byte aligned slot");

// Particle constants of a wave-uniform particle index, kept in scalar
// registers (each 32-bit word is made uniform explicitly: the compiler cannot
// prove that the record stores of the kernel leave the array untouched).
__device__ __forceinline__ ParticleConst load_uniform(const ParticleConst* src) {
  ParticleConst r;
  const int* s = reinterpret_cast<const int*>(src);
  int* d = reinterpret_cast<int*>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(ParticleConst) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(s[i]);
  return r;
}

// Persistent trace: every block takes work items (a tile of `tile` incident
// rays of one particle) from the chunk's queue until it is empty.  Items are
// numbered particle by particle in launch order (largest particles first),
// so the cheap items of small particles fill the tail.  The GEN instance
// traces the particles observed at a finite radius or absorbing (see
// trace_ray), the other one the rest; each skips the other's items, so a
// particle's result never depends on the particles it is batched with.
template <typename G, bool GEN>
__global__ void __launch_bounds__(256, (sizeof(G) == 8 || GEN) ? 2 : 3)
    k_trace_tiles(const BatchDev B, const Records<G> rec, unsigned* queue) {
  __shared__ long s_item;
  const long n_items = B.tile_off[B.n] - B.tile_base;
  for (;;) {
    if (threadIdx.x == 0) s_item = (long)atomicAdd(queue, 1u);
    __syncthreads();
    const long item = s_item;
    __syncthreads();
    if (item >= n_items) break;
    const int p = __builtin_amdgcn_readfirstlane(find_part(B.tile_off, B.n, B.tile_base, item));
    const ParticleConst P = load_uniform(B.P + p);
    if (GEN != needs_general_trace(P)) continue;
    const long NN = (long)P.N * P.N;
    const long first = (item - (B.tile_off[p] - B.tile_base)) * B.tile;
    const long last = min(first + (long)B.tile, NN);
    const long rbase = B.n_ord * (B.ray_off[p] - B.ray_base);
    const long chunk_ray0 = B.ray_off[p] - B.ray_base;
    for (long r0 = first; r0 < last; r0 += blockDim.x) {
      const long id = r0 + threadIdx.x;
      bool redo = false;
      if (id < last) {
        for (int o = 0; o < B.n_ord; ++o) rec.flags[rbase + o * NN + id] = 0;
        RecordSink<G> sink{rec, rbase, NN, id, P.k, P.amplif_limit, false, P.k * P.robs};
        const int iy = div_quot15((int)id, P.N), ix = (int)id - iy * P.N;
        trace_ray<G, GEN>(P, ix, iy, sink);
        redo = sink.need64;
      }
      if (sizeof(G) == 4) {
        // rays whose divergence factor is ill-conditioned in FP32 are listed
        // for the FP64 pass (one append per wave)
        const unsigned long long mask = __ballot(redo);
        if (mask) {
          const int lane = threadIdx.x & 63, leader = __ffsll((long long)mask) - 1;
          unsigned base = 0;
          if (lane == leader) base = atomicAdd(rec.n_fp64, (unsigned)__popcll(mask));
          base = __shfl(base, leader);
          if (redo) rec.redo_list[base + __popcll(mask & ((1ull << lane) - 1ull))] = (int)(chunk_ray0 + id);
        }
      }
    }
  }
}

// FP64 re-trace of the listed rays, writing into the FP32 records.  A fixed
// grid strides over the list, whose length is only known on the device.
__global__ void __launch_bounds__(256) k_retrace64(const BatchDev B, const Records<float> rec) {
  const unsigned n = *rec.n_fp64;
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const long g = rec.redo_list[i];
    const int p = find_part(B.ray_off, B.n, B.ray_base, g);
    const ParticleConst& P = B.P[p];
    const long NN = (long)P.N * P.N;
    const long id = g - (B.ray_off[p] - B.ray_base);
    const long rbase = B.n_ord * (B.ray_off[p] - B.ray_base);
    for (int o = 0; o < B.n_ord; ++o) rec.flags[rbase + o * NN + id] = 0;
    RecordSink<float> sink{rec, rbase, NN, id, P.k, 0.0, false, P.k * P.robs};
    const int iy = (int)(id / P.N), ix = (int)(id - (long)iy * P.N);
    trace_ray<double>(P, ix, iy, sink);
  }
}

// FP64 re-trace of one ray inside k_fused, into its scratch records.
template <bool GEN>
__device__ __forceinline__ void fused_retrace(const ParticleConst& P, int ix, int iy, LRec* rb, int n_ord,
                                              double kappa) {
  for (int o = 0; o < n_ord; ++o) rb[o].flags = 0;
  ScratchSink sk{rb, P.k, kappa, P.n_pol};
  trace_ray<double, GEN>(P, ix, iy, sk);
}

// The mixed-path far field of plain particles (or, GEN, of those observed at
// a finite radius or absorbing) in one persistent kernel: blocks take tiles
// of 64 x 4 steps rays from the chunk's queue; per step, each interaction
// that emits an order is followed by the rasterisation of that order's quads
// of the step (fused_raster), rays ill-conditioned in FP32 being re-traced in
// FP64 by the block.  carry: dynamic LDS, n_ord x 64 records (the last ray
// row of the previous step, per order slot).
template <bool GEN>
__global__ void __launch_bounds__(256, FUSED_BPC)
    k_fused(const BatchDev B, const NodeGrid ng, const FusedPool fp, unsigned* queue, const int steps,
            const double margin) {
  __shared__ FusedShared sh;
  extern __shared__ LRec carry[];
  const int tid = threadIdx.x, lane = tid & 63, row = tid >> 6;
  const long n_items = B.tile_off[B.n] - B.tile_base;
  const AxisFast axt = axis_fast(ng.seg_t, ng.n_theta), axp = axis_fast(ng.seg_p, ng.n_phi);
  LRec* scratch = fp.scratch + (long)blockIdx.x * 256 * B.n_ord;
  const int QH = FUSED_ROWS * steps - 1;  // quad rows per tile
  // the wave's run of hit-pool slots (empty: the first hit takes a run)
  SlotRun run;
  run.part = (int)(((long)blockIdx.x * FUSED_ROWS + row) % NPART);
  run.next = run.end = 0;
  if (tid == 0) sh.n_hit = 0;
  for (;;) {
    if (tid == 0) sh.item = (long)atomicAdd(queue, 1u);
    __syncthreads();
    const long item = sh.item;
    __syncthreads();
    if (item >= n_items) break;
    const int p = __builtin_amdgcn_readfirstlane(find_part(B.tile_off, B.n, B.tile_base, item));
    const ParticleConst P = load_uniform(B.P + p);
    if (GEN != needs_general_trace(P)) continue;
    const int N = P.N;
    const int tiles_x = (N - 2) / 63 + 1;
    const long local = item - (B.tile_off[p] - B.tile_base);
    const int sy = (int)(local / tiles_x), sx = (int)(local - (long)sy * tiles_x);
    FusedStep st;
    st.N = N;
    st.part = p;
    st.col0 = 63 * sx;
    st.nq = (long)(N - 1) * (N - 1);
    st.node0 = p * ng.n_theta * ng.n_phi;
    const int row0 = QH * sy;
    const double kappa = P.k * P.robs;
    for (int k = 0; k < steps; ++k) {
      const int r0 = row0 + FUSED_ROWS * k;
      if (r0 >= N) break;  // block-uniform: the tile's remaining rows lie beyond the grid
      st.row_top = r0 - 1;
      st.first = k == 0;
      const int ix = st.col0 + lane, iy = r0 + row;
      RayState<float> s;
      bool alive = ix < N && iy < N && ray_init(P, ix, iy, s);
      if (tid == 0) sh.n_list = 0;
      // a step none of whose rays meets the particle: the next step's first
      // quad row has no valid upper corners
      // (one vote buffer per step parity: a wave may reach the next step's vote
      // before another has read this one when the step has no interactions)
      int* vote = sh.wave_any[k & 1];
      const unsigned long long wv = __ballot(alive);
      if (lane == 0) vote[row] = wv != 0ull;
      __syncthreads();
      const bool any = vote[0] | vote[1] | vote[2] | vote[3];
      if (!any) {
        for (int o = row; o < B.n_ord; o += FUSED_ROWS) carry[o * FUSED_COLS + lane].flags = 0;
      }
      bool redo = false;
      int my_e = 0, done = 0;
      for (int q = 1; any && q <= P.p_max + 1; ++q) {
        const int slot = q - 1 - P.p_min;  // order slot emitted at this interaction, if any
        LdsSink sink{&sh.T[row][lane], P.k, kappa, P.amplif_limit, P.n_pol, false, false};
        if (alive) alive = (ray_interact<float, GEN>(P, q, s, sink) & 2) != 0;
        if (slot < 0) continue;  // block-uniform
        if (sink.need64) {
          redo = true;
          alive = false;
          my_e = atomicAdd(&sh.n_list, 1);
          sh.list[my_e] = tid;
        } else if (!sink.wrote && !redo) {
          sh.T[row][lane].flags = 0;
        }
        __syncthreads();
        // rays listed at this interaction: traced again in FP64, one per
        // thread.  Every thread parks its own FP32 ray state in global memory
        // meanwhile, so that the FP64 trace has the registers to itself.
        const int n_list = sh.n_list;
        if (n_list > done) {
          RayState<float>* park = fp.park + (long)blockIdx.x * 256 + tid;
          *park = s;
          const int e = done + tid;
          if (e < n_list) {
            const int who = sh.list[e];
            fused_retrace<GEN>(P, st.col0 + (who & 63), r0 + (who >> 6), scratch + (long)e * B.n_ord, B.n_ord, kappa);
          }
          if (tid == 0) atomicAdd(fp.n_fp64, (unsigned)(n_list - done));
          done = n_list;
          s = *park;
          __syncthreads();
        }
        if (redo) sh.T[row][lane] = scratch[(long)my_e * B.n_ord + slot];
        __syncthreads();
        st.slot = slot;
        fused_raster(sh, carry + slot * FUSED_COLS, ng, axt, axp, fp, st, margin, run);
        __syncthreads();
        if (row == FUSED_ROWS - 1) carry[slot * FUSED_COLS + lane] = sh.T[FUSED_ROWS - 1][lane];
      }
    }
  }
  close_run(fp, run);
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

constexpr double D2R = 3.14159265358979323846 / 180.0;

// Split a node-angle list (degrees, turned to radians as the node tables
// are) into uniformly spaced runs, one block of 256 threads.  A "break" is an
// index where the spacing changes; more than MAXSEG - 1 breaks leaves the
// list to binary search, and so does a run whose nodes deviate from its
// arithmetic model by more than 1e-10 of its step (the lookups allow 1e-9).
__device__ void axis_segments(const double* deg, int n, AxisSeg* out) {
  __shared__ int nbreak, bad;
  __shared__ int brk[MAXSEG];
  __shared__ AxisSeg sg;
  auto v = [&](int i) { return deg[i] * D2R; };
  if (threadIdx.x == 0) { nbreak = 0; bad = 0; }
  __syncthreads();
  for (int i = 1 + (int)threadIdx.x; i < n - 1; i += blockDim.x) {
    const double d0 = v(i) - v(i - 1), d1 = v(i + 1) - v(i);
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
      sg.v0[k] = v(lo);
      sg.vend[k] = v(hi);
      sg.step[k] = (v(hi) - v(lo)) / (double)(hi - lo);
      sg.inv_step[k] = 1.0 / sg.step[k];
      lo = hi;
    }
    sg.nseg = nb + 1;
  }
  __syncthreads();
  for (int k = 0; k < sg.nseg; ++k)
    for (int i = sg.start[k] + (int)threadIdx.x; i <= sg.end[k]; i += blockDim.x) {
      const double model = sg.v0[k] + (double)(i - sg.start[k]) * sg.step[k];
      if (!(fabs(v(i) - model) <= 1e-10 * sg.step[k])) bad = 1;
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (bad) sg.nseg = 0;
    *out = sg;
  }
}

// Once per call: the uniform runs of the two angle lists (blocks 0 and 1,
// first so that their serial part overlaps the rest), then node tables from
// the degree lists, workspace header, counters and the first chunk's node
// counts (the blocks after those).
// With one != 0 the call has one particle, whose metadata is written here
// from the kernel arguments (no host upload).
__global__ void __launch_bounds__(256) k_setup(int n_theta, const double* theta_deg, int n_phi, const double* phi_deg,
                                               double* th, double* ph, double* sth, double* cth, double* sph,
                                               double* cph, float* tf, unsigned* counter, WsHeader* hdr, WsHeader hv,
                                               ParticleConst* meta_P, long* meta_off, int* meta_out, ParticleConst P1,
                                               long items1, int one, int* count0, long n_count0, AxisSeg* seg_t,
                                               AxisSeg* seg_p) {
  if (blockIdx.x < 2) {  // block-uniform
    if (blockIdx.x == 0) axis_segments(theta_deg, n_theta, seg_t);
    else axis_segments(phi_deg, n_phi, seg_p);
    return;
  }
  const long i = (long)(blockIdx.x - 2) * blockDim.x + threadIdx.x;
  if (i < n_count0) count0[i] = 0;
  if (i < n_theta) {
    double t = theta_deg[i] * D2R;
    th[i] = t;
    sth[i] = sin(t);
    cth[i] = cos(t);
    tf[i] = (float)sth[i];
    tf[n_theta + i] = (float)cth[i];
  }
  if (i < n_phi) {
    double p = phi_deg[i] * D2R;
    ph[i] = p;
    sph[i] = sin(p);
    cph[i] = cos(p);
    tf[2 * n_theta + i] = (float)sph[i];
    tf[2 * n_theta + n_phi + i] = (float)cph[i];
  }
  if (i < C_COUNT) counter[i] = 0u;
  if (i == 0) {
    *hdr = hv;
    if (one) {
      const long NN = (long)P1.N * P1.N, nq = (long)(P1.N - 1) * (P1.N - 1);
      meta_P[0] = P1;
      meta_off[0] = 0; meta_off[1] = NN;                    // rays
      meta_off[2] = 0; meta_off[3] = nq;                    // quads
      meta_off[4] = 0; meta_off[5] = items1;                // trace work items
      meta_out[0] = 0;
    }
  }
}

// Forward Fraunhofer diffraction of each particle's shadow (Babinet), added to
// its far field: the shadow on z = 0 is the ellipse with matrix S2, the x-y
// block of R diag(a^2, b^2, c^2) R^T, and its amplitude in direction n is
// (i k / 2 pi) pi sqrt(det S2) 2 J1(k s) / (k s), s = sqrt(n_t^T S2 n_t), carried
// by the incident polarisation in the frame that turns with phi.
template <typename G>
__global__ void __launch_bounds__(256) k_diffraction(const BatchDev B, const NodeGrid ng, int n_nodes, int n_pol,
                                                     G* out) {
  const long gn = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gn >= (long)B.n * n_nodes) return;
  const int pl = (int)(gn / n_nodes);
  const int node = (int)(gn - (long)pl * n_nodes);
  const int it = node / ng.n_phi, ip = node - it * ng.n_phi;
  const ParticleConst& P = B.P[pl];
  double s00 = 0.0, s01 = 0.0, s11 = 0.0;
  for (int q = 0; q < 3; ++q) {
    const double a2 = 1.0 / P.A[q];
    s00 += P.R[q] * P.R[q] * a2;
    s01 += P.R[q] * P.R[3 + q] * a2;
    s11 += P.R[3 + q] * P.R[3 + q] * a2;
  }
  const double cp = ng.cph[ip], sp = ng.sph[ip];
  const double nx = ng.sth[it] * cp, ny = ng.sth[it] * sp;
  const double u = P.k * sqrt(s00 * nx * nx + 2.0 * s01 * nx * ny + s11 * ny * ny);
  const double shape = u < 1e-8 ? 1.0 : 2.0 * bessel_j1(u) / u;
  const double fi = 0.5 * P.k * sqrt(s00 * s11 - s01 * s01) * shape;  // F_d = i fi
  const double pol[2][2] = {{cp, -sp}, {sp, cp}};
  G* po = out + (long)B.out_index[pl] * ((long)n_pol * 2 * n_nodes * 2);
  for (int p = 0; p < n_pol; ++p)
    for (int a = 0; a < 2; ++a) po[((long)(p * 2 + a) * n_nodes + node) * 2 + 1] += (G)(fi * pol[p][a]);
}

// Reset of the per-chunk state: node hit counts and per-chunk counters.
__global__ void k_chunk_reset(int* count, long n_nodes_chunk, unsigned* counter) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_nodes_chunk) count[i] = 0;
  if (i <= C_QUEUE_GEN) counter[i] = 0u;
}

// End of a chunk's counting, one block of 256 threads: fullest partition
// (overflow check), hit and FP64 totals.  On the fused path the partition
// fills count slots handed out in runs; the chunk's hits are counted apart
// (and that count is cleared for the next chunk).
__device__ void pool_check(unsigned* counter, int fused) {
  __shared__ unsigned mx[256];
  __shared__ unsigned long long sm[256];
  const int t = (int)threadIdx.x;
  unsigned m = 0;
  unsigned long long sum = 0;
  for (int i = t; i < NPART; i += 256) {
    m = max(m, counter[i]);
    sum += counter[i];
  }
  mx[t] = m;
  sm[t] = sum;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      mx[t] = max(mx[t], mx[t + w]);
      sm[t] += sm[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    atomicMax(&counter[C_NEED], mx[0]);
    atomicAdd((unsigned long long*)&counter[C_HITS], fused ? (unsigned long long)counter[C_FUSED_HITS] : sm[0]);
    counter[C_FUSED_HITS] = 0u;
    atomicAdd(&counter[C_FP64_TOTAL], counter[C_REDO]);
  }
}

// Node ranges of a chunk, second pass (after k_scan_local): each node's
// exclusive prefix within its scan block plus the sum of the block sums
// before that block, either scanned by k_scan_sums (direct == 0) or added up
// here from the raw block sums (direct != 0: few scan blocks).  The grid's
// last block closes the chunk's counters instead; the hit counts are final
// once the rasterisers (or the fused kernel) have run, and what follows in
// the chunk reads only the partition fills.
__global__ void __launch_bounds__(256) k_scan_add(int* out, long n, const int* bsum, int direct, unsigned* counter,
                                                  int fused) {
  if (blockIdx.x == gridDim.x - 1) {  // block-uniform
    pool_check(counter, fused);
    return;
  }
  __shared__ int lds[4];
  int add;
  if (direct) {
    int s = 0;
    for (int j = (int)threadIdx.x; j < (int)blockIdx.x; j += 256) s += bsum[j];
    block_excl_scan(s, &add, lds);
  } else {
    add = bsum[blockIdx.x];
  }
  const long base = (long)blockIdx.x * SCAN_BLOCK;
  for (int j = threadIdx.x; j < SCAN_BLOCK; j += 256)
    if (base + j < n) out[base + j] += add;
}

// Scan blocks up to which k_scan_add adds up the block sums itself (its work
// grows with their square; beyond, k_scan_sums scans them first).
constexpr long SCAN_DIRECT = 4096;

// Node ranges of a chunk (exclusive scan of its node counts into the range
// cursors) and the close of its counters: two or three launches.
void launch_ranges(const int* count, int* cursor, long n_cnodes, int* bsum, unsigned* counter, int fused,
                   hipStream_t st) {
  const long nsb = (n_cnodes + SCAN_BLOCK - 1) / SCAN_BLOCK;
  const int direct = nsb <= SCAN_DIRECT ? 1 : 0;
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nsb), dim3(256), 0, st, count, n_cnodes, cursor, bsum);
  if (!direct) hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, bsum, (int)nsb);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)(nsb + 1)), dim3(256), 0, st, cursor, n_cnodes, (const int*)bsum,
                     direct, counter, fused);
}

constexpr int ROWS_CAP = 1 << 24;  // (triangle, row) items of large triangles
// row list of the static workspace (512 KB): a full list sends further large
// triangles to the rasteriser's own loop, which is slower but exact
constexpr int STATIC_ROWS_CAP = 1 << 16;

// Status word of rtw_farfield_static: whether the hit pool held every hit.
__global__ void k_static_status(const unsigned* counter, int cap_part, int32_t* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) status[0] = (long)counter[C_NEED] > cap_part ? RTW_ERR_WORKSPACE : RTW_OK;
}

// Triangle keys (order slot, quad, half) are 32-bit: 2 n_ord (N-1)^2 < 2^31.
int check_keys(const rtw_trace_opts* o) {
  const long nq = (long)(o->grid_n - 1) * (o->grid_n - 1);
  if (2L * (o->p_max - o->p_min + 1) * nq >= (1L << 31))
    return fail(RTW_ERR_UNSUPPORTED, "far field needs 2 (p_max - p_min + 1) (grid_n - 1)^2 < 2^31");
  return RTW_OK;
}

// Workspace layout (256-byte aligned sections).  Record arrays are sized for
// the largest chunk; metadata for every particle of the call.
struct Layout {
  size_t hdr, counter, th, ph, sth, cth, sph, cph, tf, seg, mP, moff, mout, flags, rr, dir, ang, ph64, head, cursor,
      bsum, redo, rows, fscr, fpark, link, contrib, desc, hphi, hnf, total;
  size_t fixed;          // everything except the hit pool
  size_t bytes_per_hit;  // link + contrib
};

struct Shape {
  int precision, n_pol, n_ord;
  int n_theta, n_phi;
  int n_parts;          // particles of the call
  long max_chunk_rays;  // incident rays of the largest chunk
  int max_chunk_parts;  // particles of the largest chunk
  long rows_cap;        // (triangle, row) items of the row list
  int corr;             // RTW_CAUSTIC | RTW_DIFFRACTION
  int fused;            // the mixed far field by k_fused (no per-ray records in the workspace)
  long fused_grid;      // blocks of k_fused (its FP64 re-trace scratch is per block)
};

Layout layout(const Shape& S, long cap_total) {
  Layout L;
  const size_t gs = S.precision == RTW_FP64 ? 8 : 4;
  const size_t rr = S.precision == RTW_FP64 ? sizeof(RayRec<double>) : sizeof(RayRec<float>);
  const long n_nodes = (long)S.n_theta * S.n_phi;
  const size_t nrec = S.fused ? 0 : (size_t)S.n_ord * S.max_chunk_rays;  // per-ray record arrays
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
  L.hdr = take(sizeof(WsHeader));
  L.counter = take(sizeof(unsigned) * C_COUNT);
  L.th = take(8 * S.n_theta); L.ph = take(8 * S.n_phi);
  L.sth = take(8 * S.n_theta); L.cth = take(8 * S.n_theta);
  L.sph = take(8 * S.n_phi); L.cph = take(8 * S.n_phi);
  L.tf = take(4 * 2 * ((size_t)S.n_theta + S.n_phi));  // FP32 sin/cos tables
  L.seg = take(2 * sizeof(AxisSeg));
  L.mP = take(sizeof(ParticleConst) * (size_t)S.n_parts);
  L.moff = take(sizeof(long) * 3 * (size_t)(S.n_parts + 1));
  L.mout = take(sizeof(int) * (size_t)S.n_parts);
  L.flags = take(4 * nrec);
  L.rr = take(rr * nrec);
  L.dir = take((S.precision == RTW_FP64 ? sizeof(Dir4<double>) : sizeof(Dir4<float>)) * nrec);
  L.ang = take(sizeof(float2) * nrec);
  const bool caustic = S.corr & RTW_CAUSTIC;
  L.ph64 = take(caustic ? sizeof(double) * nrec : 0);
  L.head = take(4 * (size_t)S.max_chunk_parts * n_nodes);
  L.cursor = take(4 * (size_t)S.max_chunk_parts * n_nodes);
  L.bsum = take(4 * ((size_t)S.max_chunk_parts * n_nodes / SCAN_BLOCK + 1));
  L.redo = take(S.precision == RTW_FP64 || S.fused ? 4 : 4 * (size_t)S.max_chunk_rays);
  L.rows = take(S.fused ? 0 : sizeof(int2) * (size_t)S.rows_cap);
  L.fscr = take(S.fused ? sizeof(LRec) * 256 * (size_t)S.n_ord * S.fused_grid : 0);
  L.fpark = take(S.fused ? sizeof(RayState<float>) * 256 * (size_t)S.fused_grid : 0);
  L.fixed = off;
  // a hit: its descriptor (fused: its hit record), then its key and contribution in node order
  const size_t ds = S.fused ? 16 * (1 + (size_t)S.n_pol)
                            : (S.precision == RTW_FP64 ? sizeof(HitDesc<double>) : sizeof(HitDesc<float>));
  L.bytes_per_hit = sizeof(int) + gs * 4 * S.n_pol + ds + (caustic ? sizeof(double) + sizeof(int) : 0);
  L.link = take(sizeof(int) * (size_t)cap_total);
  L.contrib = take(gs * 4 * S.n_pol * (size_t)cap_total);
  L.desc = take(ds * (size_t)cap_total);
  L.hphi = take(caustic ? sizeof(double) * (size_t)cap_total : 0);
  L.hnf = take(caustic ? sizeof(int) * (size_t)cap_total : 0);
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

int check_grid(const rtw_grid* g) {
  if (!g) return fail(RTW_ERR_INVALID_ARG, "NULL grid");
  if (g->n_theta < 1 || g->n_phi < 1 || !g->theta_deg || !g->phi_deg)
    return fail(RTW_ERR_INVALID_ARG, "empty node grid");
  if (g->n_theta > 65535 || g->n_phi > 65535) return fail(RTW_ERR_INVALID_ARG, "node grid sides must be < 65536");
  if ((long)g->n_theta * g->n_phi > (1L << 30)) return fail(RTW_ERR_INVALID_ARG, "node grid too large");
  return RTW_OK;
}

// Launch order, chunks and per-particle metadata of a call.
struct Plan {
  Shape S;
  std::vector<ParticleConst> P;  // launch order
  std::vector<long> ray_off, quad_off, tile_off;
  std::vector<int> out_index;
  std::vector<std::pair<int, int>> chunks;  // [first, last) in launch order
  int tile;
};

constexpr long DEFAULT_RAYS_PER_CHUNK = 1L << 26;
constexpr double DEFAULT_HITS_PER_NODE = 6.0;
constexpr int DEFAULT_TILE_STAGED = 2048;  // rays per trace work item (C2: 1.222 ms against 1.238 at 1024)
constexpr int DEFAULT_TILE_FUSED = 2048;   // 64 x 32 rays: 8 steps of 64 x 4

int compute_units();

// Whether a call runs the fused kernel: asked for by the caller, the mixed
// path, at most FUSED_MAX_ORD orders (the LDS carry), no caustic correction
// (it needs the rays' FP64 phases at every hit).
bool use_fused(const rtw_trace_opts* o, bool want) {
  return want && o->precision == RTW_MIXED && o->p_max - o->p_min + 1 <= FUSED_MAX_ORD &&
         !(o->corrections & RTW_CAUSTIC);
}

// Work items (tiles) of one particle: the staged trace's runs of `tile` rays,
// or the fused kernel's 64 x (tile / 64)-ray tiles, neighbours sharing a ray
// column or row (63 x (tile / 64 - 1) quads each).
long tiles_of(int N, int tile, bool fused) {
  if (!fused) return ((long)N * N + tile - 1) / tile;
  const int qh = tile / FUSED_COLS - 1;
  return (long)((N - 2) / (FUSED_COLS - 1) + 1) * ((N - 2) / qh + 1);
}

// Largest particles first (LPT); chunks are filled greedily up to the ray
// budget (a larger particle is a chunk of its own).  Every chunk keeps its
// 32-bit triangle keys and record indices in range.
int make_plan(int n, const rtw_particle* parts, const int* grid_n, const rtw_incident* inc,
              const rtw_trace_opts* opts, const rtw_grid* grid, long rays_per_chunk, int tile, bool want_fused,
              Plan& pl) {
  if (n < 1 || !parts || !grid_n) return fail(RTW_ERR_INVALID_ARG, "need n >= 1 particles and grid sides");
  int rc = check_grid(grid);
  if (rc) return rc;
  const int n_ord = opts ? opts->p_max - opts->p_min + 1 : 0;
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) {
    rtw_trace_opts o = *opts;
    o.grid_n = grid_n[i];
    rc = check_particle(&parts[i], inc, &o);
    if (rc) return fail(rc, "particle %d: %s", i, g_err.c_str());
    idx[i] = i;
  }
  const long key_limit = (1L << 30) / n_ord;  // chunk rays: 2 n_ord quads < 2^31
  for (int i = 0; i < n; ++i)
    if ((long)grid_n[i] * grid_n[i] > key_limit)
      return fail(RTW_ERR_UNSUPPORTED, "particle %d: n_ord grid_n^2 must stay below 2^30", i);
  if (rays_per_chunk <= 0) rays_per_chunk = DEFAULT_RAYS_PER_CHUNK;
  rays_per_chunk = std::min(rays_per_chunk, key_limit);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return grid_n[a] > grid_n[b]; });
  const bool fused = use_fused(opts, want_fused);
  if (tile <= 0) tile = fused ? DEFAULT_TILE_FUSED : DEFAULT_TILE_STAGED;
  pl.tile = tile;
  pl.P.resize(n);
  pl.out_index.resize(n);
  pl.ray_off.assign(n + 1, 0);
  pl.quad_off.assign(n + 1, 0);
  pl.tile_off.assign(n + 1, 0);
  for (int j = 0; j < n; ++j) {
    const int i = idx[j];
    rtw_trace_opts o = *opts;
    o.grid_n = grid_n[i];
    pl.P[j] = make_const(&parts[i], inc, &o);
    pl.out_index[j] = i;
    const long NN = (long)grid_n[i] * grid_n[i];
    pl.ray_off[j + 1] = pl.ray_off[j] + NN;
    pl.quad_off[j + 1] = pl.quad_off[j] + (long)(grid_n[i] - 1) * (grid_n[i] - 1);
    pl.tile_off[j + 1] = pl.tile_off[j] + tiles_of(grid_n[i], tile, fused);
  }
  pl.S.precision = opts->precision;
  pl.S.n_pol = inc->n_pol;
  pl.S.n_ord = n_ord;
  pl.S.n_theta = grid->n_theta;
  pl.S.n_phi = grid->n_phi;
  pl.S.n_parts = n;
  pl.S.max_chunk_rays = 0;
  pl.S.max_chunk_parts = 0;
  pl.S.rows_cap = ROWS_CAP;
  pl.S.corr = opts->corrections;
  pl.S.fused = fused ? 1 : 0;
  pl.S.fused_grid = 0;
  // node indices of a chunk (chunk particle, theta, phi) are 32-bit: a chunk
  // holds at most (2^31 - 1) / n_nodes particles
  const long n_nodes = (long)grid->n_theta * grid->n_phi;
  const long max_parts = std::min<long>(65535, ((1L << 31) - 1) / n_nodes);
  int c0 = 0;
  while (c0 < n) {
    int c1 = c0 + 1;
    while (c1 < n && c1 - c0 < max_parts && pl.ray_off[c1 + 1] - pl.ray_off[c0] <= rays_per_chunk) ++c1;
    pl.chunks.push_back({c0, c1});
    pl.S.max_chunk_rays = std::max(pl.S.max_chunk_rays, pl.ray_off[c1] - pl.ray_off[c0]);
    pl.S.max_chunk_parts = std::max(pl.S.max_chunk_parts, c1 - c0);
    if (fused) {
      // k_fused's per-block scratch is sized for the most blocks any tuning
      // can ask for (tiles of 256 rays, the smallest tile_rays accepted), so
      // that the workspace size does not depend on the tuning of the call
      long items = 0;
      for (int c = c0; c < c1; ++c) items += tiles_of(pl.P[c].N, 256, true);
      pl.S.fused_grid = std::max(pl.S.fused_grid, std::min<long>(items, (long)compute_units() * FUSED_BPC));
    }
    c0 = c1;
  }
  return RTW_OK;
}

struct Tuning {
  int tile, blocks_per_cu, cand_inline;
};

Tuning tuning_of(const rtw_tune* t) {
  Tuning u{0, 8, CAND_INLINE};  // tile 0: the pipeline's default
  if (t) {
    if (t->tile_rays > 0) u.tile = t->tile_rays;
    if (t->blocks_per_cu > 0) u.blocks_per_cu = t->blocks_per_cu;
    if (t->cand_inline > 0) u.cand_inline = t->cand_inline;
  }
  return u;
}

int check_tuning(const Tuning& u) {
  if (u.tile % 256 != 0 || u.tile > (1 << 20)) return fail(RTW_ERR_INVALID_ARG, "tile_rays must be a multiple of 256");
  if (u.blocks_per_cu > 64) return fail(RTW_ERR_INVALID_ARG, "blocks_per_cu must be at most 64");
  if (u.cand_inline > 4096) return fail(RTW_ERR_INVALID_ARG, "cand_inline must be at most 4096");
  return RTW_OK;
}

int compute_units() {
  static int cu = 0;
  if (cu == 0) {
    int dev = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1) cu = 256;
  }
  return cu;
}

// The kernels of chunk [c0, c1) on the fused path: k_fused (trace,
// rasterisation and hit contributions), the scan of the node counts, the
// scatter into node order, the ordered per-node sum, the diffraction term,
// the pool check.
int launch_fused(const Plan& pl, const Tuning& tu, int c0, int c1, const BatchDev& B, const NodeGrid& ng,
                 const HitPool<float>& pool, char* ws, const Layout& L, unsigned* counter, long items, long n_cnodes,
                 int n_nodes, void* out, int32_t* ncontrib, void* incoh, hipStream_t st) {
  const Shape& S = pl.S;
  FusedPool fp;
  fp.count = pool.count;
  fp.counter = counter;
  fp.hits = (V4<float>*)(ws + L.desc);
  fp.cap_part = pool.cap_part;
  fp.n_pol = S.n_pol;
  fp.scratch = (LRec*)(ws + L.fscr);
  fp.park = (RayState<float>*)(ws + L.fpark);
  fp.n_fp64 = counter + C_REDO;
  fp.n_hits = counter + C_FUSED_HITS;
  const long grid_f = std::min<long>({items, (long)compute_units() * std::min(tu.blocks_per_cu, FUSED_BPC),
                                      S.fused_grid});
  const size_t lds = sizeof(LRec) * FUSED_COLS * (size_t)S.n_ord;  // the carry
  const int steps = pl.tile / (FUSED_COLS * FUSED_ROWS);
  // the carry with the static LDS exceeds 64 KB: allow the kernels that much
  // dynamic LDS, once per device with that device current
  {
    static std::mutex lds_mu;
    static bool lds_set[64] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
      return fail(RTW_ERR_DEVICE, "fused far field: no current device");
    std::lock_guard<std::mutex> lk(lds_mu);
    if (!lds_set[dev]) {
      const int most = (int)(sizeof(LRec) * FUSED_COLS * FUSED_MAX_ORD);
      hipError_t e = hipFuncSetAttribute((const void*)k_fused<false>, hipFuncAttributeMaxDynamicSharedMemorySize, most);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_fused<true>, hipFuncAttributeMaxDynamicSharedMemorySize, most);
      if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "fused far field: LDS attribute: %s", hipGetErrorString(e));
      lds_set[dev] = true;
    }
  }
  { ProfScope ps("k_fused_mixed", st);
  bool any_gen = false, any_plain = false;
  for (int c = c0; c < c1; ++c) (needs_general_trace(pl.P[c]) ? any_gen : any_plain) = true;
  if (any_plain)
    hipLaunchKernelGGL(k_fused<false>, dim3((unsigned)grid_f), dim3(256), lds, st, B, ng, fp, counter + C_QUEUE,
                       steps, BOX_MARGIN);
  if (any_gen)
    hipLaunchKernelGGL(k_fused<true>, dim3((unsigned)grid_f), dim3(256), lds, st, B, ng, fp, counter + C_QUEUE_GEN,
                       steps, BOX_MARGIN); }
  { ProfScope ps("k_scan", st);
  launch_ranges(pool.count, pool.cursor, n_cnodes, (int*)(ws + L.bsum), counter, 1, st); }
  { ProfScope ps("k_scatter", st);
  const long slots = (long)NPART * pool.cap_part;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, st, fp, pool); }
  { ProfScope ps("k_node_sum_mixed", st);
  hipLaunchKernelGGL((k_node_sum<float, false>), dim3((unsigned)((n_cnodes + 255) / 256)), dim3(256), 0, st, B, pool,
                     n_nodes, S.n_pol, (float*)out, ncontrib, (float*)incoh, 1); }
  if (S.corr & RTW_DIFFRACTION) {
    ProfScope ps("k_diffraction", st);
    hipLaunchKernelGGL(k_diffraction<float>, dim3((unsigned)((n_cnodes + 255) / 256)), dim3(256), 0, st, B, ng,
                       n_nodes, S.n_pol, (float*)out);
  }
  return RTW_OK;
}

// Queue every kernel of a call on the stream.  With one_meta the single
// particle's metadata is written by k_setup; otherwise the caller uploaded it.
template <typename G>
int launch_plan(const Plan& pl, const Tuning& tu, const rtw_grid* grid, void* out, int32_t* ncontrib, void* incoh,
                char* ws, size_t ws_bytes, hipStream_t st, bool one_meta) {
  const Shape& S = pl.S;
  const int n_nodes = grid->n_theta * grid->n_phi;
  Layout base = layout(S, 0);
  long cap_part = cap_from_bytes(base, ws_bytes);
  if (cap_part < 1) return fail(RTW_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu-byte minimum",
                                ws_bytes, base.fixed + base.bytes_per_hit * NPART + 512);
  if (cap_part > (1L << 30) / NPART) cap_part = (1L << 30) / NPART;
  Layout L = layout(S, cap_part * NPART);
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
  ng.kappa = pl.P[0].k * pl.P[0].robs;  // one incident set-up for every particle of a call
  float* tf = (float*)(ws + L.tf);
  ng.sthf = tf; ng.cthf = tf + grid->n_theta;
  ng.sphf = tf + 2 * grid->n_theta; ng.cphf = tf + 2 * grid->n_theta + grid->n_phi;
  unsigned* counter = (unsigned*)(ws + L.counter);
  Records<G> rec;
  rec.flags = (int32_t*)(ws + L.flags);
  rec.rr = (RayRec<G>*)(ws + L.rr);
  rec.dir = (Dir4<G>*)(ws + L.dir);
  rec.ang = (float2*)(ws + L.ang);
  rec.n_pol = S.n_pol;
  rec.n_fp64 = counter + C_REDO;
  rec.redo_list = (int*)(ws + L.redo);
  const bool caustic = S.corr & RTW_CAUSTIC;
  rec.ph64 = caustic ? (double*)(ws + L.ph64) : nullptr;
  HitPool<G> pool;
  pool.count = (int*)(ws + L.head);
  pool.cursor = (int*)(ws + L.cursor);
  pool.key = (int*)(ws + L.link);
  pool.contrib = (G*)(ws + L.contrib);
  pool.desc = (HitDesc<G>*)(ws + L.desc);
  pool.counter = counter;
  pool.cap_part = (int)cap_part;
  pool.rows = (int2*)(ws + L.rows);
  pool.n_rows = counter + C_ROWS;
  pool.rows_cap = (int)S.rows_cap;
  pool.phi = caustic ? (double*)(ws + L.hphi) : nullptr;
  pool.nf = caustic ? (int*)(ws + L.hnf) : nullptr;

  ParticleConst* mP = (ParticleConst*)(ws + L.mP);
  long* moff = (long*)(ws + L.moff);
  int* mout = (int*)(ws + L.mout);
  const int n = S.n_parts;
  long* m_ray = moff;
  long* m_quad = moff + (n + 1);
  long* m_tile = moff + 2 * (n + 1);
  if (one_meta) { m_ray = moff; m_quad = moff + 2; m_tile = moff + 4; }

  // the first chunk's node counts are cleared by k_setup, later chunks' by k_chunk_reset
  const long n_count0 = (long)(pl.chunks.front().second - pl.chunks.front().first) * n_nodes;
  const long setup_n = std::max<long>({(long)grid->n_theta, (long)grid->n_phi, (long)C_COUNT, n_count0});
  const int n_main = (int)((setup_n + 255) / 256);
  { ProfScope ps("k_setup", st);
  hipLaunchKernelGGL(k_setup, dim3((unsigned)(n_main + 2)), dim3(256), 0, st, grid->n_theta, grid->theta_deg,
                     grid->n_phi, grid->phi_deg, (double*)ng.th, (double*)ng.ph, (double*)ng.sth, (double*)ng.cth,
                     (double*)ng.sph, (double*)ng.cph, tf, counter, (WsHeader*)(ws + L.hdr), hv, mP, moff, mout,
                     pl.P[0], pl.tile_off[1], one_meta ? 1 : 0, pool.count, n_count0, (AxisSeg*)(ws + L.seg),
                     (AxisSeg*)(ws + L.seg) + 1); }

  const bool fp64 = S.precision == RTW_FP64;
  const int cu = compute_units();
  for (const auto& ch : pl.chunks) {
    const int c0 = ch.first, c1 = ch.second, nc = c1 - c0;
    BatchDev B;
    B.n = nc;
    B.n_ord = S.n_ord;
    B.P = mP + c0;
    B.ray_off = m_ray + c0;
    B.quad_off = m_quad + c0;
    B.tile_off = m_tile + c0;
    B.out_index = mout + c0;
    B.ray_base = pl.ray_off[c0];
    B.quad_base = pl.quad_off[c0];
    B.tile_base = pl.tile_off[c0];
    B.tile = pl.tile;
    const long rays = pl.ray_off[c1] - pl.ray_off[c0];
    const long quads = pl.quad_off[c1] - pl.quad_off[c0];
    const long items = pl.tile_off[c1] - pl.tile_off[c0];
    const long n_cnodes = (long)nc * n_nodes;
    if (c0 != pl.chunks.front().first)
      hipLaunchKernelGGL(k_chunk_reset, dim3((unsigned)((std::max<long>(n_cnodes, C_COUNT) + 255) / 256)),
                         dim3(256), 0, st, pool.count, n_cnodes, counter);
    if constexpr (sizeof(G) == 4) {
      if (S.fused) {
        int rc = launch_fused(pl, tu, c0, c1, B, ng, pool, ws, L, counter, items, n_cnodes, n_nodes, out, ncontrib,
                              incoh, st);
        if (rc) return rc;
        continue;
      }
    }
    { ProfScope ps(fp64 ? "k_trace_fp64" : "k_trace_mixed", st);
    const long grid_t = std::min<long>(items, (long)cu * tu.blocks_per_cu);
    bool any_gen = false, any_plain = false;
    for (int c = c0; c < c1; ++c) (needs_general_trace(pl.P[c]) ? any_gen : any_plain) = true;
    if (any_plain)
      hipLaunchKernelGGL((k_trace_tiles<G, false>), dim3((unsigned)grid_t), dim3(256), 0, st, B, rec,
                         counter + C_QUEUE);
    if (any_gen)
      hipLaunchKernelGGL((k_trace_tiles<G, true>), dim3((unsigned)grid_t), dim3(256), 0, st, B, rec,
                         counter + C_QUEUE_GEN); }
    if (!fp64) {
      ProfScope ps("k_retrace64", st);
      // two waves per SIMD (its registers): the grid that fits at once strides over the list
      hipLaunchKernelGGL(k_retrace64, dim3((unsigned)std::min<long>(2L * cu, (rays + 255) / 256)), dim3(256), 0, st,
                         B, *reinterpret_cast<Records<float>*>(&rec));
    }
    { ProfScope ps(fp64 ? "k_raster_fp64" : "k_raster_mixed", st);
    hipLaunchKernelGGL(k_raster<G>, dim3((unsigned)((quads + 255) / 256), S.n_ord), dim3(256), 0, st, B, rec, ng,
                       pool, BOX_MARGIN, tu.cand_inline); }
    { ProfScope ps(fp64 ? "k_raster_rows_fp64" : "k_raster_rows_mixed", st);
    hipLaunchKernelGGL(k_raster_rows<G>, dim3(1024), dim3(256), 0, st, B, rec, ng, pool, BOX_MARGIN); }
    { ProfScope ps("k_scan", st);
    launch_ranges(pool.count, pool.cursor, n_cnodes, (int*)(ws + L.bsum), counter, 0, st); }
    { ProfScope ps(fp64 ? "k_store_hits_fp64" : "k_store_hits_mixed", st);
    const long slots = (long)NPART * cap_part;
    hipLaunchKernelGGL(k_store_hits<G>, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, st, B, rec, ng, pool); }
    { ProfScope ps(fp64 ? "k_node_sum_fp64" : "k_node_sum_mixed", st);
    if (pool.phi)
      hipLaunchKernelGGL((k_node_sum<G, true>), dim3((unsigned)((n_cnodes + 255) / 256)), dim3(256), 0, st, B, pool,
                         n_nodes, S.n_pol, (G*)out, ncontrib, (G*)incoh, 0);
    else
      hipLaunchKernelGGL((k_node_sum<G, false>), dim3((unsigned)((n_cnodes + 255) / 256)), dim3(256), 0, st, B, pool,
                         n_nodes, S.n_pol, (G*)out, ncontrib, (G*)incoh, 0); }
    if (S.corr & RTW_DIFFRACTION) {
      ProfScope ps("k_diffraction", st);
      hipLaunchKernelGGL(k_diffraction<G>, dim3((unsigned)((n_cnodes + 255) / 256)), dim3(256), 0, st, B, ng, n_nodes,
                         S.n_pol, (G*)out);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return RTW_OK;
}

// Upload of the plan's metadata into the workspace (synchronises the stream:
// the host copy must outlive the transfer).
int upload_plan(const Plan& pl, const Layout& L, char* ws, hipStream_t st) {
  const int n = pl.S.n_parts;
  std::vector<long> off(3 * (size_t)(n + 1));
  std::copy(pl.ray_off.begin(), pl.ray_off.end(), off.begin());
  std::copy(pl.quad_off.begin(), pl.quad_off.end(), off.begin() + (n + 1));
  std::copy(pl.tile_off.begin(), pl.tile_off.end(), off.begin() + 2 * (n + 1));
  hipError_t e = hipMemcpyAsync(ws + L.mP, pl.P.data(), sizeof(ParticleConst) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.moff, off.data(), sizeof(long) * off.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.mout, pl.out_index.data(), sizeof(int) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "metadata upload failed: %s", hipGetErrorString(e));
  return RTW_OK;
}

size_t plan_bytes(const Plan& pl, double hits_per_node) {
  if (!(hits_per_node > 0.0)) hits_per_node = DEFAULT_HITS_PER_NODE;
  const long n_nodes = (long)pl.S.n_theta * pl.S.n_phi;
  long cap_part = (long)std::ceil(hits_per_node * (double)n_nodes * pl.S.max_chunk_parts / NPART) + 256;
  cap_part = std::min(cap_part, (1L << 30) / NPART);
  return layout(pl.S, cap_part * NPART).total + 512;
}

}  // namespace

extern "C" {

const char* rtw_last_error(void) { return g_err.c_str(); }

int rtw_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return RTW_OK;
}

int rtw_profile_only(const char* name) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_only = name ? name : "";
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

const char* rtw_version(void) { return "rtw-mi355x 0.2 (gfx950)"; }

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
  if (!bytes) return fail(RTW_ERR_INVALID_ARG, "NULL bytes");
  if (!opts) return fail(RTW_ERR_INVALID_ARG, "NULL argument struct");
  int rc = check_particle(part, inc, opts);
  if (rc) return rc;
  rc = check_keys(opts);
  if (rc) return rc;
  Plan pl;
  rc = make_plan(1, part, &opts->grid_n, inc, opts, grid, 0, tuning_of(nullptr).tile, false, pl);
  if (rc) return rc;
  *bytes = plan_bytes(pl, hits_per_node);
  return RTW_OK;
}

int rtw_farfield(const rtw_particle* part, const rtw_incident* inc, const rtw_trace_opts* opts,
                 const rtw_grid* grid, void* out_field, int32_t* ncontrib, void* workspace, size_t workspace_bytes,
                 void* hip_stream) {
  if (!opts) return fail(RTW_ERR_INVALID_ARG, "NULL argument struct");
  int rc = check_particle(part, inc, opts);
  if (rc) return rc;
  rc = check_keys(opts);
  if (rc) return rc;
  if (!out_field || !workspace) return fail(RTW_ERR_INVALID_ARG, "NULL output or workspace");
  if (((uintptr_t)workspace & 255) != 0) return fail(RTW_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const Tuning tu = tuning_of(nullptr);
  Plan pl;
  rc = make_plan(1, part, &opts->grid_n, inc, opts, grid, 0, tu.tile, false, pl);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if (opts->precision == RTW_FP64)
    return launch_plan<double>(pl, tu, grid, out_field, ncontrib, nullptr, (char*)workspace, workspace_bytes, st,
                               true);
  return launch_plan<float>(pl, tu, grid, out_field, ncontrib, nullptr, (char*)workspace, workspace_bytes, st, true);
}

int rtw_farfield_static(const rtw_particle* part, const rtw_incident* inc, const rtw_trace_opts* opts,
                        const rtw_grid* grid, void* out_field, int32_t* ncontrib, int32_t* status_out,
                        void* hip_stream) {
  if (!opts) return fail(RTW_ERR_INVALID_ARG, "NULL argument struct");
  int rc = check_particle(part, inc, opts);
  if (rc) return rc;
  rc = check_keys(opts);
  if (rc) return rc;
  if (!out_field) return fail(RTW_ERR_INVALID_ARG, "NULL output");
  const Tuning tu = tuning_of(nullptr);
  Plan pl;
  rc = make_plan(1, part, &opts->grid_n, inc, opts, grid, 0, tu.tile, false, pl);
  if (rc) return rc;
  pl.S.rows_cap = STATIC_ROWS_CAP;
  const size_t need = plan_bytes(pl, 0.0);
  if (need > STATIC_WS_BYTES)
    return fail(RTW_ERR_WORKSPACE, "rtw_farfield_static: this call needs %zu bytes of workspace, the static "
                "workspace holds %zu", need, STATIC_WS_BYTES);
  // the device's copy of the static workspace: its address is taken once per
  // device, with that device current
  static std::mutex mu;
  static void* dev_ptr[64] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= 64)
    return fail(RTW_ERR_DEVICE, "rtw_farfield_static: no current device (%s)", hipGetErrorString(e));
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (!dev_ptr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(RTW_ERR_DEVICE, "rtw_farfield_static: static workspace address: %s", hipGetErrorString(e));
      dev_ptr[dev] = p;
    }
    ws = dev_ptr[dev];
  }
  hipStream_t st = (hipStream_t)hip_stream;
  g_prof_off = true;  // no events (they would be created here)
  if (opts->precision == RTW_FP64)
    rc = launch_plan<double>(pl, tu, grid, out_field, ncontrib, nullptr, (char*)ws, STATIC_WS_BYTES, st, true);
  else
    rc = launch_plan<float>(pl, tu, grid, out_field, ncontrib, nullptr, (char*)ws, STATIC_WS_BYTES, st, true);
  g_prof_off = false;
  if (rc) return rc;
  if (status_out) {
    const Layout L0 = layout(pl.S, 0);
    long cap_part = cap_from_bytes(L0, STATIC_WS_BYTES);
    if (cap_part > (1L << 30) / NPART) cap_part = (1L << 30) / NPART;
    hipLaunchKernelGGL(k_static_status, dim3(1), dim3(64), 0, st, (const unsigned*)((char*)ws + L0.counter),
                       (int)cap_part, status_out);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  }
  return RTW_OK;
}

int rtw_batch_workspace_size(int n, const rtw_particle* parts, const int* grid_n, const rtw_incident* inc,
                             const rtw_trace_opts* opts, const rtw_grid* grid, const rtw_batch_opts* bopts,
                             size_t* bytes) {
  if (!bytes || !opts || !inc) return fail(RTW_ERR_INVALID_ARG, "NULL argument");
  Plan pl;
  int rc = make_plan(n, parts, grid_n, inc, opts, grid, bopts ? (long)bopts->rays_per_chunk : 0,
                     tuning_of(nullptr).tile, bopts && bopts->fused, pl);
  if (rc) return rc;
  *bytes = plan_bytes(pl, bopts ? bopts->hits_per_node : 0.0);
  return RTW_OK;
}

int rtw_batch(int n, const rtw_particle* parts, const int* grid_n, const rtw_incident* inc,
              const rtw_trace_opts* opts, const rtw_grid* grid, void* out_field, int32_t* ncontrib, void* out_incoh,
              const rtw_tune* tune, const rtw_batch_opts* bopts, void* workspace, size_t workspace_bytes,
              void* hip_stream) {
  if (!opts || !inc) return fail(RTW_ERR_INVALID_ARG, "NULL argument struct");
  if (!out_field || !workspace) return fail(RTW_ERR_INVALID_ARG, "NULL output or workspace");
  if (((uintptr_t)workspace & 255) != 0) return fail(RTW_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const Tuning tu = tuning_of(tune);
  int rc = check_tuning(tu);
  if (rc) return rc;
  Plan pl;
  rc = make_plan(n, parts, grid_n, inc, opts, grid, bopts ? (long)bopts->rays_per_chunk : 0, tu.tile,
                 bopts && bopts->fused, pl);
  if (rc) return rc;
  Layout base = layout(pl.S, 0);
  if (workspace_bytes < base.fixed + base.bytes_per_hit * NPART + 512)
    return fail(RTW_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu-byte minimum", workspace_bytes,
                base.fixed + base.bytes_per_hit * NPART + 512);
  hipStream_t st = (hipStream_t)hip_stream;
  rc = upload_plan(pl, base, (char*)workspace, st);
  if (rc) return rc;
  if (opts->precision == RTW_FP64)
    return launch_plan<double>(pl, tu, grid, out_field, ncontrib, out_incoh, (char*)workspace, workspace_bytes, st,
                               false);
  return launch_plan<float>(pl, tu, grid, out_field, ncontrib, out_incoh, (char*)workspace, workspace_bytes, st,
                            false);
}

int rtw_batch_autotune(int n, const rtw_particle* parts, const int* grid_n, const rtw_incident* inc,
                       const rtw_trace_opts* opts, const rtw_grid* grid, const rtw_batch_opts* bopts,
                       void* out_field, void* workspace, size_t workspace_bytes, void* hip_stream, rtw_tune* best) {
  if (!best) return fail(RTW_ERR_INVALID_ARG, "NULL result");
  if (n < 1 || !parts || !grid_n) return fail(RTW_ERR_INVALID_ARG, "need n >= 1 particles");
  hipStream_t st = (hipStream_t)hip_stream;
  // Sample: every k-th particle in size order, at most 64, so that the trial
  // runs see the batch's mix of sizes.
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return grid_n[a] > grid_n[b]; });
  const int m = std::min(n, 64);
  std::vector<rtw_particle> sp(m);
  std::vector<int> sg(m);
  for (int j = 0; j < m; ++j) {
    const int i = idx[(long)j * n / m];
    sp[j] = parts[i];
    sg[j] = grid_n[i];
  }
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return fail(RTW_ERR_DEVICE, "event creation failed");
  auto trial = [&](const rtw_tune& t, float* ms) -> int {
    int rc = rtw_batch(m, sp.data(), sg.data(), inc, opts, grid, out_field, nullptr, nullptr, &t, bopts, workspace,
                       workspace_bytes, st);  // warm-up and upload
    if (rc) return rc;
    hipEventRecord(a, st);
    rc = rtw_batch(m, sp.data(), sg.data(), inc, opts, grid, out_field, nullptr, nullptr, &t, bopts, workspace,
                   workspace_bytes, st);
    if (rc) return rc;
    hipEventRecord(b, st);
    if (hipEventSynchronize(b) != hipSuccess) return fail(RTW_ERR_DEVICE, "event wait failed");
    hipEventElapsedTime(ms, a, b);
    return rtw_farfield_status(workspace, hip_stream, nullptr);
  };
  // coordinate search: trace tile and persistence, then the binning threshold
  rtw_tune cur{1024, 8, CAND_INLINE};
  float best_ms = 0.f;
  int rc = trial(cur, &best_ms);
  const int tiles[] = {256, 512, 1024, 2048, 4096};
  const int bpcs[] = {4, 8, 16};
  const int cands[] = {64, 256, 1024, 4096};
  for (int t : tiles)
    for (int bp : bpcs) {
      if (rc) break;
      rtw_tune c{t, bp, cur.cand_inline};
      if (t == cur.tile_rays && bp == cur.blocks_per_cu) continue;
      float ms = 0.f;
      rc = trial(c, &ms);
      if (!rc && ms < best_ms) { best_ms = ms; cur = c; }
    }
  rtw_tune base = cur;
  for (int c : cands) {
    if (rc) break;
    if (c == base.cand_inline) continue;
    rtw_tune t{base.tile_rays, base.blocks_per_cu, c};
    float ms = 0.f;
    rc = trial(t, &ms);
    if (!rc && ms < best_ms) { best_ms = ms; cur = t; }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (rc) return rc;
  *best = cur;
  return RTW_OK;
}

int rtw_farfield_stats(const void* workspace, void* hip_stream, uint64_t* hits, uint64_t* fp64_rays) {
  if (!workspace) return fail(RTW_ERR_INVALID_ARG, "NULL workspace");
  hipStream_t st = (hipStream_t)hip_stream;
  WsHeader h;
  unsigned cnt[C_COUNT];
  hipError_t e = hipMemcpyAsync(&h, workspace, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cnt, (const char*)workspace + align256(sizeof(WsHeader)), sizeof(cnt), hipMemcpyDeviceToHost,
                       st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "stats read failed: %s", hipGetErrorString(e));
  if (h.magic != WS_MAGIC) return fail(RTW_ERR_INVALID_ARG, "workspace was not used by rtw_farfield");
  uint64_t tot = 0;
  std::memcpy(&tot, &cnt[C_HITS], sizeof(tot));
  if (hits) *hits = tot;
  if (fp64_rays) *fp64_rays = cnt[C_FP64_TOTAL];
  return RTW_OK;
}

int rtw_farfield_status(const void* workspace, void* hip_stream, size_t* bytes_needed) {
  if (!workspace) return fail(RTW_ERR_INVALID_ARG, "NULL workspace");
  hipStream_t st = (hipStream_t)hip_stream;
  WsHeader h;
  unsigned cnt[C_COUNT];
  hipError_t e = hipMemcpyAsync(&h, workspace, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "status read failed: %s", hipGetErrorString(e));
  if (h.magic != WS_MAGIC) return fail(RTW_ERR_INVALID_ARG, "workspace was not used by rtw_farfield");
  // the counters follow the header at the next 256-byte boundary
  e = hipMemcpyAsync(cnt, (const char*)workspace + align256(sizeof(WsHeader)), sizeof(cnt), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(RTW_ERR_DEVICE, "status read failed: %s", hipGetErrorString(e));
  const unsigned mx = cnt[C_NEED];
  if (bytes_needed) {
    size_t per = (size_t)mx + (mx >> 2) + 64;
    *bytes_needed = (size_t)h.fixed_bytes + per * NPART * h.bytes_per_hit + 1024;
  }
  if ((long)mx > h.cap_part)
    return fail(RTW_ERR_WORKSPACE, "hit pool overflow: %u hits in the fullest partition, capacity %d", mx, h.cap_part);
  return RTW_OK;
}

}  // extern "C"
