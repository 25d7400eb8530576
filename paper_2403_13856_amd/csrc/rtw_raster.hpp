// rtw_raster.hpp -- far-field assembly on gfx950: triangle rasterisation of the
// per-ray emission records onto the (theta, phi) node grid, and the per-node
// ordered sum (section "Strategy of Ray Theory of Waves": the amplitude and
// phase are functions of the incident ray; interpolate, then sum coherently).
//
// Each quad (ix, iy)-(ix+1, iy+1) of the incident grid is split along its
// (ix, iy)-(ix+1, iy+1) diagonal.  A triangle contributes when its three rays
// emit the order with the same focal-line count (the direction map folds
// exactly where that count changes).  A node direction n inside the spherical
// triangle (d0, d1, d2) receives sum_v lambda_v F_v exp(i k r_v.(d_v - n)):
// barycentric weights of the central projection, each ray field carried to n
// with the stationary-phase gradient dPhi/d(dir) = -k r_exit.
//
// Membership is watertight: the edge normal of an edge is always formed from
// its lower ray index to its higher one, and its product with a node
// direction is a fixed sequence of correctly rounded operations, so the two
// triangles sharing an edge see the same value and exactly one of them claims
// a node on it (the one on the edge's positive side on an exact tie).
//
// Hits are appended to a pool as descriptors with one atomic per wave per pass
// (wave ballot) on one of NPART counters; each hit takes its rank among its
// node's hits from the node's count atomic (issued first, so that the two
// round trips overlap).  A scan of the counts gives each
// node's range, the hit store places every hit's contribution at its range
// start plus its rank, and the per-node kernel sorts the node's hits by
// triangle key and sums them in that order.  No floating-point atomics are
// used, so the sums are deterministic.
#pragma once
#include "rtw_device.hpp"

namespace rtw {

constexpr int NPART = 1024;        // hit-pool partitions (spreads the append atomics)
constexpr int NODE_SORT_MAX = 16;  // hits per node sorted in registers; more use a selection pass

// An angle list split into uniformly spaced runs (detected on the device), so
// that "first node >= x" is arithmetic rather than a binary search.  nseg == 0
// means the list is not piecewise uniform in at most MAXSEG runs.
constexpr int MAXSEG = 8;
struct AxisSeg {
  int nseg;
  int start[MAXSEG], end[MAXSEG];  // index range [start, end] of each run (ends shared)
  double v0[MAXSEG], step[MAXSEG], inv_step[MAXSEG], vend[MAXSEG];
};

struct NodeGrid {
  int n_theta, n_phi;
  const double* th;   // radians, ascending
  const double* ph;   // radians, ascending, in [0, 2 pi)
  const double* sth;  // sin theta
  const double* cth;
  const double* sph;
  const double* cph;
  const float* sthf;  // FP32 copies of the four tables
  const float* cthf;
  const float* sphf;
  const float* cphf;
  const AxisSeg* seg_t;
  const AxisSeg* seg_p;
  double kappa;       // k R for nodes on the sphere of radius R; 0: far field
};

// One ray's emission record for one order, contiguous so that the three
// vertices of a hit are a few cache lines each (gathered at random).  The
// exit direction lives in its own array of 4-vectors (Records::dir), read
// coalesced by the rasteriser's per-quad pass; the record holds a copy, so
// that the hit store reads one aligned 64 B record (FP32) per vertex.  The
// field is transverse to the direction, so it is stored as its two
// components on the direction's own (e_theta, e_phi) basis (dir_basis of the
// stored direction), which leaves room for the copy.
//
// An FP32 record also keeps what rounding took from its direction, as three
// 16-bit integers in units of 2^-39 (each component's residual is at most half
// an FP32 ulp, 2^-25, so |q| <= 2^14; the rebuilt direction is exact to
// 2^-40): the hit store forms the interpolation weights from the FP64
// direction, because on a long thin triangle (rays near grazing incidence,
// whose exit directions spread along one edge) the rounding of a vertex moves
// the weights by its size over the triangle's small height, up to ~1e-4.
template <typename G>
struct RecTail {
  G pad[2];
};
template <>
struct RecTail<float> {
  int16_t dlo[3];  // (direction - stored FP32 direction) * 2^39
  int16_t pad;
};
constexpr double DLO_SCALE = 549755813888.0;  // 2^39

template <typename G>
struct alignas(16 * sizeof(G)) RayRec {
  G kr[3];   // k r_exit (lab)
  G dir[3];  // the stored exit direction (as in Records::dir)
  G f[8];    // [pol][e_theta|e_phi][re|im]: field amp e^{i phase} (J_perp e_perp + J_par e_par)
  RecTail<G> tail;
};
static_assert(sizeof(RayRec<float>) == 64 && sizeof(RayRec<double>) == 128, "record sizes");

// (e_theta, e_phi) of a direction d (not necessarily of unit length, as
// stored): with rho = |(dx, dy)|, cos phi = dx / rho, sin phi = dy / rho
// (phi = 0 on the axis), e_theta = (dz cos phi, dz sin phi, -rho) and
// e_phi = (-sin phi, cos phi, 0).  1 / rho from the reciprocal square root
// (rsq_d: about one ulp).  Both the writer and the reader of a record evaluate
// it in FP64 from the same stored direction, so they agree exactly.
__device__ __forceinline__ void dir_basis(double dx, double dy, double dz, v3<double>& et, v3<double>& ep) {
  const double rho2 = dx * dx + dy * dy;
  double cp = 1.0, sp = 0.0, rho = 0.0;
  if (rho2 > 1e-300) {
    const double r = rsq_d(rho2);
    cp = dx * r;
    sp = dy * r;
    rho = rho2 * r;
  }
  et = mk3<double>(dz * cp, dz * sp, -rho);
  ep = mk3<double>(-sp, cp, 0.0);
}

template <typename G>
struct alignas(4 * sizeof(G)) Dir4 {
  G x, y, z, pad;
};

// Emission records of the particles of one chunk: particle p owns the index
// range [n_ord (ray_off[p] - ray_base), ... + n_ord N_p^2), laid out
// [order slot][ray], so that record (p, slot, ray) is at rb(p, slot) + ray.
template <typename G>
struct Records {
  int32_t* flags;  // bit0 valid, bits 1..7 nf, bit 8 det_neg
  RayRec<G>* rr;
  Dir4<G>* dir;    // exit direction
  float2* ang;     // (theta, phi) of the exit direction (rad), phi in [0, 2 pi)
  int n_pol;
  unsigned* n_fp64;  // rays listed for the FP64 re-trace (mixed path)
  int* redo_list;    // their chunk ray indices
  double* ph64;      // caustic correction only (else NULL): unreduced FP64 phase at the stored direction
};

// The particles of one launch (a chunk of a batch, or one particle).  Offsets
// are prefix sums over the whole batch in batch-launch order; subtracting the
// chunk's base gives chunk-local values.
struct BatchDev {
  int n;                    // particles in the chunk
  int n_ord;                // orders p_min..p_max
  const ParticleConst* P;   // [n]
  const long* ray_off;      // [n + 1] first incident ray of each particle (N^2 rays each)
  const long* quad_off;     // [n + 1] first grid quad ((N - 1)^2 quads each)
  const long* tile_off;     // [n + 1] first trace work item (ceil(N^2 / tile) each)
  const int* out_index;     // [n] position of each particle in the caller's output
  long ray_base, quad_base, tile_base;
  int tile;                 // incident rays per trace work item
};

// Largest p in [0, n) with off[p] - base <= x (off non-decreasing, x >= 0).
__device__ __forceinline__ int find_part(const long* off, int n, long base, long x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] - base <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// A node hit found by the rasteriser, waiting for k_store_hits: which
// triangle (record base, corner ray, grid side, half, key), which node, and
// the barycentric weights.
// Four values loaded or stored at once (the alignment makes it one vector access).
template <typename G>
struct alignas(4 * sizeof(G)) V4 {
  G x, y, z, w;
};

template <typename G>
struct HitDesc {
  int key;    // 2 (n_ord quad_off + slot (N-1)^2 + quad) + t: also gives the triangle's rays
  int nt;     // t | N << 1 | chunk particle << 16
  int itip;   // node row | node column << 16
  int node;   // node index within the chunk (particle-major)
  int rank;   // place among the node's hits (taken with the node's count, before the pool slot)
  G lam[3];
};

template <typename G>
struct HitPool {
  int* count;         // [n_nodes] hits of each node (counted by the rasterisers)
  int* cursor;        // [n_nodes] exclusive prefix of count: the start of each node's range
  int* key;           // [cap] triangle key of each stored contribution (node-major order)
  G* contrib;         // [cap][n_pol * 4]: (pol, theta|phi, re|im), node-major order
  HitDesc<G>* desc;   // [cap] hits found, stored by k_store_hits
  unsigned* counter;  // [NPART]
  int cap_part;       // capacity of each partition
  int2* rows;         // [rows_cap] (triangle key, theta row) of triangles rasterised row by row
  unsigned* n_rows;   // rows listed
  int rows_cap;
  double* phi;        // caustic correction only (else NULL): [cap] phase carried to the node
  int* nf;            // [cap] focal-line count of the contribution's triangle
};

constexpr int CAND_INLINE = 4096;  // default: triangles with more box candidates go to the row list
// (draining large boxes inline spreads them over the rasteriser's many waves;
// the row kernel only serves boxes beyond this, e.g. triangles holding a pole)
// Angular margin (rad) of the FP32 bounding box: well above its rounding error,
// so the box never excludes a node that the exact membership test accepts.
constexpr double BOX_MARGIN = 4e-6;

__device__ __forceinline__ void set_tail(RecTail<double>& t, const v3<double>&, const Dir4<double>&) {
  t.pad[0] = t.pad[1] = 0.0;
}
__device__ __forceinline__ void set_tail(RecTail<float>& t, const v3<double>& d, const Dir4<float>& dv) {
  const double q[3] = {rint((d.x - (double)dv.x) * DLO_SCALE), rint((d.y - (double)dv.y) * DLO_SCALE),
                       rint((d.z - (double)dv.z) * DLO_SCALE)};
#pragma unroll
  for (int i = 0; i < 3; ++i) t.dlo[i] = (int16_t)fmin(32767.0, fmax(-32767.0, q[i]));
  t.pad = 0;
}

// The compact record of one emission, as the rasteriser and the hit store
// read it (fields as RayRec and Records), built from an emission traced in E.
template <typename G>
struct RecVals {
  int flags;        // bit0 valid, bits 1..7 nf, bit 8 det_neg
  G kr[3], dir[3], f[8];
  RecTail<G> tail;
  float th, ph;     // (theta, phi) of the stored direction (rad), phi in [0, 2 pi)
  double ph64;      // the ray's unreduced FP64 phase at the stored direction
};

template <typename G, typename E>
__device__ __forceinline__ void record_values(const Emission<E>& e, double k, double kappa, int n_pol,
                                              RecVals<G>& r) {
  r.flags = 1 | (e.nf << 1) | (e.det_neg << 8);
  Dir4<G> dv;
  dv.x = (G)e.obs.x; dv.y = (G)e.obs.y; dv.z = (G)e.obs.z; dv.pad = (G)0;
  r.kr[0] = (G)(k * e.rexit.x); r.kr[1] = (G)(k * e.rexit.y); r.kr[2] = (G)(k * e.rexit.z);
  // The field's phase contains -k dir.r_exit and the rasteriser carries it
  // with k r_exit.(dir - n) using the stored direction, so the two must use
  // the same direction.  An FP64 emission stored in FP32 records is turned
  // to the rounded direction: phase += k r_exit.(dir - (G)dir), in FP64
  // (k |r_exit| reaches 10^4 rad, the correction ~10^-4 rad).
  double cre = 1.0, cim = 0.0;
  r.ph64 = e.phase;
  if (sizeof(E) > sizeof(G)) {
    const double dphi = near_carry(kappa, k * e.rexit.x, k * e.rexit.y, k * e.rexit.z, (double)e.obs.x,
                                   (double)e.obs.y, (double)e.obs.z, (double)dv.x, (double)dv.y, (double)dv.z);
    sincos(dphi, &cim, &cre);
    r.ph64 = e.phase + dphi;
  }
  v3<double> et, ep;
  dir_basis((double)dv.x, (double)dv.y, (double)dv.z, et, ep);
  for (int p = 0; p < 2; ++p) {
    const double ar = (double)e.f[p][0].re * et.x + (double)e.f[p][1].re * et.y + (double)e.f[p][2].re * et.z;
    const double ai = (double)e.f[p][0].im * et.x + (double)e.f[p][1].im * et.y + (double)e.f[p][2].im * et.z;
    const double br = (double)e.f[p][0].re * ep.x + (double)e.f[p][1].re * ep.y;
    const double bi = (double)e.f[p][0].im * ep.x + (double)e.f[p][1].im * ep.y;
    const bool live = p < n_pol;
    r.f[p * 4 + 0] = live ? (G)(ar * cre - ai * cim) : (G)0;
    r.f[p * 4 + 1] = live ? (G)(ar * cim + ai * cre) : (G)0;
    r.f[p * 4 + 2] = live ? (G)(br * cre - bi * cim) : (G)0;
    r.f[p * 4 + 3] = live ? (G)(br * cim + bi * cre) : (G)0;
  }
  r.dir[0] = dv.x; r.dir[1] = dv.y; r.dir[2] = dv.z;
  set_tail(r.tail, e.obs64, dv);
  const float dx = (float)e.obs.x, dy = (float)e.obs.y, dz = (float)e.obs.z;
  float phi = atan2_f32(dy, dx);
  if (phi < 0.0f) phi += 6.28318531f;
  if (phi >= 6.28318531f) phi = 0.0f;
  r.th = atan2_f32(sqrtf(dx * dx + dy * dy), dz);
  r.ph = phi;
}

// Sink writing the compact emission records used by the rasteriser.  In the
// mixed path an emission whose divergence factor is ill-conditioned for FP32
// (amplif > amplif_limit) marks the ray for an FP64 re-trace.
template <typename G>
struct RecordSink {
  Records<G> rec;
  long base;  // record index of (this particle, slot 0, ray 0)
  long NN;    // rays of this particle
  long id;
  double k;
  double amplif_limit;
  bool need64;
  double kappa;  // k R at a finite observation radius, 0 in the far field
  template <typename E>
  __device__ void emit(const Emission<E>& e) {
    if (sizeof(E) == 4 && e.amplif > amplif_limit) need64 = true;
    const long at = base + e.slot * NN + id;
    RecVals<G> v;
    record_values(e, k, kappa, rec.n_pol, v);
    rec.flags[at] = v.flags;
    if (rec.ph64) rec.ph64[at] = v.ph64;
    RayRec<G> r;
    Dir4<G> dv;
    dv.x = v.dir[0]; dv.y = v.dir[1]; dv.z = v.dir[2]; dv.pad = (G)0;
    for (int i = 0; i < 3; ++i) { r.kr[i] = v.kr[i]; r.dir[i] = v.dir[i]; }
    for (int i = 0; i < 8; ++i) r.f[i] = v.f[i];
    r.tail = v.tail;
    rec.rr[at] = r;
    rec.dir[at] = dv;
    rec.ang[at] = make_float2(v.th, v.ph);
  }
};

__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float sub_rn(float a, float b) { return __fsub_rn(a, b); }
__device__ __forceinline__ double sub_rn(double a, double b) { return __dsub_rn(a, b); }

__host__ __device__ __forceinline__ int lower_idx(const double* v, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (v[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__host__ __device__ __forceinline__ int upper_idx(const double* v, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (v[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// First index with v[i] >= x (lower) or v[i] > x (upper), from the run table
// when there is one.  Both may err towards including one more node when x is
// within rounding of a node -- the callers only need a superset.
__host__ __device__ __forceinline__ int seg_lower(const AxisSeg* sg, const double* v, int n, double x) {
  const int ns = sg->nseg;
  if (ns == 0) return lower_idx(v, n, x);
  for (int k = 0; k < ns; ++k)
    if (x <= sg->vend[k]) {
      double f = (x - sg->v0[k]) * sg->inv_step[k];
      int i = sg->start[k] + (f <= 0.0 ? 0 : (int)ceil(f - 1e-9));
      return min(i, sg->end[k]);
    }
  return n;
}
__host__ __device__ __forceinline__ int seg_upper(const AxisSeg* sg, const double* v, int n, double x) {
  const int ns = sg->nseg;
  if (ns == 0) return upper_idx(v, n, x);
  for (int k = 0; k < ns; ++k)
    if (x < sg->vend[k]) {
      double f = (x - sg->v0[k]) * sg->inv_step[k];
      int i = sg->start[k] + (f < 0.0 ? 0 : (int)floor(f + 1e-9) + 1);
      return min(i, sg->end[k] + 1);
    }
  return n;
}

// One uniformly spaced axis (a single run) in FP32 registers: the index of the
// first node >= x is ceil((x - v0) / step), of the last node <= x plus one
// floor((x - v0) / step) + 1, clamped to [0, n].  FP32 misplaces a bound by
// at most ~4e-7 rad on the finest grids used here (0.02 deg), a tenth of the
// box margin, so a node it adds or drops lies outside the triangle anyway;
// 1e-3 index units of slack are added on both sides regardless.
struct AxisFast {
  int uni;  // the axis is one uniform run (else the segment tables are used)
  int n;
  float v0, inv_step;
};

__device__ __forceinline__ AxisFast axis_fast(const AxisSeg* sg, int n) {
  AxisFast a;
  a.uni = sg->nseg == 1 && sg->start[0] == 0 && sg->end[0] == n - 1;
  a.n = n;
  a.v0 = (float)sg->v0[0];
  a.inv_step = (float)sg->inv_step[0];
  return a;
}

__device__ __forceinline__ int fast_lower(const AxisFast& a, float x) {
  const float f = (x - a.v0) * a.inv_step;
  const int i = f <= 0.0f ? 0 : (int)ceilf(f - 1e-3f);
  return min(i, a.n);
}

__device__ __forceinline__ int fast_upper(const AxisFast& a, float x) {
  const float f = (x - a.v0) * a.inv_step;
  const int i = f < 0.0f ? 0 : (int)floorf(f + 1e-3f) + 1;
  return min(i, a.n);
}

// Candidate node set of one triangle: rows [i0, i1) x (phi segment a  U  segment b).
struct Cand {
  int i0, i1, ja0, ja1, jb0, jb1;
  __device__ int len() const { return (ja1 - ja0) + (jb1 - jb0); }
  __device__ int count() const { return (i1 - i0) * len(); }
};

// Angular bounding box: colatitudes [tlo, thi] (rad) x longitudes [plo, phi]
// (0 <= plo < 2 pi, phi - plo < 2 pi) or every longitude (full).
struct Box {
  float tlo, thi;
  double plo, phi;
  bool full;
};

// Node index ranges [j0, j1) of the phi list inside the absolute interval
// [lo, hi] (length < 2 pi, possibly wrapping): up to two ranges.
__device__ inline int phi_ranges(const NodeGrid& ng, double lo, double hi, int* j0, int* j1) {
  const double TWO_PI = 6.283185307179586;
  if (hi - lo >= TWO_PI) { j0[0] = 0; j1[0] = ng.n_phi; return 1; }
  double l = fmod(lo, TWO_PI);
  if (l < 0) l += TWO_PI;
  double h = l + (hi - lo);
  if (h < TWO_PI) {
    j0[0] = seg_lower(ng.seg_p, ng.ph, ng.n_phi, l); j1[0] = seg_upper(ng.seg_p, ng.ph, ng.n_phi, h);
    return 1;
  }
  j0[0] = seg_lower(ng.seg_p, ng.ph, ng.n_phi, l); j1[0] = ng.n_phi;
  j0[1] = 0; j1[1] = seg_upper(ng.seg_p, ng.ph, ng.n_phi, h - TWO_PI);
  return 2;
}

template <typename G>
__device__ __forceinline__ v3<G> load_dir(const Records<G>& rec, long at) {
  const Dir4<G> d = rec.dir[at];
  return mk3<G>(d.x, d.y, d.z);
}

// One triangle of one order of one particle, as the rasteriser needs it.
template <typename G>
struct Tri {
  long vid[3];  // ray ids (within the particle) in triangle order
  v3<G> dv[3];  // stored exit directions
  int sig[3];   // +1 if edge e (cyclic, opposite vertex e) runs from the lower ray id
  int orient;   // sign of the triple product of the directions
  v3<G> m[3];   // canonical edge normals d_lo x d_hi of the edges opposite each vertex
  long rb;      // record index of (particle, order slot, ray 0)
  int part;     // particle within the chunk (selects its nodes)
  int N;        // rays per side of the particle
  int key;      // 2 (n_ord quad_off + slot (N-1)^2 + quad) + t: the per-node summation order
};

// Key of triangle t of quad `quad` of order slot `slot` of a particle whose
// quads start at chunk quad qoff: unique within the chunk, increasing in
// (slot, quad, t) within a particle.
__device__ __forceinline__ int tri_key(int n_ord, long qoff, int slot, long nq, long quad, int t) {
  return (int)((n_ord * qoff + (long)slot * nq + quad) * 2 + t);
}

template <typename G>
__device__ inline void tri_load(const Records<G>& rec, long rb, int N, long quad, int t, int key, int part,
                                Tri<G>& T) {
  const int Nq = N - 1;
  const int iy = div_quot15((int)quad, Nq), ix = (int)quad - iy * Nq;
  const long v00 = (long)iy * N + ix;
  T.vid[0] = v00;
  T.vid[1] = t == 0 ? v00 + 1 : v00 + N + 1;
  T.vid[2] = t == 0 ? v00 + N + 1 : v00 + N;
  for (int k = 0; k < 3; ++k) T.dv[k] = load_dir(rec, rb + T.vid[k]);
  T.rb = rb;
  T.part = part;
  T.N = N;
  T.key = key;
  // orientation from the FP64 triple product (d1 - d0) x (d2 - d0) . d0 of the
  // stored directions (their differences are exact in FP64)
  v3<double> e1 = mk3<double>((double)T.dv[1].x - (double)T.dv[0].x, (double)T.dv[1].y - (double)T.dv[0].y,
                              (double)T.dv[1].z - (double)T.dv[0].z);
  v3<double> e2 = mk3<double>((double)T.dv[2].x - (double)T.dv[0].x, (double)T.dv[2].y - (double)T.dv[0].y,
                              (double)T.dv[2].z - (double)T.dv[0].z);
  double vol = dot(cross(e1, e2), cvt<double>(T.dv[0]));
  T.orient = vol > 0.0 ? 1 : (vol < 0.0 ? -1 : 0);
  for (int e = 0; e < 3; ++e) T.sig[e] = T.vid[(e + 1) % 3] < T.vid[(e + 2) % 3] ? 1 : -1;
}

// Bounding (theta, phi) box of the spherical triangle, in FP32 with an angular
// margin (it only prunes; membership is decided exactly).  Longitude is
// monotonic along a great-circle arc that avoids the poles, so without a pole
// inside, the phi extent is the shortest circular interval holding the three
// vertex longitudes; theta is extremal at a vertex or at an edge's closest
// approach to a pole.  A triangle holding a pole spans every phi.
template <typename G>
__device__ inline Box tri_box(const Tri<G>& T, float margin) {
  const float PI_F = 3.14159265f, TWO_PI_F = 6.2831853f;
  const double TWO_PI = 6.283185307179586;
  v3<float> u[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const v3<float> dd = cvt<float>(T.dv[k]);
    u[k] = scl(rsqrtf(dot(dd, dd)), dd);
  }
  float tmin = PI_F, tmax = 0.0f;
  float ph[3];
  bool has_n = true, has_s = true;  // triangle contains the north / south pole
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float rho = sqrtf(u[k].x * u[k].x + u[k].y * u[k].y);
    const float th = atan2f(rho, u[k].z);
    tmin = fminf(tmin, th);
    tmax = fmaxf(tmax, th);
    float p = atan2f(u[k].y, u[k].x);
    ph[k] = p < 0.0f ? p + TWO_PI_F : p;
    // edge opposite vertex k, cyclic order: m = d_a x d_b, inside is o m.n >= 0.
    // m is formed in FP64 from the stored directions (products of FP32 values
    // are exact there), so the pole tests and the edge's closest approach to
    // a pole stay accurate for very short edges too.
    const v3<double> da = cvt<double>(T.dv[(k + 1) % 3]), db = cvt<double>(T.dv[(k + 2) % 3]);
    const v3<double> m64 = cross(da, db);
    const double mz = (double)T.orient * m64.z;
    has_n = has_n && (mz >= 0.0);
    has_s = has_s && (mz <= 0.0);
    const double mm = dot(m64, m64);
    if (mm > 0.0) {
      const v3<float> mh = cvt<float>(scl(rsqrt(mm), m64));
      const v3<float>& ua = u[(k + 1) % 3];
      const v3<float>& ub = u[(k + 2) % 3];
      // closest point of the edge's great circle to the north pole: z - (z.mh) mh
      const float rz = sqrtf(fmaxf(0.0f, 1.0f - mh.z * mh.z));
      if (rz > 1e-20f) {
        const v3<float> pz = mk3<float>(-mh.z * mh.x / rz, -mh.z * mh.y / rz, rz);
        // on the arc from ua to ub?  (ua x p) and (p x ub) both along m
        const bool on_n = dot(cross(ua, pz), mh) >= 0.0f && dot(cross(pz, ub), mh) >= 0.0f;
        const v3<float> ps = scl(-1.0f, pz);
        const bool on_s = dot(cross(ua, ps), mh) >= 0.0f && dot(cross(ps, ub), mh) >= 0.0f;
        const float thp = asinf(fminf(1.0f, fabsf(mh.z)));  // pole distance of the great circle
        if (on_n) tmin = fminf(tmin, thp);
        if (on_s) tmax = fmaxf(tmax, PI_F - thp);
      }
    }
  }
  if (has_n) tmin = 0.0f;
  if (has_s) tmax = PI_F;
  Box bx;
  bx.tlo = tmin - margin;
  bx.thi = tmax + margin;
  bx.full = true;
  bx.plo = 0.0;
  bx.phi = TWO_PI;
  if (has_n || has_s || bx.tlo <= 1e-3f || bx.thi >= PI_F - 1e-3f) return bx;
  const float sden = fminf(sinf(bx.tlo), sinf(bx.thi));
  // shortest circular interval holding the three longitudes
  float a0 = ph[0], a1 = ph[1], a2 = ph[2], t;
  if (a0 > a1) { t = a0; a0 = a1; a1 = t; }
  if (a1 > a2) { t = a1; a1 = a2; a2 = t; }
  if (a0 > a1) { t = a0; a0 = a1; a1 = t; }
  const float g01 = a1 - a0, g12 = a2 - a1, g20 = a0 + TWO_PI_F - a2;
  float lo_f, hi_f;
  if (g20 >= g01 && g20 >= g12) { lo_f = a0; hi_f = a2; }
  else if (g01 >= g12) { lo_f = a1; hi_f = a0 + TWO_PI_F; }
  else { lo_f = a2; hi_f = a1 + TWO_PI_F; }
  const double pm = (double)margin / (double)sden + 1e-6;
  const double lo = (double)lo_f - pm, hi = (double)hi_f + pm;
  if (hi - lo >= TWO_PI) return bx;
  bx.full = false;
  bx.plo = lo < 0.0 ? lo + TWO_PI : lo;
  bx.phi = bx.plo + (hi - lo);
  return bx;
}

// Node index ranges of a box: rows [i0, i1) x the phi ranges of [plo, phi].
__device__ inline Cand box_cand(const NodeGrid& ng, const Box& bx) {
  const double TWO_PI = 6.283185307179586;
  Cand cd;
  cd.ja0 = cd.ja1 = cd.jb0 = cd.jb1 = 0;
  cd.i0 = seg_lower(ng.seg_t, ng.th, ng.n_theta, (double)bx.tlo);
  cd.i1 = seg_upper(ng.seg_t, ng.th, ng.n_theta, (double)bx.thi);
  if (cd.i1 <= cd.i0) return cd;  // no node row crosses the box
  if (bx.full) { cd.ja1 = ng.n_phi; return cd; }
  if (bx.phi < TWO_PI) {
    cd.ja0 = seg_lower(ng.seg_p, ng.ph, ng.n_phi, bx.plo);
    cd.ja1 = seg_upper(ng.seg_p, ng.ph, ng.n_phi, bx.phi);
  } else {
    cd.ja0 = seg_lower(ng.seg_p, ng.ph, ng.n_phi, bx.plo); cd.ja1 = ng.n_phi;
    cd.jb0 = 0; cd.jb1 = seg_upper(ng.seg_p, ng.ph, ng.n_phi, bx.phi - TWO_PI);
  }
  return cd;
}

// Bounding box of a small triangle away from the poles from its vertices'
// (theta, phi) alone (no directions needed).  Returns false when the triangle
// is too large or too close to a pole for the bounds below; tri_box decides
// those.  With l the longest edge (l^2 <= 1.1 q, q from the angle
// differences and sin theta <= s_hi):
//   - every point of the triangle lies within l of each vertex, so a pole
//     farther than l from the nearest vertex is outside;
//   - along a great-circle arc of length l, cos theta exceeds its end values
//     by at most l^2 / 8, so theta leaves the vertex range by at most
//     l^2 / (8 sin theta) (bounded here by 0.132 q / s_lo, s_lo <= sin theta;
//     on random and near-pole east-west arcs the true excursion stays below
//     0.55 of it); the theta range is widened by that bound, capped at
//     1e-3 rad;
//   - longitude is monotonic along pole-free arcs: the phi extent is the
//     shortest circular interval holding the three vertex longitudes.
__device__ inline bool fast_box(const NodeGrid& ng, const AxisFast& at, const AxisFast& ap, float2 a, float2 b,
                                float2 c, float margin, Cand& cd) {
  const float PI_F = 3.14159265f, TWO_PI_F = 6.2831853f;
  const float tmin = fminf(a.x, fminf(b.x, c.x)), tmax = fmaxf(a.x, fmaxf(b.x, c.x));
  const float s_hi = fminf(1.0f, fminf(tmax, PI_F - tmin));
  auto dp = [&](float p, float q) { const float d = fabsf(p - q); return fminf(d, TWO_PI_F - d); };
  auto e2 = [&](float2 u, float2 v) {
    const float dt = u.x - v.x, dph = dp(u.y, v.y) * s_hi;
    return dt * dt + dph * dph;
  };
  const float q = 1.1f * fmaxf(e2(a, b), fmaxf(e2(b, c), e2(c, a)));
  if (!(q < 1e-2f)) return false;
  // bounds only: the hardware square root and reciprocal (1 ulp) with a
  // 1e-4 relative allowance in the safe direction
  const float l = __builtin_amdgcn_sqrtf(q) * 1.0001f;
  const float pole_gap = fminf(tmin, PI_F - tmax) - l;  // lower bound of the pole distance of any point
  if (!(pole_gap > 2.0f * margin + 1e-3f)) return false;
  const float s_lo = 0.63661977f * pole_gap;  // sin x >= 2x / pi on [0, pi/2]
  const float bulge = 0.132f * q * __builtin_amdgcn_rcpf(s_lo) * 1.0001f;
  if (!(bulge <= 1e-3f)) return false;
  const float m = margin + 2e-6f;
  const float tlo = tmin - m - bulge, thi = tmax + m + bulge;
  cd.ja0 = cd.ja1 = cd.jb0 = cd.jb1 = 0;
  if (at.uni) {
    cd.i0 = fast_lower(at, tlo);
    cd.i1 = fast_upper(at, thi);
  } else {
    cd.i0 = seg_lower(ng.seg_t, ng.th, ng.n_theta, (double)tlo);
    cd.i1 = seg_upper(ng.seg_t, ng.th, ng.n_theta, (double)thi);
  }
  if (cd.i1 <= cd.i0) return true;  // no node row crosses the triangle: nothing else to do
  float a0 = a.y, a1 = b.y, a2 = c.y, t;
  if (a0 > a1) { t = a0; a0 = a1; a1 = t; }
  if (a1 > a2) { t = a1; a1 = a2; a2 = t; }
  if (a0 > a1) { t = a0; a0 = a1; a1 = t; }
  const float g01 = a1 - a0, g12 = a2 - a1, g20 = a0 + TWO_PI_F - a2;
  float lo_f, hi_f;
  if (g20 >= g01 && g20 >= g12) { lo_f = a0; hi_f = a2; }
  else if (g01 >= g12) { lo_f = a1; hi_f = a0 + TWO_PI_F; }
  else { lo_f = a2; hi_f = a1 + TWO_PI_F; }
  // phi margin: m / sin(theta) over the box, with sin bounded below by 2 theta / pi
  const float pm = m * __builtin_amdgcn_rcpf(0.63661977f * fminf(tlo, PI_F - thi)) * 1.0002f + 1e-6f;
  if (ap.uni) {  // FP32 throughout: its ~5e-7 rad error is a fraction of the margin
    const float lo = lo_f - pm, hi = hi_f + pm;
    if (hi - lo >= TWO_PI_F) return false;
    const float plo = lo < 0.0f ? lo + TWO_PI_F : lo, phi = plo + (hi - lo);
    cd.ja0 = fast_lower(ap, plo);
    if (phi < TWO_PI_F) {
      cd.ja1 = fast_upper(ap, phi);
    } else {
      cd.ja1 = ng.n_phi;
      cd.jb0 = 0; cd.jb1 = fast_upper(ap, phi - TWO_PI_F);
    }
    return true;
  }
  const double TWO_PI = 6.283185307179586;
  const double lo = (double)lo_f - (double)pm, hi = (double)hi_f + (double)pm;
  if (hi - lo >= TWO_PI) return false;
  const double plo = lo < 0.0 ? lo + TWO_PI : lo, phi = plo + (hi - lo);
  if (phi < TWO_PI) {
    cd.ja0 = seg_lower(ng.seg_p, ng.ph, ng.n_phi, plo);
    cd.ja1 = seg_upper(ng.seg_p, ng.ph, ng.n_phi, phi);
  } else {
    cd.ja0 = seg_lower(ng.seg_p, ng.ph, ng.n_phi, plo); cd.ja1 = ng.n_phi;
    cd.jb0 = 0; cd.jb1 = seg_upper(ng.seg_p, ng.ph, ng.n_phi, phi - TWO_PI);
  }
  return true;
}

// Longitude window of the triangle on one node row (colatitude theta_r, given
// as sr = sin theta_r, cr = cos theta_r; sm = sin margin): the
// box window with every part removed that lies more than `margin` outside one
// of the three edge hemispheres o (d_a x d_b).x >= 0.  On the row circle, the
// points outside an edge form one arc (a "hole") centred opposite the edge
// normal's longitude; holes are cut from the window's ends, which keeps the
// window a single interval holding the triangle's part of the row.  FP64,
// because near-tangent rows make the hole ends ill-conditioned.
template <typename G>
__device__ inline bool row_window(const Tri<G>& T, const Box& bx, double sr, double cr, double sm, double& lo,
                                  double& hi) {
  const double TWO_PI = 6.283185307179586, PI = 3.141592653589793;
  lo = bx.plo;
  hi = bx.phi;
  bool full = bx.full;
  double hc[3], hw[3];
  bool has[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const v3<double> da = cvt<double>(T.dv[(k + 1) % 3]), db = cvt<double>(T.dv[(k + 2) % 3]);
    v3<double> m = scl((double)T.orient, cross(da, db));
    const double mm = dot(m, m);
    has[k] = false;
    hc[k] = 0.0;
    hw[k] = 0.0;
    if (!(mm > 0.0)) continue;
    m = scl(rsqrt(mm), m);
    const double R = sqrt(m.x * m.x + m.y * m.y);
    // outside by more than the margin:  R sr cos(phi - phi0) + m.z cr < -sin(margin)
    const double rhs = -m.z * cr - sm;
    if (R * sr <= 1e-300) {
      if (rhs > 0.0) return false;  // the whole row is outside this edge
      continue;
    }
    const double th = rhs / (R * sr);
    if (th <= -1.0) continue;     // no point of the row is outside
    if (th >= 1.0) return false;  // every point of the row is outside
    has[k] = true;
    hc[k] = atan2(m.y, m.x) + PI;  // hole centre
    hw[k] = PI - acos(th);         // hole half-width
  }
  // cut holes from the window ends (two passes: a cut can expose another hole)
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (!has[k]) continue;
      if (full) {
        lo = hc[k] + hw[k];
        hi = hc[k] + TWO_PI - hw[k];
        full = false;
        continue;
      }
      double d = remainder(lo - hc[k], TWO_PI);
      if (fabs(d) < hw[k]) lo += hw[k] - d;
      d = remainder(hi - hc[k], TWO_PI);
      if (fabs(d) < hw[k]) hi -= hw[k] + d;
      if (hi <= lo) return false;
    }
  }
  if (full) { lo = 0.0; hi = TWO_PI; }
  lo = fmod(lo, TWO_PI);
  if (lo < 0.0) lo += TWO_PI;
  hi = lo + fmin(hi - lo, TWO_PI);
  return true;
}

// Canonical edge normals: for the edge opposite vertex k, m_k = d_lo x d_hi
// with lo/hi its endpoint of lower/higher ray id, formed in FP64 from the
// stored directions and rounded to G.  The neighbouring triangle across the
// edge forms the same vector bit for bit, so both evaluate the same edge
// function m_k . n at every node: membership is watertight.
template <typename G>
__device__ __forceinline__ void edge_normals(Tri<G>& T) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const v3<G>& a = T.dv[(k + 1) % 3];
    const v3<G>& b = T.dv[(k + 2) % 3];
    const v3<double> lo = cvt<double>(T.sig[k] > 0 ? a : b), hi = cvt<double>(T.sig[k] > 0 ? b : a);
    T.m[k] = cvt<G>(cross(lo, hi));
  }
}

// m . n as a fixed sequence of correctly rounded operations.
template <typename T>
__device__ __forceinline__ T dot_rn(const v3<T>& m, const v3<T>& n) {
  return add_rn(add_rn(mul_rn(m.x, n.x), mul_rn(m.y, n.y)), mul_rn(m.z, n.z));
}

// Membership of node direction n (watertight canonical-edge rule) and its
// barycentric weights: the central-projection weights are proportional to
// the triple products (d_a x d_b) . n of the cyclic edges.
template <typename G>
__device__ __forceinline__ bool tri_member(const Tri<G>& T, const v3<G>& n, G lam[3]) {
  const int o = T.orient;
  const G e0 = dot_rn(T.m[0], n), e1 = dot_rn(T.m[1], n), e2 = dot_rn(T.m[2], n);
  const G w0 = T.sig[0] > 0 ? e0 : -e0, w1 = T.sig[1] > 0 ? e1 : -e1, w2 = T.sig[2] > 0 ? e2 : -e2;
  const bool ok0 = (o > 0 ? w0 > 0 : w0 < 0) || (e0 == 0 && T.sig[0] * o > 0);
  const bool ok1 = (o > 0 ? w1 > 0 : w1 < 0) || (e1 == 0 && T.sig[1] * o > 0);
  const bool ok2 = (o > 0 ? w2 > 0 : w2 < 0) || (e2 == 0 && T.sig[2] * o > 0);
  if (!(ok0 && ok1 && ok2)) return false;
  const G sw = 1 / (w0 + w1 + w2);
  lam[0] = w0 * sw; lam[1] = w1 * sw; lam[2] = w2 * sw;
  return true;
}

// Unit direction of node (it, ip), FP64, and in the rasteriser's precision
// (the FP32 tables give the mixed path's membership tests).
__device__ __forceinline__ v3<double> node_dir(const NodeGrid& ng, int it, int ip) {
  return mk3<double>(ng.sth[it] * ng.cph[ip], ng.sth[it] * ng.sph[ip], ng.cth[it]);
}
template <typename G>
__device__ __forceinline__ v3<G> node_dir_g(const NodeGrid& ng, int it, int ip);
template <>
__device__ __forceinline__ v3<double> node_dir_g<double>(const NodeGrid& ng, int it, int ip) {
  return node_dir(ng, it, ip);
}
template <>
__device__ __forceinline__ v3<float> node_dir_g<float>(const NodeGrid& ng, int it, int ip) {
  const float st = ng.sthf[it];
  return mk3<float>(st * ng.cphf[ip], st * ng.sphf[ip], ng.cthf[it]);
}

// The FP64 node-space direction of a record: for FP32 records the stored
// direction plus its rounding residual.
__device__ __forceinline__ v3<double> full_dir(const RayRec<double>& r) { return mk3(r.dir[0], r.dir[1], r.dir[2]); }
__device__ __forceinline__ v3<double> full_dir(const RayRec<float>& r) {
  const double s = 1.0 / DLO_SCALE;
  return mk3((double)r.dir[0] + (double)r.tail.dlo[0] * s, (double)r.dir[1] + (double)r.tail.dlo[1] * s,
             (double)r.dir[2] + (double)r.tail.dlo[2] * s);
}

// Contribution of a triangle (vertex records v[0..2], in triangle order) to
// node (it, ip): sum_v lambda_v F_v exp(i k r_v.(d_v - n)) on the node's
// (e_theta, e_phi), accumulated into acc[pol][theta|phi][re|im].  lam: the
// weights of the membership test; an FP32 record set recomputes them in FP64
// from the directions plus their residuals.  With_phase: phi_t receives the
// triangle's phase carried to the node, from the vertices' FP64 phases ph64.
template <typename G, typename R>
__device__ __forceinline__ void hit_contrib(const R& v0, const R& v1, const R& v2, const NodeGrid& ng, int it,
                                            int ip, int n_pol, const G lam_in[3], G acc[2][2][2], bool with_phase,
                                            double ph0, double ph1, double ph2, double& phi_t) {

  const double st = ng.sth[it], ct = ng.cth[it], sp = ng.sph[ip], cp = ng.cph[ip];
  const v3<double> eth = mk3<double>(ct * cp, ct * sp, -st);
  const v3<double> eph = mk3<double>(-sp, cp, 0.0);
  for (int p = 0; p < 2; ++p)
    for (int a = 0; a < 2; ++a) acc[p][a][0] = acc[p][a][1] = 0;
  const v3<double> n = node_dir(ng, it, ip);
  G lam[3] = {lam_in[0], lam_in[1], lam_in[2]};
  double lam64[3] = {(double)lam_in[0], (double)lam_in[1], (double)lam_in[2]};
  if (sizeof(G) == 4) {
    // weights of the central projection from the FP64 vertex directions
    // (stored direction plus its rounding residual): (d_a x d_b).n over the
    // cyclic edges, normalised
    v3<double> dd[3];
    dd[0] = full_dir(v0);
    dd[1] = full_dir(v1);
    dd[2] = full_dir(v2);
    const double w0 = dot(cross(dd[1], dd[2]), n), w1 = dot(cross(dd[2], dd[0]), n), w2 = dot(cross(dd[0], dd[1]), n);
    const double sw = w0 + w1 + w2;
    if (sw != 0.0) {
      const double is = 1.0 / sw;
      lam64[0] = w0 * is; lam64[1] = w1 * is; lam64[2] = w2 * is;
      lam[0] = (G)lam64[0]; lam[1] = (G)lam64[1]; lam[2] = (G)lam64[2];
    }
  }
  double ph = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R& vr = k == 0 ? v0 : (k == 1 ? v1 : v2);
    const double lk = k == 0 ? lam64[0] : (k == 1 ? lam64[1] : lam64[2]);
    const G lkg = k == 0 ? lam[0] : (k == 1 ? lam[1] : lam[2]);
    const G dkx = vr.dir[0], dky = vr.dir[1], dkz = vr.dir[2];
    // carried phase k r.(d - n) in FP64: for large particles k |r| reaches
    // 10^4 and the product tens of radians, beyond FP32's absolute accuracy
    const double psi = near_carry(ng.kappa, (double)vr.kr[0], (double)vr.kr[1], (double)vr.kr[2], (double)dkx,
                                  (double)dky, (double)dkz, n.x, n.y, n.z);
    if (with_phase) ph += lk * ((k == 0 ? ph0 : (k == 1 ? ph1 : ph2)) + psi);
    G s_, c_;
    if (sizeof(G) == 8) sincos_t((G)psi, &s_, &c_);
    else sincos_red((G)(psi - 6.283185307179586 * rint(psi * 0.15915494309189535)), &s_, &c_);
    const G lr = lkg * c_, li = lkg * s_;
    // the vertex field is stored on its direction's (e_theta, e_phi); turn it
    // onto the node's
    v3<double> et, ep;
    dir_basis((double)dkx, (double)dky, (double)dkz, et, ep);
    const G ctt = (G)dot(et, eth), cpt = (G)dot(ep, eth), ctp = (G)dot(et, eph), cpp = (G)dot(ep, eph);
    const G* fp = vr.f;
    for (int p = 0; p < n_pol; ++p) {
      const G ar = fp[p * 4 + 0], ai = fp[p * 4 + 1], br = fp[p * 4 + 2], bi = fp[p * 4 + 3];
      const G tr = ar * ctt + br * cpt, ti = ai * ctt + bi * cpt;
      const G pr = ar * ctp + br * cpp, pi_ = ai * ctp + bi * cpp;
      acc[p][0][0] += lr * tr - li * ti;  acc[p][0][1] += lr * ti + li * tr;
      acc[p][1][0] += lr * pr - li * pi_; acc[p][1][1] += lr * pi_ + li * pr;
    }
  }
  phi_t = ph;
}

// Contribution of the hit in pool slot idx (its descriptor), stored at its
// place in its node's range (node-major order): the range start from the
// scan plus the rank the rasteriser took with the node's count, so this
// kernel needs no atomic.
template <typename G>
__device__ inline void store_hit(const BatchDev& B, const Records<G>& rec, const NodeGrid& ng, const HitPool<G>& pool,
                                 long idx) {
  const HitDesc<G> d = pool.desc[idx];
  const long at = (long)pool.cursor[d.node] + d.rank;
  // after an overflow the node counts include hits the pool could not keep,
  // so a place can fall outside the pool (the result is reported incomplete)
  if (at < 0 || at >= (long)NPART * pool.cap_part) return;
  const int it = d.itip & 0xffff, ip = (int)((unsigned)d.itip >> 16);
  const int t = d.nt & 1, N = (d.nt >> 1) & 0x7fff, part = (int)((unsigned)d.nt >> 16);
  // the triangle's rays from its key: order slot, quad, corner ray
  const unsigned within = (unsigned)((long)(d.key >> 1) - (long)B.n_ord * (B.quad_off[part] - B.quad_base));
  const unsigned nq = (unsigned)(N - 1) * (unsigned)(N - 1);
  const unsigned slot = (unsigned)div_quot15((int)within, (int)nq), quad = within - slot * nq;
  const long v00 = (long)quad + div_quot15((int)quad, N - 1);
  const long rb = (long)B.n_ord * (B.ray_off[part] - B.ray_base) + (long)slot * N * N;
  const long vid[3] = {v00, t == 0 ? v00 + 1 : v00 + N + 1, t == 0 ? v00 + N + 1 : v00 + N};
  const bool with_phase = pool.phi != nullptr;
  G acc[2][2][2];
  double phi_t = 0.0;  // the triangle's phase carried to the node (caustic correction)
  hit_contrib<G>(rec.rr[rb + vid[0]], rec.rr[rb + vid[1]], rec.rr[rb + vid[2]], ng, it, ip, rec.n_pol, d.lam, acc,
                 with_phase, with_phase ? rec.ph64[rb + vid[0]] : 0.0, with_phase ? rec.ph64[rb + vid[1]] : 0.0,
                 with_phase ? rec.ph64[rb + vid[2]] : 0.0, phi_t);
  V4<G>* out = reinterpret_cast<V4<G>*>(pool.contrib + at * (rec.n_pol * 4));
  for (int p = 0; p < rec.n_pol; ++p) {
    V4<G> v4;
    v4.x = acc[p][0][0]; v4.y = acc[p][0][1]; v4.z = acc[p][1][0]; v4.w = acc[p][1][1];
    out[p] = v4;
  }
  pool.key[at] = d.key;
  if (pool.phi) {
    pool.phi[at] = phi_t;
    pool.nf[at] = (rec.flags[rb + vid[0]] >> 1) & 127;
  }
}

// One thread per pool slot: contributions of every hit the rasterisers found,
// placed node by node (slots past a partition's fill are idle).
template <typename G>
__global__ void __launch_bounds__(256) k_store_hits(const BatchDev B, const Records<G> rec, const NodeGrid ng,
                                                    const HitPool<G> pool) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long part = i / pool.cap_part;
  if (part >= NPART) return;
  const unsigned pos = (unsigned)(i - part * pool.cap_part);
  if (pos >= min(pool.counter[part], (unsigned)pool.cap_part)) return;
  store_hit(B, rec, ng, pool, i);
}

__device__ inline int wave_partition() {
  return (int)(((long)blockIdx.y * gridDim.x * (blockDim.x >> 6) + (long)blockIdx.x * (blockDim.x >> 6) +
                (threadIdx.x >> 6)) % NPART);
}

// A triangle staged in LDS for the flattened candidate loop (56 bytes in the
// mixed path, so that five blocks' stages fit a CU's LDS).  Its rays are not
// kept: the hit store derives them from the key.  Node-grid sides and chunk
// particle counts are below 2^16 (checked on the host), so index pairs share
// a word.
template <typename G>
struct TriSlot {
  G m[9];    // canonical edge normals (edge_normals)
  int meta;  // bit 0: t (which half of the quad), bit 1: orient > 0, bits 2..16: N
  int key;   // per-node summation order
  int pk0;   // i0 | len << 16: candidate rows start at i0; len candidates per row
  int pk1;   // ja0 | la << 16: phi range a = [ja0, ja0 + la)
  int pk2;   // jb0 | part << 16: phi range b starts at jb0 (len - la nodes); chunk particle
};

template <typename G>
__device__ __forceinline__ void slot_put(TriSlot<G>& S, Tri<G>& T, const Cand& cd) {
  edge_normals(T);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    S.m[3 * k] = T.m[k].x; S.m[3 * k + 1] = T.m[k].y; S.m[3 * k + 2] = T.m[k].z;
  }
  S.meta = (T.vid[1] == T.vid[0] + 1 ? 0 : 1) | (T.orient > 0 ? 2 : 0) | (T.N << 2);
  S.key = T.key;
  S.pk0 = cd.i0 | (cd.len() << 16);
  S.pk1 = cd.ja0 | ((cd.ja1 - cd.ja0) << 16);
  S.pk2 = cd.jb0 | (T.part << 16);
}

template <typename G>
__device__ __forceinline__ void slot_get(const TriSlot<G>& S, Tri<G>& T) {
#pragma unroll
  for (int k = 0; k < 3; ++k) T.m[k] = mk3<G>(S.m[3 * k], S.m[3 * k + 1], S.m[3 * k + 2]);
  const int t = S.meta & 1;
  const int N = (S.meta >> 2) & 0x7fff;
  // ray ids relative to the quad's corner: their order (all the tie rule
  // needs) is that of the absolute ids
  T.vid[0] = 0;
  T.vid[1] = t == 0 ? 1 : N + 1;
  T.vid[2] = t == 0 ? N + 1 : N;
  T.orient = (S.meta & 2) ? 1 : -1;
  T.N = N;
  T.rb = -1;
  T.part = (int)((unsigned)S.pk2 >> 16);
  T.key = S.key;
  for (int e = 0; e < 3; ++e) T.sig[e] = T.vid[(e + 1) % 3] < T.vid[(e + 2) % 3] ? 1 : -1;
}

// A triangle of the block that needs its directions loaded: its quad, particle,
// half (bit 0), whether the vertex-angle box applies (bit 1) and that box.
struct TriQueued {
  int quad, part, tf;
  int i0, i1, ja0, ja1, jb0, jb1;
};

// Per-wave LDS area of the row kernel: one staged (triangle, row) per lane.
constexpr int WAVE_SLOTS = 64;
template <typename G>
struct WaveStage {
  TriSlot<G> tri[WAVE_SLOTS];
  int excl[WAVE_SLOTS];  // exclusive prefix of the slots' candidate counts
};

// Per-block LDS area of the rasteriser: the triangles of the block's 256 quads
// that have candidates (at most two per quad), shared by its four waves; the
// queue of triangles to load shares the slot storage.  The mixed path stages
// all 512 at once; the FP64 path's slots are 96 bytes, so it stages and drains
// 256 at a time (five blocks per CU instead of three).
template <typename G>
struct BlockSlots {
  static constexpr int value = sizeof(G) == 8 ? 256 : 512;
  static constexpr int log2 = sizeof(G) == 8 ? 8 : 9;
};
template <typename G>
struct BlockStage {
  union {
    TriSlot<G> tri[BlockSlots<G>::value];
    TriQueued queued[512];
  };
  int excl[BlockSlots<G>::value];  // exclusive prefix of the slots' candidate counts (unused slots: the total)
  int wave_q[4];                   // queued triangles of each wave
};

// What the candidate loop needs of a stage: 2^log_slots slots with their
// exclusive candidate prefix.
template <typename G>
struct StageView {
  const TriSlot<G>* tri;
  const int* excl;
  int log_slots;
};

template <typename G>
__device__ __forceinline__ StageView<G> view(WaveStage<G>& W) {
  return StageView<G>{W.tri, W.excl, 6};
}

template <typename G>
__device__ __forceinline__ StageView<G> view(BlockStage<G>& S) {
  return StageView<G>{S.tri, S.excl, BlockSlots<G>::log2};
}

// Candidate g of the stage: its triangle and node (row it, column ip).
template <typename G>
__device__ __forceinline__ void locate(const StageView<G>& W, int g, Tri<G>& T, int& it, int& ip) {
  int L = 0;  // last slot whose prefix is <= g
  for (int step = 1 << (W.log_slots - 1); step > 0; step >>= 1)
    if (W.excl[L + step] <= g) L += step;
  const int c = g - W.excl[L];
  const TriSlot<G>& S = W.tri[L];
  const int i0 = S.pk0 & 0xffff, len = (int)((unsigned)S.pk0 >> 16);
  const int ja0 = S.pk1 & 0xffff, la = (int)((unsigned)S.pk1 >> 16), jb0 = S.pk2 & 0xffff;
  int row = (int)((float)c * __frcp_rn((float)len));  // c / len, then corrected
  if (row * len > c) --row;
  else if ((row + 1) * len <= c) ++row;
  const int jj = c - row * len;
  it = i0 + row;
  ip = jj < la ? ja0 + jj : jb0 + (jj - la);
  slot_get(S, T);
}

// Test every staged candidate, 64 per wave at a time: candidate g goes to a
// lane whatever triangle owns it, so one large triangle costs its size / 64
// iterations instead of its size.  Wave w of a group of n_waves takes g =
// base + 64 w + lane for base = 0, 64 n_waves, ...  The hits of one pass take
// their pool slots with one atomic and are written from registers: a
// descriptor each (triangle, node, barycentric weights; k_store_hits computes
// the contributions) and one count for the node.  Successive passes of a
// wave go to different pool partitions (97 is odd: every partition is
// reached).  The slots and the prefix must be written, and a barrier passed,
// before the call; the loop bound is uniform over the group.
template <typename G>
__device__ void raster_drain(const Records<G>& rec, const NodeGrid& ng, const HitPool<G>& pool,
                             const StageView<G>& W, int total, int wave_in_group, int n_waves, int part) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  int flushes = 0;
  const int stride = 64 * n_waves;
  for (int base = 0; base < total; base += stride) {
    const int g = base + 64 * wave_in_group + lane;
    bool hit = false;
    Tri<G> T;
    int it = 0, ip = 0;
    G lam[3];
    if (g < total) {
      locate(W, g, T, it, ip);
      hit = tri_member(T, node_dir_g<G>(ng, it, ip), lam);
    }
    const unsigned long long mask = __ballot(hit);
    if (mask == 0ull) continue;  // wave-uniform
    // the hit's rank among its node's hits first, so that the round trip of
    // that atomic overlaps the partition atomic's; a hit that then finds its
    // partition full stays counted (the pool has overflowed: the status call
    // reports it, and the consumers of the counts keep to the pool)
    int node = 0, rank = 0;
    if (hit) {
      node = (T.part * ng.n_theta + it) * ng.n_phi + ip;
      rank = atomicAdd(&pool.count[node], 1);
    }
    const int pt = (part + 97 * flushes) % NPART;
    ++flushes;
    const int leader = __ffsll((long long)mask) - 1;
    unsigned first = 0;
    if (lane == leader) first = atomicAdd(&pool.counter[pt], (unsigned)__popcll(mask));
    first = __shfl(first, leader);
    if (!hit) continue;
    const unsigned pos = first + (unsigned)__popcll(mask & below);
    if (pos < (unsigned)pool.cap_part) {  // beyond: overflow, reported by the status call
      HitDesc<G> d;
      d.key = T.key;
      d.nt = (T.vid[1] == T.vid[0] + 1 ? 0 : 1) | (T.N << 1) | (T.part << 16);
      d.itip = it | (ip << 16);
      d.node = node;
      d.rank = rank;
      d.lam[0] = lam[0]; d.lam[1] = lam[1]; d.lam[2] = lam[2];
      pool.desc[(long)pt * pool.cap_part + pos] = d;
    }
  }
}

// Exclusive wave prefix of v; *total receives the wave's sum.
__device__ __forceinline__ int wave_excl_scan(int v, int* total) {
  const int lane = threadIdx.x & 63;
  int incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  *total = __shfl(incl, 63);
  return incl - v;
}

// Exclusive block prefix of v (256 threads); *total receives the block's sum.
// lds: 4 ints of scratch; the call holds two block barriers.
__device__ __forceinline__ int block_excl_scan(int v, int* total, int* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int wt;
  const int ex = wave_excl_scan(v, &wt);
  if (lane == 0) lds[wave] = wt;
  __syncthreads();
  int before = 0, all = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < wave) before += lds[w];
    all += lds[w];
  }
  __syncthreads();
  *total = all;
  return before + ex;
}

// One thread per (order slot, quad) of the chunk: blockIdx.y is the slot,
// blockIdx.x * 256 + threadIdx.x the chunk quad.  Triangles whose bounding box
// holds at most cand_inline nodes are staged for the block's flattened
// candidate loop (queue, slots and candidates shared by the block's four
// waves, so that sparse work fills whole waves); larger ones are listed row
// by row for k_raster_rows.
template <typename G>
__global__ void __launch_bounds__(256) k_raster(const BatchDev B, const Records<G> rec, const NodeGrid ng,
                                                const HitPool<G> pool, const double margin, const int cand_inline) {
  __shared__ BlockStage<G> S;
  __shared__ int s_p0;
  const int lane = threadIdx.x & 63;
  const int slot = blockIdx.y;
  const long n_quads = B.quad_off[B.n] - B.quad_base;
  const long gq0 = (long)blockIdx.x * blockDim.x;
  if (threadIdx.x == 0) s_p0 = find_part(B.quad_off, B.n, B.quad_base, gq0);
  const AxisFast axt = axis_fast(ng.seg_t, ng.n_theta), axp = axis_fast(ng.seg_p, ng.n_phi);
  __syncthreads();
  const long gq = gq0 + threadIdx.x;

  // Phase one, every quad: validity from the flags, then the box of each valid
  // triangle from its vertex angles where fast_box applies.  Triangles with
  // candidate nodes, or whose box needs the directions, are queued in LDS.
  Cand c0, c1;
  bool need0 = false, need1 = false, fast0 = false, fast1 = false;
  int p = s_p0;
  long quad = 0;
  // the block's first particle: its metadata in one round of independent loads
  const long qend0 = B.quad_off[p + 1] - B.quad_base;
  const int N0 = B.P[p].N;
  const long qoff0 = B.quad_off[p] - B.quad_base, roff0 = B.ray_off[p] - B.ray_base;
  if (gq < n_quads) {
    int N = N0;
    long qoff = qoff0, roff = roff0;
    if (gq >= qend0) {  // a block spans few particles
      ++p;
      while (B.quad_off[p + 1] - B.quad_base <= gq) ++p;
      N = B.P[p].N;
      qoff = B.quad_off[p] - B.quad_base;
      roff = B.ray_off[p] - B.ray_base;
    }
    quad = gq - qoff;
    const int Nq = N - 1;
    const long NN = (long)N * N;
    const long rb = B.n_ord * roff + (long)slot * NN;
    const int iy = div_quot15((int)quad, Nq), ix = (int)quad - iy * Nq;
    const long v00 = (long)iy * N + ix;
    // flags and vertex angles are loaded together: one memory round trip per
    // block instead of two (the angles of an invalid quad are not used)
    const float2* an = rec.ang + rb;
    const int f0 = rec.flags[rb + v00], f1 = rec.flags[rb + v00 + 1];
    const int f2 = rec.flags[rb + v00 + N], f3 = rec.flags[rb + v00 + N + 1];
    const float2 a00 = an[v00], a01 = an[v00 + 1], a10 = an[v00 + N], a11 = an[v00 + N + 1];
    const int nf0 = f0 >> 1 & 127;
    const bool tv0 = (f0 & 1) && (f1 & 1) && (f3 & 1) && nf0 == (f1 >> 1 & 127) && nf0 == (f3 >> 1 & 127);
    const bool tv1 = (f0 & 1) && (f2 & 1) && (f3 & 1) && nf0 == (f2 >> 1 & 127) && nf0 == (f3 >> 1 & 127);
    if (tv0 || tv1) {
      if (tv0) {
        fast0 = fast_box(ng, axt, axp, a00, a01, a11, (float)margin, c0);
        need0 = !fast0 || c0.count() > 0;
      }
      if (tv1) {
        fast1 = fast_box(ng, axt, axp, a00, a11, a10, (float)margin, c1);
        need1 = !fast1 || c1.count() > 0;
      }
    }
  }
  // block-wide queue: wave w's entries follow those of waves < w
  const int wave = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  const unsigned long long q0 = __ballot(need0), q1 = __ballot(need1);
  const int nq0 = __popcll(q0), nqw = nq0 + __popcll(q1);
  if (lane == 0) S.wave_q[wave] = nqw;
  __syncthreads();
  int qbase = 0, nq = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    qbase += w < wave ? S.wave_q[w] : 0;
    nq += S.wave_q[w];
  }
  auto enqueue = [&](int at, int t, bool fast, const Cand& c) {
    TriQueued& e = S.queued[at];
    e.quad = (int)quad; e.part = p; e.tf = t | (fast ? 2 : 0);
    e.i0 = c.i0; e.i1 = c.i1; e.ja0 = c.ja0; e.ja1 = c.ja1; e.jb0 = c.jb0; e.jb1 = c.jb1;
  };
  if (need0) enqueue(qbase + __popcll(q0 & below), 0, fast0, c0);
  if (need1) enqueue(qbase + nq0 + __popcll(q1 & below), 1, fast1, c1);
  __syncthreads();

  // Phase two, 256 queued triangles at a time over the block: directions and
  // orientation, the direction box where the angle box did not apply; boxes
  // of at most cand_inline nodes are staged in slot k, larger ones listed by
  // row.  The queue shares the slots' storage with a different element size,
  // so every entry is read into registers before the first slot is written.
  TriQueued mine[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
    if (256 * h + (int)threadIdx.x < nq) mine[h] = S.queued[256 * h + threadIdx.x];
  __syncthreads();
  int block_total = 0;
  const int n_iter = nq > 256 ? 2 : 1;  // block-uniform
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h >= n_iter) break;
    const int k = 256 * h + (int)threadIdx.x;
    Tri<G> T;
    Cand c;
    int n = 0, r = 0;
    if (k < nq) {
      const TriQueued& e = mine[h];
      const int t = e.tf & 1, pp = e.part;
      const bool first = pp == s_p0;  // the block's first particle: metadata already in registers
      const int N = first ? N0 : B.P[pp].N;
      const long qoff = first ? qoff0 : B.quad_off[pp] - B.quad_base;
      const long nq2 = (long)(N - 1) * (N - 1);
      const long rb = B.n_ord * (first ? roff0 : B.ray_off[pp] - B.ray_base) + (long)slot * N * N;
      tri_load(rec, rb, N, (long)e.quad, t, tri_key(B.n_ord, qoff, slot, nq2, (long)e.quad, t), pp, T);
      if (T.orient != 0) {
        if (e.tf & 2) {
          c.i0 = e.i0; c.i1 = e.i1; c.ja0 = e.ja0; c.ja1 = e.ja1; c.jb0 = e.jb0; c.jb1 = e.jb1;
        } else {
          c = box_cand(ng, tri_box(T, (float)margin));
        }
        const int cnt = c.count();
        if (cnt > 0) {
          if (cnt <= cand_inline) n = cnt; else r = c.i1 - c.i0;
        }
      }
    }
    // rows of large triangles: wave-level exclusive scan, one atomic per wave
    int wave_rows;
    const int before = wave_excl_scan(r, &wave_rows);
    if (wave_rows > 0) {
      unsigned rbase = 0;
      if (lane == 63) rbase = atomicAdd(pool.n_rows, (unsigned)wave_rows);
      rbase = __shfl(rbase, 63);
      const unsigned at = rbase + (unsigned)before;
      const bool fits = (unsigned long long)rbase + (unsigned)wave_rows <= (unsigned long long)pool.rows_cap;
      for (int j = 0; j < r; ++j) {
        const unsigned pos = at + j;
        if (fits) pool.rows[pos] = make_int2(T.key, c.i0 + j);
        else if (pos < (unsigned)pool.rows_cap) pool.rows[pos] = make_int2(-1, 0);  // unused slot
      }
      if (!fits && r > 0) n = c.count();  // list full: rasterise the whole box here (slow but exact)
    }
    constexpr bool all_at_once = BlockSlots<G>::value == 512;
    const int sk = all_at_once ? k : (int)threadIdx.x;
    if (n > 0) slot_put(S.tri[sk], T, c);
    int it_total;
    const int ex = block_excl_scan(n, &it_total, S.wave_q);
    if constexpr (all_at_once) {
      S.excl[k] = block_total + ex;
      block_total += it_total;
    } else {
      // this half's triangles: drain them before the next half takes the slots
      S.excl[threadIdx.x] = ex;
      __syncthreads();
      raster_drain(rec, ng, pool, view(S), it_total, wave, 4, wave_partition());
      __syncthreads();
    }
  }
  if constexpr (BlockSlots<G>::value == 512) {
    if (n_iter == 1) S.excl[256 + threadIdx.x] = block_total;
    __syncthreads();
    raster_drain(rec, ng, pool, view(S), block_total, wave, 4, wave_partition());
  }
}

// One thread per listed (triangle, theta row).  A large triangle's rows sit
// next to each other in the list, so consecutive items go to different waves
// (item = pass base + lane x total waves + global wave index): the rows of
// one triangle near a pole, thousands of nodes each, are drained by many
// waves instead of one.  Each row's candidates are the nodes of the row's
// longitude window (row_window).
template <typename G>
__global__ void __launch_bounds__(256) k_raster_rows(const BatchDev B, const Records<G> rec, const NodeGrid ng,
                                                     const HitPool<G> pool, const double margin) {
  __shared__ WaveStage<G> stage[4];
  WaveStage<G>& W = stage[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63;
  const unsigned n_items = min(*pool.n_rows, (unsigned)pool.rows_cap);
  const int part = wave_partition();
  const double sin_margin = sin(margin);
  const unsigned n_waves = gridDim.x * (blockDim.x >> 6);
  const unsigned gwave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  for (unsigned first = 0; first < n_items; first += n_waves * 64u) {
    const unsigned item = first + (unsigned)lane * n_waves + gwave;
    int n = 0;
    int2 w = make_int2(-1, 0);
    if (item < n_items) w = pool.rows[item];
    if (w.x >= 0) {
      const int key = w.x;
      const int it = w.y;
      const int t = key & 1;
      const long sq = key >> 1;  // n_ord quad_off + slot nq + quad
      // particle: largest p with n_ord (quad_off[p] - base) <= sq
      int lo = 0, hi = B.n - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.n_ord * (B.quad_off[mid] - B.quad_base) <= sq) lo = mid; else hi = mid - 1;
      }
      const int p = lo;
      const int N = B.P[p].N;
      const long nq = (long)(N - 1) * (N - 1);
      const long within = sq - B.n_ord * (B.quad_off[p] - B.quad_base);
      const int slot = (int)(within / nq);
      const long quad = within - (long)slot * nq;
      const long rb = B.n_ord * (B.ray_off[p] - B.ray_base) + (long)slot * N * N;
      Tri<G> T;
      tri_load(rec, rb, N, quad, t, key, p, T);
      if (T.orient != 0) {
        const Box bx = tri_box(T, (float)margin);
        double lo_phi, hi_phi;
        if (row_window(T, bx, ng.sth[it], ng.cth[it], sin_margin, lo_phi, hi_phi)) {
          int j0[2], j1[2];
          const int nr = phi_ranges(ng, lo_phi, hi_phi, j0, j1);
          Cand cd;
          cd.i0 = it;
          cd.i1 = it + 1;
          cd.ja0 = j0[0];
          cd.ja1 = j1[0];
          cd.jb0 = nr > 1 ? j0[1] : 0;
          cd.jb1 = nr > 1 ? j1[1] : 0;
          n = cd.count();
          if (n > 0) slot_put(W.tri[lane], T, cd);
        }
      }
    }
    int wave_total;
    W.excl[lane] = wave_excl_scan(n, &wave_total);
    __syncthreads();
    raster_drain(rec, ng, pool, view(W), wave_total, 0, 1, part);
    __syncthreads();  // the stage is rewritten by the next block of items
  }
}

// Exclusive prefix of the node counts (three phases: per-block scans of
// SCAN_BLOCK counts, a scan of the block sums, their addition).
constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_BLOCK = 256 * SCAN_PER_THREAD;


__global__ void __launch_bounds__(256) k_scan_local(const int* count, long n, int* out, int* bsum) {
  __shared__ int lds[4];
  const long base = (long)blockIdx.x * SCAN_BLOCK + (long)threadIdx.x * SCAN_PER_THREAD;
  int v[SCAN_PER_THREAD], s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    v[j] = base + j < n ? count[base + j] : 0;
    s += v[j];
  }
  int total;
  int run = block_excl_scan(s, &total, lds);
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One block: exclusive scan of the nb block sums in place.
__global__ void __launch_bounds__(1024) k_scan_sums(int* bsum, int nb) {
  __shared__ int lds[16];
  const int per = (nb + blockDim.x - 1) / blockDim.x;
  const int b0 = threadIdx.x * per;
  int s = 0;
  for (int j = 0; j < per; ++j)
    if (b0 + j < nb) s += bsum[b0 + j];
  int total;
  int run = block_excl_scan(s, &total, lds);
  for (int j = 0; j < per; ++j)
    if (b0 + j < nb) { const int x = bsum[b0 + j]; bsum[b0 + j] = run; run += x; }
}


// Sum of the fold pair at pool positions a, b (the same order slot): the
// uniform Airy form of the two branches (focal-line counts n and n + 1) with
// Delta = (phi_b - phi_a) / 2 + pi / 4 from their phases carried to the node,
// (2/3) zeta^{3/2} = Delta; the plain sum where the counts do not differ by
// one or Delta <= 0.  FP64 throughout, rounded to G once.
template <typename G>
__device__ inline void add_fold_pair(const HitPool<G>& pool, long a, long b, int n_pol, int w, G* acc, G* inc) {
  if (pool.nf[a] > pool.nf[b]) { const long t = a; a = b; b = t; }
  const double delta = 0.5 * (pool.phi[b] - pool.phi[a]) + 0.78539816339744830962;
  const bool fold = pool.nf[b] - pool.nf[a] == 1 && delta > 0.0;
  double zeta = 0.0, ai = 0.0, aip = 0.0, z4 = 1.0, ed_r = 1.0, ed_i = 0.0;
  if (fold) {
    zeta = pow(1.5 * delta, 2.0 / 3.0);
    airy_neg(zeta, ai, aip);
    z4 = sqrt(sqrt(zeta));
    sincos(delta, &ed_i, &ed_r);
  }
  // sqrt(pi) e^{-i pi/4}
  const double pr = 1.2533141373155002512, pi_ = -1.2533141373155002512;
  for (int p = 0; p < n_pol; ++p) {
    const G* fa = pool.contrib + a * w + 4 * p;
    const G* fb = pool.contrib + b * w + 4 * p;
    for (int c = 0; c < 2; ++c) {
      const double ar = fa[2 * c], aI = fa[2 * c + 1], br = fb[2 * c], bI = fb[2 * c + 1];
      inc[p] += (G)(ar * ar + aI * aI + br * br + bI * bI);
      double ur = ar + br, ui = aI + bI;
      if (fold) {
        // s = f_a e^{i D} + i f_b e^{-i D},  t = f_a e^{i D} - i f_b e^{-i D}
        const double xr = ar * ed_r - aI * ed_i, xi = ar * ed_i + aI * ed_r;     // f_a e^{iD}
        const double yr = br * ed_r + bI * ed_i, yi = bI * ed_r - br * ed_i;     // f_b e^{-iD}
        const double sr = xr - yi, si = xi + yr;                                // + i y
        const double tr = xr + yi, ti = xi - yr;                                // - i y
        // v = s z4 Ai - i t Ai' / z4
        const double vr = sr * z4 * ai + ti * aip / z4, vi = si * z4 * ai - tr * aip / z4;
        ur = pr * vr - pi_ * vi;
        ui = pr * vi + pi_ * vr;
      }
      acc[4 * p + 2 * c] += (G)ur;
      acc[4 * p + 2 * c + 1] += (G)ui;
    }
  }
}

// One thread per node of the chunk (particle-major): order the node's
// contributions (a contiguous range after k_store_hits) by triangle key, sum
// them in that order and write (F_theta, F_phi) for every polarisation into
// the particle's output block; optionally also the incoherent intensity
// sum_b (|f_b,theta|^2 + |f_b,phi|^2) of the node's contributions per
// polarisation.  CAUSTIC (pool.phi and pool.nf set) adds fold pairs in the
// uniform Airy form; the plain instantiation keeps its arrays in registers.
template <typename G, bool CAUSTIC>
__global__ void __launch_bounds__(256) k_node_sum(const BatchDev B, const HitPool<G> pool, int n_nodes, int n_pol,
                                                  G* out, int32_t* ncontrib, G* incoh, int cursor_at_end) {
  const long gn = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gn >= (long)B.n * n_nodes) return;
  const int pl = (int)(gn / n_nodes);
  const int node = (int)(gn - (long)pl * n_nodes);
  const long ob = (long)B.out_index[pl];
  int cnt = pool.count[gn];
  // the range start (the fused path's scatter leaves the cursor at its end)
  const long s0 = (long)pool.cursor[gn] - (cursor_at_end ? cnt : 0);
  {
    // after an overflow the counts include hits the pool could not keep (the
    // result is reported incomplete): the range is kept inside the pool
    const long cap = (long)NPART * pool.cap_part;
    if (s0 < 0 || s0 >= cap) cnt = 0;
    else if (s0 + cnt > cap) cnt = (int)(cap - s0);
  }
  int keys[NODE_SORT_MAX], idxs[NODE_SORT_MAX];
  const int w = n_pol * 4;
  G acc[8], inc[2] = {0, 0};
  for (int i = 0; i < 8; ++i) acc[i] = 0;
  auto add = [&](long at) {
    // one polarisation's contribution is 4 values (16 B / 32 B, aligned): vector loads
    for (int p = 0; p < n_pol; ++p) {
      const V4<G> c = *reinterpret_cast<const V4<G>*>(pool.contrib + at * w + 4 * p);
      acc[4 * p] += c.x; acc[4 * p + 1] += c.y; acc[4 * p + 2] += c.z; acc[4 * p + 3] += c.w;
      inc[p] += c.x * c.x + c.y * c.y + c.z * c.z + c.w * c.w;
    }
  };
  // Caustic correction: contributions of one order slot arrive together (the
  // key orders them by slot first); a slot holding exactly two whose focal-line
  // counts differ by one is a fold pair and is added in the uniform Airy form.
  long qoff = 0, nq = 1;
  if constexpr (CAUSTIC) {
    const int N = B.P[pl].N;
    qoff = (long)B.n_ord * (B.quad_off[pl] - B.quad_base);
    nq = (long)(N - 1) * (N - 1);
  }
  long pend[2];
  int npend = 0, cur_slot = -1;
  auto flush = [&]() {
    if (npend == 2) add_fold_pair(pool, pend[0], pend[1], n_pol, w, acc, inc);
    else if (npend == 1) add(pend[0]);
    npend = 0;
  };
  auto take = [&](long at, int key) {
    if constexpr (!CAUSTIC) {
      (void)key;
      add(at);
      return;
    }
    const int slot = (int)(((long)(key >> 1) - qoff) / nq);
    if (slot != cur_slot) { flush(); cur_slot = slot; }
    if (npend < 0) { add(at); return; }  // a slot with more than two: plain sum
    if (npend < 2) { pend[npend++] = at; return; }
    add(pend[0]); add(pend[1]); add(at);
    npend = -1;
  };
  if (cnt <= NODE_SORT_MAX) {
    for (int h = 0; h < cnt; ++h) {  // insertion into the sorted prefix
      const int kk = pool.key[s0 + h];
      int j = h;
      while (j > 0 && keys[j - 1] > kk) { keys[j] = keys[j - 1]; idxs[j] = idxs[j - 1]; --j; }
      keys[j] = kk; idxs[j] = h;
    }
    for (int i = 0; i < cnt; ++i) take(s0 + idxs[i], keys[i]);
  } else {
    // more hits than the register window: repeated minimum search, same order
    long last = -1;
    for (int r = 0; r < cnt; ++r) {
      long best = 0x7fffffffffffL;
      int bi = 0;
      for (int h = 0; h < cnt; ++h) {
        const long kk = pool.key[s0 + h];
        if (kk > last && kk < best) { best = kk; bi = h; }
      }
      last = best;
      take(s0 + bi, (int)best);
    }
  }
  if constexpr (CAUSTIC) flush();
  G* po = out + ob * ((long)n_pol * 2 * n_nodes * 2);
  for (int p = 0; p < n_pol; ++p)
    for (int a = 0; a < 2; ++a) {
      long o = ((long)(p * 2 + a) * n_nodes + node) * 2;
      po[o] = acc[p * 4 + a * 2];
      po[o + 1] = acc[p * 4 + a * 2 + 1];
    }
  if (ncontrib) ncontrib[ob * n_nodes + node] = cnt;
  if (incoh)
    for (int p = 0; p < n_pol; ++p) incoh[(ob * n_pol + p) * n_nodes + node] = inc[p];
}

}  // namespace rtw
