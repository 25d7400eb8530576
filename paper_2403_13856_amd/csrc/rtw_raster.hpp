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
// Membership is watertight: the edge function of an edge is always evaluated
// from its lower ray index to its higher one with contraction disabled, so the
// two triangles sharing an edge see the same value and exactly one of them
// claims a node on it (the one on the edge's positive side on an exact tie).
//
// Hits are appended to a pool with one atomic per wave per step (wave ballot)
// on one of NPART counters; each hit is pushed on its node's list with an
// atomic exchange.  No floating-point atomics are used: the per-node kernel
// sorts the node's hits by triangle key and sums them in that order.
#pragma once
#include "rtw_device.hpp"

namespace rtw {

constexpr int NPART = 1024;        // hit-pool partitions (spreads the append atomics)
constexpr int NODE_SORT_MAX = 16;  // hits per node sorted in registers; more use a selection pass

struct NodeGrid {
  int n_theta, n_phi;
  const double* th;   // radians, ascending
  const double* ph;   // radians, ascending, in [0, 2 pi)
  const double* sth;  // sin theta
  const double* cth;
  const double* sph;
  const double* cph;
};

template <typename G>
struct Records {
  int32_t* flags;  // [n_ord][NN]  bit0 valid, bits 1..7 nf, bit 8 det_neg
  G* dir;          // [n_ord][3][NN]
  G* kr;           // [n_ord][3][NN] (k r_exit, lab)
  G* field;        // [n_ord][n_pol][3][2][NN]
  long NN;
  int n_pol;
  unsigned* n_fp64;  // rays re-traced in FP64 (mixed path)
  int* redo_list;    // their ray indices
};

template <typename G>
struct HitPool {
  int* head;          // [n_nodes] first hit of each node, -1 = none
  int2* link;         // [cap] (key, next)
  G* contrib;         // [cap][n_pol * 4]: (pol, theta|phi, re|im)
  unsigned* counter;  // [NPART]
  int cap_part;       // capacity of each partition
  int2* rows;         // [rows_cap] (triangle key, theta row) of triangles rasterised row by row
  unsigned* n_rows;   // rows listed
  int rows_cap;
};

constexpr int CAND_INLINE = 256;  // triangles with more box candidates go to the row list

// Sink writing the compact emission records used by the rasteriser.  In the
// mixed path an emission whose divergence factor is ill-conditioned for FP32
// (amplif > amplif_limit) marks the ray for an FP64 re-trace.
template <typename G>
struct RecordSink {
  Records<G> rec;
  long id;
  double k;
  double amplif_limit;
  bool need64;
  template <typename E>
  __device__ void emit(const Emission<E>& e) {
    if (sizeof(E) == 4 && e.amplif > amplif_limit) need64 = true;
    const long NN = rec.NN;
    rec.flags[e.slot * NN + id] = 1 | (e.nf << 1) | (e.det_neg << 8);
    G* dp = rec.dir + (long)e.slot * 3 * NN + id;
    dp[0] = e.dir.x; dp[NN] = e.dir.y; dp[2 * NN] = e.dir.z;
    G* kp = rec.kr + (long)e.slot * 3 * NN + id;
    kp[0] = (G)(k * e.rexit.x); kp[NN] = (G)(k * e.rexit.y); kp[2 * NN] = (G)(k * e.rexit.z);
    G* fp = rec.field + (long)e.slot * rec.n_pol * 6 * NN + id;
    for (int p = 0; p < rec.n_pol; ++p)
      for (int x = 0; x < 3; ++x) {
        fp[((p * 3 + x) * 2 + 0) * NN] = e.f[p][x].re;
        fp[((p * 3 + x) * 2 + 1) * NN] = e.f[p][x].im;
      }
  }
};

__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float sub_rn(float a, float b) { return __fsub_rn(a, b); }
__device__ __forceinline__ double sub_rn(double a, double b) { return __dsub_rn(a, b); }

// (a x b) . n evaluated as a fixed sequence of correctly rounded operations.
template <typename T>
__device__ __forceinline__ T edge_fn(const v3<T>& a, const v3<T>& b, const v3<T>& n) {
  T cx_ = sub_rn(mul_rn(a.y, b.z), mul_rn(a.z, b.y));
  T cy_ = sub_rn(mul_rn(a.z, b.x), mul_rn(a.x, b.z));
  T cz_ = sub_rn(mul_rn(a.x, b.y), mul_rn(a.y, b.x));
  return add_rn(add_rn(mul_rn(cx_, n.x), mul_rn(cy_, n.y)), mul_rn(cz_, n.z));
}

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

// Candidate node set of one triangle: rows [i0, i1) x (phi segment a  U  segment b).
struct Cand {
  int i0, i1, ja0, ja1, jb0, jb1;
  __device__ int len() const { return (ja1 - ja0) + (jb1 - jb0); }
  __device__ int count() const { return (i1 - i0) * len(); }
};

// Conservative candidate set: the spherical cap of radius rho about the unit
// vector c contains the triangle; nodes outside the cap's (theta, phi) box
// cannot be inside it.
__device__ inline Cand cap_candidates(const NodeGrid& ng, const v3<double>& c, double rho) {
  const double PI_ = 3.141592653589793, TWO_PI = 6.283185307179586;
  Cand cd;
  double cz = fmin(1.0, fmax(-1.0, c.z));
  double thc = acos(cz);
  double phc = atan2(c.y, c.x);
  if (phc < 0) phc += TWO_PI;
  double tlo = thc - rho, thi = thc + rho;
  cd.i0 = lower_idx(ng.th, ng.n_theta, tlo);
  cd.i1 = upper_idx(ng.th, ng.n_theta, thi);
  cd.jb0 = cd.jb1 = 0;
  bool full = (tlo <= 0.0) || (thi >= PI_) || (rho >= 0.5 * PI_);
  double dphi = 0.0;
  if (!full) {
    double sr = sin(rho) / sin(thc);
    if (sr >= 1.0) full = true;
    else dphi = asin(sr);
  }
  if (full) {
    cd.ja0 = 0; cd.ja1 = ng.n_phi;
    return cd;
  }
  double lo = phc - dphi, hi = phc + dphi;
  if (lo < 0.0) {
    cd.ja0 = lower_idx(ng.ph, ng.n_phi, lo + TWO_PI); cd.ja1 = ng.n_phi;
    cd.jb0 = 0; cd.jb1 = upper_idx(ng.ph, ng.n_phi, hi);
  } else if (hi >= TWO_PI) {
    cd.ja0 = lower_idx(ng.ph, ng.n_phi, lo); cd.ja1 = ng.n_phi;
    cd.jb0 = 0; cd.jb1 = upper_idx(ng.ph, ng.n_phi, hi - TWO_PI);
  } else {
    cd.ja0 = lower_idx(ng.ph, ng.n_phi, lo); cd.ja1 = upper_idx(ng.ph, ng.n_phi, hi);
  }
  return cd;
}

// phi intervals (up to two, absolute radians, each within [lo, lo + 2 pi)) of
// the latitude circle (sin t, cos t) inside the three oriented half-spaces
// m_e . n >= 0.  Each is R cos(phi - phi_e) >= -c on the circle.  Widened by eps.
struct Arcs {
  int n;
  double lo[4], hi[4];
};
__host__ __device__ inline Arcs row_arcs(const v3<double>* m, double st, double ct, double eps) {
  const double TWO_PI = 6.283185307179586;
  Arcs A;
  A.n = 1;
  A.lo[0] = 0.0;
  A.hi[0] = TWO_PI;  // start with the full circle, relative frame origin 0
  bool full_so_far = true;
  double base = 0.0;  // absolute angle of the relative frame origin
  for (int e = 0; e < 3; ++e) {
    double R = st * sqrt(m[e].x * m[e].x + m[e].y * m[e].y);
    double c = m[e].z * ct;
    double scale = fabs(R) + fabs(c);
    if (R <= fabs(c)) {
      if (c + eps * scale >= 0.0) continue;  // whole circle satisfies this edge
      A.n = 0;
      return A;
    }
    double alpha = acos(fmax(-1.0, fmin(1.0, -c / R))) + eps;
    double ph0 = atan2(m[e].y, m[e].x);
    if (alpha >= 0.5 * TWO_PI) continue;
    double a0 = ph0 - alpha, len = 2.0 * alpha;
    if (full_so_far) {
      base = a0;
      A.n = 1;
      A.lo[0] = 0.0;
      A.hi[0] = len;
      full_so_far = false;
      continue;
    }
    // arc [s, s + len] in the relative frame, s in [0, 2 pi)
    double sr = fmod(a0 - base, TWO_PI);
    if (sr < 0) sr += TWO_PI;
    double ilo[2] = {sr, 0.0}, ihi[2] = {sr + len, sr + len - TWO_PI};
    int ni = (sr + len > TWO_PI) ? 2 : 1;
    if (ni == 1) ihi[0] = sr + len; else ihi[0] = TWO_PI;
    Arcs B;
    B.n = 0;
    for (int i = 0; i < A.n; ++i)
      for (int j = 0; j < ni; ++j) {
        double lo = fmax(A.lo[i], ilo[j]), hi = fmin(A.hi[i], ihi[j]);
        if (lo <= hi && B.n < 4) { B.lo[B.n] = lo; B.hi[B.n] = hi; ++B.n; }
      }
    A = B;
    if (A.n == 0) return A;
  }
  if (full_so_far) {
    A.n = 1; A.lo[0] = 0.0; A.hi[0] = TWO_PI;
    return A;
  }
  for (int i = 0; i < A.n; ++i) { A.lo[i] += base; A.hi[i] += base; }
  return A;
}

// Node index ranges [j0, j1) of the phi list inside the absolute interval
// [lo, hi] (length < 2 pi, possibly wrapping): up to two ranges.
__host__ __device__ inline int phi_ranges(const NodeGrid& ng, double lo, double hi, int* j0, int* j1) {
  const double TWO_PI = 6.283185307179586;
  if (hi - lo >= TWO_PI) { j0[0] = 0; j1[0] = ng.n_phi; return 1; }
  double l = fmod(lo, TWO_PI);
  if (l < 0) l += TWO_PI;
  double h = l + (hi - lo);
  if (h < TWO_PI) {
    j0[0] = lower_idx(ng.ph, ng.n_phi, l); j1[0] = upper_idx(ng.ph, ng.n_phi, h);
    return 1;
  }
  j0[0] = lower_idx(ng.ph, ng.n_phi, l); j1[0] = ng.n_phi;
  j0[1] = 0; j1[1] = upper_idx(ng.ph, ng.n_phi, h - TWO_PI);
  return 2;
}

template <typename G>
__device__ __forceinline__ v3<G> load_dir(const Records<G>& rec, int slot, long id) {
  const G* p = rec.dir + (long)slot * 3 * rec.NN + id;
  return mk3<G>(p[0], p[rec.NN], p[2 * rec.NN]);
}

// One triangle of one order, as the rasteriser needs it.
template <typename G>
struct Tri {
  long vid[3];  // global ray ids in triangle order
  v3<G> dv[3];  // stored exit directions
  int sig[3];   // +1 if edge e (cyclic, opposite vertex e) runs from the lower ray id
  int orient;   // sign of the triple product of the directions
  int slot;
  int key;      // ((slot * nquad + quad) * 2 + t): the per-node summation order
};

template <typename G>
__device__ inline void tri_load(const Records<G>& rec, int N, int slot, long quad, int t, Tri<G>& T) {
  const int Nq = N - 1;
  const int iy = (int)(quad / Nq), ix = (int)(quad - (long)iy * Nq);
  const long v00 = (long)iy * N + ix;
  T.vid[0] = v00;
  T.vid[1] = t == 0 ? v00 + 1 : v00 + N + 1;
  T.vid[2] = t == 0 ? v00 + N + 1 : v00 + N;
  for (int k = 0; k < 3; ++k) T.dv[k] = load_dir(rec, slot, T.vid[k]);
  T.slot = slot;
  T.key = (int)(((long)slot * Nq * Nq + quad) * 2 + t);
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

// Bounding cap (centre, radius) of the triangle: chords of the normalised
// directions, which stay accurate for tiny triangles.
template <typename G>
__device__ inline void tri_cap(const Tri<G>& T, double margin, v3<double>& s, double& rho) {
  v3<double> un[3];
  for (int k = 0; k < 3; ++k) {
    v3<double> dd = cvt<double>(T.dv[k]);
    un[k] = scl(1.0 / sqrt(dot(dd, dd)), dd);
  }
  s = mk3<double>(un[0].x + un[1].x + un[2].x, un[0].y + un[1].y + un[2].y, un[0].z + un[1].z + un[2].z);
  s = scl(1.0 / sqrt(dot(s, s)), s);
  double chord = 0.0;
  for (int k = 0; k < 3; ++k) {
    v3<double> df = mk3<double>(un[k].x - s.x, un[k].y - s.y, un[k].z - s.z);
    chord = fmax(chord, sqrt(dot(df, df)));
  }
  rho = 2.0 * asin(fmin(1.0, 0.5 * chord)) * (1.0 + 1e-6) + margin;
}

// Membership of node direction n (watertight canonical-edge rule) and its
// barycentric weights; dl receives d_v - n.
template <typename G>
__device__ inline bool tri_member(const Tri<G>& T, const v3<double>& n, G lam[3], v3<G> dl[3]) {
  for (int k = 0; k < 3; ++k)
    dl[k] = mk3<G>((G)((double)T.dv[k].x - n.x), (G)((double)T.dv[k].y - n.y), (G)((double)T.dv[k].z - n.z));
  const v3<G> nG = cvt<G>(n);
  bool inside = true;
  G w[3];
  const int o = T.orient;
  for (int e = 0; e < 3; ++e) {
    // canonical edge function (lower ray index first), shared bit-for-bit
    // with the neighbouring triangle across this edge
    int i = (e + 1) % 3, j = (e + 2) % 3;
    if (T.sig[e] < 0) { int tmp = i; i = j; j = tmp; }
    G ev = edge_fn(dl[i], dl[j], nG);
    G se = T.sig[e] > 0 ? ev : -ev;  // cyclic-order edge function = barycentric weight of vertex e
    w[e] = se;
    bool ok = (o > 0 ? se > 0 : se < 0) || (ev == 0 && T.sig[e] * o > 0);
    inside = inside && ok;
  }
  if (!inside) return false;
  G sw = 1 / (w[0] + w[1] + w[2]);
  lam[0] = w[0] * sw; lam[1] = w[1] * sw; lam[2] = w[2] * sw;
  return true;
}

// Contribution of triangle T at node (it, ip), stored at pool slot idx and
// pushed on the node's list.
template <typename G>
__device__ inline void tri_store_hit(const Records<G>& rec, const NodeGrid& ng, const HitPool<G>& pool, const Tri<G>& T,
                                     int it, int ip, const G lam[3], const v3<G> dl[3], long idx) {
  const long NN = rec.NN;
  const G st = (G)ng.sth[it], ct = (G)ng.cth[it], sp = (G)ng.sph[ip], cp = (G)ng.cph[ip];
  const v3<G> eth = mk3<G>(ct * cp, ct * sp, -st);
  const v3<G> eph = mk3<G>(-sp, cp, (G)0);
  G acc[2][2][2];
  for (int p = 0; p < 2; ++p)
    for (int a = 0; a < 2; ++a) acc[p][a][0] = acc[p][a][1] = 0;
  for (int k = 0; k < 3; ++k) {
    const long id = T.vid[k];
    const G* kp = rec.kr + (long)T.slot * 3 * NN + id;
    G psi = kp[0] * dl[k].x + kp[NN] * dl[k].y + kp[2 * NN] * dl[k].z;  // k r.(d - n)
    G s_, c_;
    sincos_t(psi, &s_, &c_);
    const G lr = lam[k] * c_, li = lam[k] * s_;
    const G* fp = rec.field + (long)T.slot * rec.n_pol * 6 * NN + id;
    for (int p = 0; p < rec.n_pol; ++p) {
      G fxr = fp[(p * 6 + 0) * NN], fxi = fp[(p * 6 + 1) * NN];
      G fyr = fp[(p * 6 + 2) * NN], fyi = fp[(p * 6 + 3) * NN];
      G fzr = fp[(p * 6 + 4) * NN], fzi = fp[(p * 6 + 5) * NN];
      G tr = fxr * eth.x + fyr * eth.y + fzr * eth.z, ti = fxi * eth.x + fyi * eth.y + fzi * eth.z;
      G pr = fxr * eph.x + fyr * eph.y, pi_ = fxi * eph.x + fyi * eph.y;
      acc[p][0][0] += lr * tr - li * ti;  acc[p][0][1] += lr * ti + li * tr;
      acc[p][1][0] += lr * pr - li * pi_; acc[p][1][1] += lr * pi_ + li * pr;
    }
  }
  G* out = pool.contrib + idx * (rec.n_pol * 4);
  for (int p = 0; p < rec.n_pol; ++p) {
    out[p * 4 + 0] = acc[p][0][0]; out[p * 4 + 1] = acc[p][0][1];
    out[p * 4 + 2] = acc[p][1][0]; out[p * 4 + 3] = acc[p][1][1];
  }
  const int node = it * ng.n_phi + ip;
  int prev = atomicExch(&pool.head[node], (int)idx);
  pool.link[idx] = make_int2(T.key, prev);
}

// Wave-aggregated append: every lane with hit == true receives a pool slot
// (or -1 on overflow).  Must be called in wave-uniform control flow.
__device__ inline long wave_reserve(bool hit, unsigned* counter, int part, int cap_part) {
  const int lane = threadIdx.x & 63;
  unsigned long long mask = __ballot(hit);
  if (mask == 0ull) return -1;
  int leader = __ffsll((long long)mask) - 1;
  unsigned base = 0;
  if (lane == leader) base = atomicAdd(&counter[part], (unsigned)__popcll(mask));
  base = __shfl(base, leader);
  if (!hit) return -1;
  unsigned pos = base + (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
  if (pos >= (unsigned)cap_part) return -1;  // overflow: counted, reported by the status call
  return (long)part * cap_part + pos;
}

__device__ inline int wave_partition() {
  return (int)(((long)blockIdx.y * gridDim.x * (blockDim.x >> 6) + (long)blockIdx.x * (blockDim.x >> 6) +
                (threadIdx.x >> 6)) % NPART);
}

// One thread per (order slot, quad).  Small triangles are rasterised here from
// their cap box; triangles whose box holds more than CAND_INLINE nodes are
// listed row by row for k_raster_rows (exact per-row arcs, one row per thread),
// which keeps one large triangle from stalling its wave.
template <typename G>
__global__ void __launch_bounds__(256) k_raster(const ParticleConst P, const Records<G> rec, const NodeGrid ng,
                                                const HitPool<G> pool, const double rho_margin) {
  const int slot = blockIdx.y;
  const int Nq = P.N - 1;
  const long nquad = (long)Nq * Nq;
  const long quad = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long NN = rec.NN;

  Tri<G> T[2];
  Cand cand[2];
  int ncand[2] = {0, 0};
  int nrow[2] = {0, 0};
  if (quad < nquad) {
    int iy = (int)(quad / Nq), ix = (int)(quad - (long)iy * Nq);
    long v00 = (long)iy * P.N + ix;
    int fl[4];
    fl[0] = rec.flags[slot * NN + v00];
    fl[1] = rec.flags[slot * NN + v00 + 1];
    fl[2] = rec.flags[slot * NN + v00 + P.N];
    fl[3] = rec.flags[slot * NN + v00 + P.N + 1];
    const int nf0 = fl[0] >> 1 & 127;
    bool tv[2];
    tv[0] = (fl[0] & 1) && (fl[1] & 1) && (fl[3] & 1) && nf0 == (fl[1] >> 1 & 127) && nf0 == (fl[3] >> 1 & 127);
    tv[1] = (fl[0] & 1) && (fl[2] & 1) && (fl[3] & 1) && nf0 == (fl[2] >> 1 & 127) && nf0 == (fl[3] >> 1 & 127);
    for (int t = 0; t < 2; ++t) {
      if (!tv[t]) continue;
      tri_load(rec, P.N, slot, quad, t, T[t]);
      if (T[t].orient == 0) continue;
      v3<double> s;
      double rho;
      tri_cap(T[t], rho_margin, s, rho);
      cand[t] = cap_candidates(ng, s, rho);
      int cnt = cand[t].count();
      if (cnt <= CAND_INLINE) ncand[t] = cnt;
      else nrow[t] = cand[t].i1 - cand[t].i0;  // listed below
    }
  }
  // wave-level exclusive scan of the rows to list, one atomic per wave
  {
    const int lane = threadIdx.x & 63;
    int mine = nrow[0] + nrow[1];
    int incl = mine;
    for (int off = 1; off < 64; off <<= 1) {
      int y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    const int wave_total = __shfl(incl, 63);
    if (wave_total > 0) {
      unsigned base = 0;
      if (lane == 63) base = atomicAdd(pool.n_rows, (unsigned)wave_total);
      base = __shfl(base, 63);
      const unsigned at = base + (unsigned)(incl - mine);
      const bool fits = (unsigned long long)base + (unsigned)wave_total <= (unsigned long long)pool.rows_cap;
      int r = 0;
      for (int t = 0; t < 2; ++t)
        for (int k = 0; k < nrow[t]; ++k, ++r) {
          const unsigned pos = at + r;
          if (fits) pool.rows[pos] = make_int2(T[t].key, cand[t].i0 + k);
          else if (pos < (unsigned)pool.rows_cap) pool.rows[pos] = make_int2(-1, 0);  // unused slot
        }
      if (!fits)  // list full: rasterise from the cap box here (slow but exact)
        for (int t = 0; t < 2; ++t)
          if (nrow[t] > 0) ncand[t] = cand[t].count();
    }
  }
  const int total = ncand[0] + ncand[1];
  const int part = wave_partition();

  for (int ci = 0; __any(ci < total); ++ci) {
    bool hit = false;
    int t = 0, it = 0, ip = 0;
    G lam[3];
    v3<G> dl[3];
    if (ci < total) {
      t = ci < ncand[0] ? 0 : 1;
      const Cand& cd = cand[t];
      int c = t == 0 ? ci : ci - ncand[0];
      int len = cd.len();
      it = cd.i0 + c / len;
      int jj = c - (c / len) * len;
      ip = jj < (cd.ja1 - cd.ja0) ? cd.ja0 + jj : cd.jb0 + (jj - (cd.ja1 - cd.ja0));
      v3<double> n = mk3<double>(ng.sth[it] * ng.cph[ip], ng.sth[it] * ng.sph[ip], ng.cth[it]);
      hit = tri_member(T[t], n, lam, dl);
    }
    long idx = wave_reserve(hit, pool.counter, part, pool.cap_part);
    if (idx >= 0) tri_store_hit(rec, ng, pool, T[t], it, ip, lam, dl, idx);
  }
}

// One thread per listed (triangle, theta row): the exact phi arcs of the row
// inside the triangle, then the membership test node by node.
template <typename G>
__global__ void __launch_bounds__(256) k_raster_rows(const ParticleConst P, const Records<G> rec, const NodeGrid ng,
                                                     const HitPool<G> pool, const double arc_eps) {
  const unsigned n_items = min(*pool.n_rows, (unsigned)pool.rows_cap);
  const long nquad = (long)(P.N - 1) * (P.N - 1);
  const int part = wave_partition();
  // every lane runs the same number of outer iterations (wave-uniform)
  const unsigned stride = gridDim.x * blockDim.x;
  const unsigned first = blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
  for (unsigned base_item = first; base_item < n_items; base_item += stride) {
    const unsigned item = base_item + (threadIdx.x & 63);
    Tri<G> T;
    int it = 0, nr = 0;
    int j0[8], j1[8];
    int2 w = make_int2(-1, 0);
    if (item < n_items) w = pool.rows[item];
    if (w.x >= 0) {
      const int key = w.x;
      it = w.y;
      const int t = key & 1;
      const long sq = key >> 1;
      const int slot = (int)(sq / nquad);
      const long quad = sq - (long)slot * nquad;
      tri_load(rec, P.N, slot, quad, t, T);
      // oriented edge normals o (d_a x d_b), cyclic edges
      v3<double> m[3];
      for (int e = 0; e < 3; ++e) {
        v3<double> a = cvt<double>(T.dv[(e + 1) % 3]), b = cvt<double>(T.dv[(e + 2) % 3]);
        m[e] = scl((double)T.orient, cross(a, b));
      }
      Arcs A = row_arcs(m, ng.sth[it], ng.cth[it], arc_eps);
      for (int a = 0; a < A.n; ++a) {
        int r0[2], r1[2];
        int k = phi_ranges(ng, A.lo[a], A.hi[a], r0, r1);
        for (int q = 0; q < k; ++q)
          if (r1[q] > r0[q]) { j0[nr] = r0[q]; j1[nr] = r1[q]; ++nr; }
      }
    }
    int total = 0;
    for (int q = 0; q < nr; ++q) total += j1[q] - j0[q];
    int q = 0, ip = nr > 0 ? j0[0] : 0;
    for (int ci = 0; __any(ci < total); ++ci) {
      bool hit = false;
      G lam[3];
      v3<G> dl[3];
      int cur = ip;
      if (ci < total) {
        while (cur >= j1[q]) { ++q; cur = j0[q]; }
        ip = cur + 1;
        v3<double> n = mk3<double>(ng.sth[it] * ng.cph[cur], ng.sth[it] * ng.sph[cur], ng.cth[it]);
        hit = T.orient != 0 && tri_member(T, n, lam, dl);
      }
      long idx = wave_reserve(hit, pool.counter, part, pool.cap_part);
      if (idx >= 0) tri_store_hit(rec, ng, pool, T, it, cur, lam, dl, idx);
    }
  }
}

// One thread per node: walk the node's hit list, order the hits by triangle
// key, sum them in that order and write (F_theta, F_phi) for every polarisation.
template <typename G>
__global__ void __launch_bounds__(256) k_node_sum(const HitPool<G> pool, int n_nodes, int n_pol, G* out,
                                                  int32_t* ncontrib) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= n_nodes) return;
  int keys[NODE_SORT_MAX], idxs[NODE_SORT_MAX];
  int cnt = 0;
  for (int h = pool.head[node]; h >= 0; h = pool.link[h].y) {
    int2 l = pool.link[h];
    if (cnt < NODE_SORT_MAX) {
      // insertion into the sorted prefix
      int j = cnt;
      while (j > 0 && keys[j - 1] > l.x) { keys[j] = keys[j - 1]; idxs[j] = idxs[j - 1]; --j; }
      keys[j] = l.x; idxs[j] = h;
    }
    ++cnt;
  }
  G acc[8];
  for (int i = 0; i < 8; ++i) acc[i] = 0;
  const int w = n_pol * 4;
  if (cnt <= NODE_SORT_MAX) {
    for (int i = 0; i < cnt; ++i) {
      const G* c = pool.contrib + (long)idxs[i] * w;
      for (int k = 0; k < w; ++k) acc[k] += c[k];
    }
  } else {
    // more hits than the register window: repeated minimum search, same order
    long last = -1;
    for (int r = 0; r < cnt; ++r) {
      long best = 0x7fffffffffffL;
      int bi = -1;
      for (int h = pool.head[node]; h >= 0; h = pool.link[h].y) {
        long kk = pool.link[h].x;
        if (kk > last && kk < best) { best = kk; bi = h; }
      }
      last = best;
      const G* c = pool.contrib + (long)bi * w;
      for (int k = 0; k < w; ++k) acc[k] += c[k];
    }
  }
  for (int p = 0; p < n_pol; ++p)
    for (int a = 0; a < 2; ++a) {
      long o = ((long)(p * 2 + a) * n_nodes + node) * 2;
      out[o] = acc[p * 4 + a * 2];
      out[o + 1] = acc[p * 4 + a * 2 + 1];
    }
  if (ncontrib) ncontrib[node] = cnt;
}

}  // namespace rtw
