// rtw_fused.hpp -- the mixed-precision far field of one particle tile in one
// pass through the CU: trace, rasterisation and hit contributions without
// per-ray records in HBM.
//
// A block takes a tile of 64 x (4 S) incident rays (63 x (4 S - 1) quads:
// neighbouring tiles share their edge column and row of rays, traced by both,
// bit for bit alike) and walks it in S steps of 64 x 4 rays, one ray per
// thread.  Within a step the rays advance one interaction at a time (Eq. 3,
// 4, 6, 8 of each ray); after the interaction that emits order slot s, every
// ray's record of that order sits in LDS and the block rasterises the step's
// quads of slot s: those between the four new ray rows, and those between the
// previous step's last row (kept per order slot in LDS, the carry) and the
// first new row.  A hit's contribution (the interpolation of the RTW strategy
// section: barycentric field, phase carried to the node by the stationary-
// phase gradient) is formed from the three LDS records at once and leaves the
// CU as one hit record; a scan of the node counts and a scatter then put the
// hits in node order for the ordered per-node sum.
//
// Rays whose divergence factor is ill-conditioned in FP32 (the mixed path's
// FP64 re-trace) are collected in LDS when their emission is found so and
// traced again in FP64 by the block, all lanes taking one listed ray each;
// the FP64 records of that and every later order go to the block's area of a
// global scratch array, from which the ray's own thread copies each order's
// record into LDS.  A record, once in LDS, is the one every triangle of that
// ray and order uses (the canonical edge normals stay watertight).
#pragma once
#include "rtw_raster.hpp"

namespace rtw {

constexpr int FUSED_COLS = 64;     // rays per tile row (63 quads)
constexpr int FUSED_ROWS = 4;      // ray rows per step (one wave each)
constexpr int FUSED_MAX_ORD = 6;   // order slots the carry holds (p <= 5 from p_min = 0)
constexpr int FUSED_BPC = 2;       // resident blocks per CU (LDS and registers)

// One ray's record of one order in LDS: 19 words, so that the records of
// consecutive rays start in different banks.
struct LRec {
  float kr[3];   // k r_exit (lab)
  float dir[3];  // stored exit direction
  float f[8];    // [pol][e_theta|e_phi][re|im] on the direction's own basis
  RecTail<float> tail;
  int flags;     // bit0 valid, bits 1..7 nf, bit 8 det_neg
  float th, ph;  // (theta, phi) of dir
};
static_assert(sizeof(LRec) == 76, "LDS record size");

__device__ __forceinline__ v3<double> full_dir(const LRec& r) {
  return mk3((double)r.dir[0] + (double)r.tail.dlo[0] * (1.0 / DLO_SCALE),
             (double)r.dir[1] + (double)r.tail.dlo[1] * (1.0 / DLO_SCALE),
             (double)r.dir[2] + (double)r.tail.dlo[2] * (1.0 / DLO_SCALE));
}

__device__ __forceinline__ void put_lrec(LRec& d, const RecVals<float>& v) {
  LRec r;
  for (int i = 0; i < 3; ++i) { r.kr[i] = v.kr[i]; r.dir[i] = v.dir[i]; }
  for (int i = 0; i < 8; ++i) r.f[i] = v.f[i];
  r.tail = v.tail;
  r.flags = v.flags;
  r.th = v.th;
  r.ph = v.ph;
  d = r;
}

// FP32 trace: the emission's record goes to the ray's LDS place, unless its
// divergence factor is ill-conditioned for FP32 (the ray is then listed for
// the FP64 re-trace and this record is not used).
struct LdsSink {
  LRec* dst;
  double k, kappa, amplif_limit;
  int n_pol;
  bool wrote, need64;
  template <typename E>
  __device__ void emit(const Emission<E>& e) {
    if (e.amplif > amplif_limit) {
      need64 = true;
      return;
    }
    RecVals<float> v;
    record_values(e, k, kappa, n_pol, v);
    put_lrec(*dst, v);
    wrote = true;
  }
};

// FP64 re-trace: the records of every emitted order into the ray's scratch
// area (one record per order slot, cleared beforehand).
struct ScratchSink {
  LRec* base;
  double k, kappa;
  int n_pol;
  template <typename E>
  __device__ void emit(const Emission<E>& e) {
    RecVals<float> v;
    record_values(e, k, kappa, n_pol, v);
    put_lrec(base[e.slot], v);
  }
};

// Where the fused kernel puts its hits: per hit one record of 1 + n_pol
// 16-byte words, (key, node, 0, 0) then per polarisation the contribution
// (F_theta re, im, F_phi re, im), in one of NPART partitions.  Each wave takes
// its slots in runs of FUSED_RUN from one partition at a time (one atomic per
// run); slots of a run it leaves unused hold node -1.
constexpr int FUSED_RUN = 256;
struct FusedPool {
  int* count;          // [n_nodes of the chunk] hits per node (counted without waiting on the atomic)
  unsigned* counter;   // [NPART] partition fills (slots handed out in runs)
  unsigned* n_hits;    // hits stored over the call
  V4<float>* hits;     // [NPART][cap_part][1 + n_pol]
  int cap_part;
  int n_pol;
  LRec* scratch;       // [grid blocks][256][n_ord] records of the rays re-traced in FP64
  RayState<float>* park;  // [grid blocks][256] FP32 ray states parked during an FP64 re-trace
  unsigned* n_fp64;    // rays re-traced in FP64 (chunk)
};

// A wave's current run of pool slots: [next, end) of partition part.
struct SlotRun {
  int part;
  unsigned next, end;
};

// Slots [r.next, r.end) of the wave's run will not be used: mark them empty.
__device__ __forceinline__ void close_run(const FusedPool& fp, const SlotRun& r) {
  const int lane = threadIdx.x & 63;
  for (unsigned at = r.next + lane; at < r.end && at < (unsigned)fp.cap_part; at += 64) {
    V4<float> h0;
    h0.x = 0.0f; h0.y = __int_as_float(-1); h0.z = 0.0f; h0.w = 0.0f;
    fp.hits[((long)r.part * fp.cap_part + at) * (1 + fp.n_pol)] = h0;
  }
}

// A node hit waiting in LDS for its contribution: triangle key, node (row |
// column << 16), barycentric weights of the membership test.
struct HitEntry {
  int key;
  int itip;
  float lam[3];
};
constexpr int FUSED_HITS = 256;  // the list's capacity: one drain pass adds at most 256

// LDS of one fused block besides the carry (dynamic, n_ord x 64 records).
struct FusedShared {
  LRec T[FUSED_ROWS][FUSED_COLS];  // the step's rays, current order slot
  BlockStage<float> S;             // rasteriser queue and staged triangles
  int list[256];                   // rays listed for the FP64 re-trace in this step
  int n_list;
  HitEntry hit[FUSED_HITS];        // hits waiting for their contributions
  int n_hit;
  int wave_any[2][FUSED_ROWS];      // per step parity: does wave w hold a ray that meets the particle
  long item;
};

// The triangle (slot k of the stage) from LDS records, as tri_load does from
// HBM: rays (corner, +1 or +N+1, ...) in triangle order, stored directions,
// FP64 orientation, edge signs.
__device__ __forceinline__ void tri_load_lds(const LRec& a, const LRec& b, const LRec& c, int N, int t, int key,
                                             int part, Tri<float>& T) {
  T.vid[0] = 0;
  T.vid[1] = t == 0 ? 1 : N + 1;
  T.vid[2] = t == 0 ? N + 1 : N;
  T.dv[0] = mk3<float>(a.dir[0], a.dir[1], a.dir[2]);
  T.dv[1] = mk3<float>(b.dir[0], b.dir[1], b.dir[2]);
  T.dv[2] = mk3<float>(c.dir[0], c.dir[1], c.dir[2]);
  T.rb = -1;
  T.part = part;
  T.N = N;
  T.key = key;
  v3<double> e1 = mk3<double>((double)T.dv[1].x - (double)T.dv[0].x, (double)T.dv[1].y - (double)T.dv[0].y,
                              (double)T.dv[1].z - (double)T.dv[0].z);
  v3<double> e2 = mk3<double>((double)T.dv[2].x - (double)T.dv[0].x, (double)T.dv[2].y - (double)T.dv[0].y,
                              (double)T.dv[2].z - (double)T.dv[0].z);
  double vol = dot(cross(e1, e2), cvt<double>(T.dv[0]));
  T.orient = vol > 0.0 ? 1 : (vol < 0.0 ? -1 : 0);
  for (int e = 0; e < 3; ++e) T.sig[e] = T.vid[(e + 1) % 3] < T.vid[(e + 2) % 3] ? 1 : -1;
}

// What one rasterisation phase of the fused kernel needs to know.
struct FusedStep {
  int N;          // rays per side
  int part;       // chunk particle
  int slot;       // order slot
  int col0;       // first ray column of the tile
  int row_top;    // grid row of the carry row (the step's first ray row - 1)
  int first;      // the step is the tile's first (no carry row)
  long nq;        // quads per order of the particle, (N - 1)^2
  int node0;      // the particle's first node in the chunk
};

// Contributions of the block's listed hits, one per thread: the triangle's
// three LDS records (rays from the key), the interpolation of hit_contrib,
// and a hit record in the wave's run of pool slots.  Every thread of the
// block calls it with the list's length n; it clears the list.
__device__ inline void fused_hits(FusedShared& sh, const LRec* carry, const NodeGrid& ng, const FusedPool& fp,
                                  const FusedStep& st, SlotRun& run, const int n) {
  const int tid = threadIdx.x, lane = tid & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int nq1 = st.N - 1;
  for (int base = 0; base < n; base += 256) {
    const int i = base + tid;
    const bool hit = i < n;
    const unsigned long long mask = __ballot(hit);
    if (mask == 0ull) continue;  // wave-uniform
    const unsigned nh = (unsigned)__popcll(mask);
    if (run.next + nh > run.end) {
      // a new run of slots, from the next partition (97 is odd: every
      // partition is reached, and they fill evenly)
      close_run(fp, run);
      run.part = (run.part + 97) % NPART;
      unsigned first = 0;
      if (lane == 0) first = atomicAdd(&fp.counter[run.part], (unsigned)FUSED_RUN);
      run.next = __shfl(first, 0);
      run.end = run.next + FUSED_RUN;
    }
    const unsigned pos = run.next + (unsigned)__popcll(mask & below);
    run.next += nh;
    if (lane == 0) atomicAdd(fp.n_hits, nh);
    if (!hit || pos >= (unsigned)fp.cap_part) continue;  // beyond: overflow, reported by the status call
    const HitEntry h = sh.hit[i];
    const int it = h.itip & 0xffff, ip = (int)((unsigned)h.itip >> 16);
    // the triangle's rays from its key (quad rows of the step: 0 .. 3)
    const int quad = (int)((long)(h.key >> 1) - (long)st.slot * st.nq);
    const int qy = quad / nq1, qx = quad - qy * nq1;
    const int qr = qy - st.row_top, qc = qx - st.col0;
    const LRec* ru = qr == 0 ? carry : sh.T[qr - 1];
    const LRec* rd = sh.T[qr];
    const int t = h.key & 1;
    const LRec& v0 = ru[qc];
    const LRec& v1 = t == 0 ? ru[qc + 1] : rd[qc + 1];
    const LRec& v2 = t == 0 ? rd[qc + 1] : rd[qc];
    float acc[2][2][2];
    double unused = 0.0;
    hit_contrib<float>(v0, v1, v2, ng, it, ip, fp.n_pol, h.lam, acc, false, 0.0, 0.0, 0.0, unused);
    const int node = st.node0 + it * ng.n_phi + ip;
    atomicAdd(&fp.count[node], 1);
    V4<float>* out = fp.hits + ((long)run.part * fp.cap_part + pos) * (1 + fp.n_pol);
    V4<float> h0;
    h0.x = __int_as_float(h.key); h0.y = __int_as_float(node); h0.z = 0.0f; h0.w = 0.0f;
    out[0] = h0;
    for (int p = 0; p < fp.n_pol; ++p) {
      V4<float> v;
      v.x = acc[p][0][0]; v.y = acc[p][0][1]; v.z = acc[p][1][0]; v.w = acc[p][1][1];
      out[1 + p] = v;
    }
  }
  __syncthreads();
  if (tid == 0) sh.n_hit = 0;
  __syncthreads();
}

// Rasterise the step's quads of one order slot and store their hits.  up[r]
// is ray row r of the step's five (the carry, then the four traced rows).
// Every thread of the block calls it (it holds block barriers).
__device__ inline void fused_raster(FusedShared& sh, const LRec* carry, const NodeGrid& ng, const AxisFast& axt,
                                    const AxisFast& axp, const FusedPool& fp, const FusedStep& st,
                                    const double margin, SlotRun& run) {
  BlockStage<float>& S = sh.S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = st.N;
  const int nq1 = N - 1;
  // quad (row `wave`, column `lane`) between step rows wave - 1 and wave
  const int gy = st.row_top + wave, gx = st.col0 + lane;
  const bool qok = lane < 63 && gx < nq1 && gy < nq1 && (wave > 0 || !st.first);
  const LRec* up = wave == 0 ? carry : sh.T[wave - 1];
  const LRec* dn = sh.T[wave];
  Cand c0, c1;
  bool need0 = false, need1 = false, fast0 = false, fast1 = false;
  if (qok) {
    const int f0 = up[lane].flags, f1 = up[lane + 1].flags, f2 = dn[lane].flags, f3 = dn[lane + 1].flags;
    const int nf0 = f0 >> 1 & 127;
    const bool tv0 = (f0 & 1) && (f1 & 1) && (f3 & 1) && nf0 == (f1 >> 1 & 127) && nf0 == (f3 >> 1 & 127);
    const bool tv1 = (f0 & 1) && (f2 & 1) && (f3 & 1) && nf0 == (f2 >> 1 & 127) && nf0 == (f3 >> 1 & 127);
    if (tv0 || tv1) {
      const float2 a00 = make_float2(up[lane].th, up[lane].ph), a01 = make_float2(up[lane + 1].th, up[lane + 1].ph);
      const float2 a10 = make_float2(dn[lane].th, dn[lane].ph), a11 = make_float2(dn[lane + 1].th, dn[lane + 1].ph);
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
  if (nq == 0) return;  // block-uniform: nothing to rasterise
  auto enqueue = [&](int at, int t, bool fast, const Cand& c) {
    TriQueued& e = S.queued[at];
    e.quad = wave << 8 | lane; e.part = 0; e.tf = t | (fast ? 2 : 0);
    e.i0 = c.i0; e.i1 = c.i1; e.ja0 = c.ja0; e.ja1 = c.ja1; e.jb0 = c.jb0; e.jb1 = c.jb1;
  };
  if (need0) enqueue(qbase + __popcll(q0 & below), 0, fast0, c0);
  if (need1) enqueue(qbase + nq0 + __popcll(q1 & below), 1, fast1, c1);
  __syncthreads();

  // queued triangles, two per thread at most: directions and orientation from
  // LDS, the direction box where the angle box did not apply, staged in slot k
  TriQueued mine[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
    if (256 * h + tid < nq) mine[h] = S.queued[256 * h + tid];
  __syncthreads();
  int block_total = 0;
  const int n_iter = nq > 256 ? 2 : 1;  // block-uniform
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h >= n_iter) break;
    const int k = 256 * h + tid;
    int n = 0;
    if (k < nq) {
      const TriQueued& e = mine[h];
      const int t = e.tf & 1, qr = e.quad >> 8, qc = e.quad & 255;
      const LRec* ru = qr == 0 ? carry : sh.T[qr - 1];
      const LRec* rd = sh.T[qr];
      const long quad = (long)(st.row_top + qr) * nq1 + (st.col0 + qc);
      const int key = (int)(((long)st.slot * st.nq + quad) * 2 + t);
      Tri<float> T;
      if (t == 0) tri_load_lds(ru[qc], ru[qc + 1], rd[qc + 1], N, 0, key, st.part, T);
      else tri_load_lds(ru[qc], rd[qc + 1], rd[qc], N, 1, key, st.part, T);
      if (T.orient != 0) {
        Cand c;
        if (e.tf & 2) {
          c.i0 = e.i0; c.i1 = e.i1; c.ja0 = e.ja0; c.ja1 = e.ja1; c.jb0 = e.jb0; c.jb1 = e.jb1;
        } else {
          c = box_cand(ng, tri_box(T, (float)margin));
        }
        n = c.count();
        if (n > 0) slot_put(S.tri[k], T, c);
      }
    }
    int it_total;
    const int ex = block_excl_scan(n, &it_total, S.wave_q);
    S.excl[k] = block_total + ex;
    block_total += it_total;
  }
  if (n_iter == 1) S.excl[256 + tid] = block_total;
  __syncthreads();

  // every staged candidate, 64 per wave at a time: membership; the hits go to
  // the block's LDS hit list, whose contributions are then formed with full
  // waves (fused_hits) after the pass
  const StageView<float> W = view(S);
  for (int base = 0; base < block_total; base += 256) {  // block-uniform passes
    const int g = base + 64 * wave + lane;
    bool hit = false;
    Tri<float> T;
    int it = 0, ip = 0;
    float lam[3];
    if (g < block_total) {
      locate(W, g, T, it, ip);
      hit = tri_member(T, node_dir_g<float>(ng, it, ip), lam);
    }
    const unsigned long long mask = __ballot(hit);
    if (mask != 0ull) {
      int first = 0;
      if (lane == 0) first = atomicAdd(&sh.n_hit, __popcll(mask));
      first = __shfl(first, 0);
      if (hit) {
        HitEntry& h = sh.hit[first + __popcll(mask & below)];
        h.key = T.key;
        h.itip = it | ip << 16;
        h.lam[0] = lam[0]; h.lam[1] = lam[1]; h.lam[2] = lam[2];
      }
    }
    __syncthreads();
    const int listed = sh.n_hit;
    __syncthreads();  // read by every thread before the next pass adds to it
    if (listed > 0) fused_hits(sh, carry, ng, fp, st, run, listed);
  }
}
// One thread per hit-pool slot of the fused kernel: the hit's key and
// contribution at the next place of its node's range (taken with an atomic
// on the node's range cursor, which starts at the range start from the scan
// and ends at the range end), the node-major layout k_node_sum reads.  The
// order within a node's range is free: k_node_sum orders the hits by key.
__global__ void __launch_bounds__(256) k_scatter(const FusedPool fp, const HitPool<float> pool) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long part = i / fp.cap_part;
  if (part >= NPART) return;
  const unsigned pos = (unsigned)(i - part * fp.cap_part);
  if (pos >= min(fp.counter[part], (unsigned)fp.cap_part)) return;
  const V4<float>* h = fp.hits + i * (1 + fp.n_pol);
  const V4<float> h0 = h[0];
  const int key = __float_as_int(h0.x), node = __float_as_int(h0.y);
  if (node < 0) return;  // an unused slot of a run
  const long at = (long)atomicAdd(&pool.cursor[node], 1);
  V4<float>* out = reinterpret_cast<V4<float>*>(pool.contrib + at * (fp.n_pol * 4));
  for (int p = 0; p < fp.n_pol; ++p) out[p] = h[1 + p];
  pool.key[at] = key;
}

}  // namespace rtw
