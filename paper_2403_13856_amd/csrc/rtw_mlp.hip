// rtw_mlp.hip -- the learned surrogate of the RTW far field on gfx950: an MLP
// 9 features -> fixed 23-wide embedding -> 512 (x6, GELU) -> 2 means + 2
// log-sigmas, BF16 weights and activations
// with FP32 accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16),
// trained with a Gaussian negative log-likelihood and Adam, queried with an
// RTW fallback wherever the predicted sigma exceeds the caller's threshold.
//
// Layouts (row-major): activations [rows][512] BF16; each layer keeps FP32
// master weights W[in][out], Adam moments, and two BF16 copies W[in][out]
// (for dX = dZ W^T) and W^T[out][in] (for Y = X W).  The 23 embedded inputs
// are padded to 128 and the 4 outputs to 128 columns (zero weights), so every
// product is a multiple of the 128 x 128 block tile.  Training runs the
// layers as separate products (k_gemm); inference runs them all in one
// kernel per tile of 128 queries with the activations in LDS (k_mlp_infer).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rtw_surrogate.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

thread_local std::string m_err;

int mfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  m_err = buf;
  return code;
}

constexpr int IN_RAW = RTW_SURROGATE_INPUTS;  // 9 features
constexpr int IN_EMB = RTW_SURROGATE_EMBED;   // fixed embedding of the features (first-layer inputs)
constexpr int IN_PAD = 128;
static_assert(IN_EMB <= IN_PAD, "embedding wider than the padded input");
constexpr int HID = RTW_SURROGATE_WIDTH;      // 512
constexpr int N_HIDDEN = RTW_SURROGATE_DEPTH; // 6 hidden layers
constexpr int N_LAYERS = N_HIDDEN + 1;
constexpr int OUT_RAW = 4;                    // mean x, mean y, log sigma x, log sigma y
constexpr float S_MIN = -9.2103404f;          // ln 1e-4: floor of the normalised log-sigma in the loss
constexpr int OUT_PAD = 128;

constexpr int layer_in(int l) { return l == 0 ? IN_PAD : HID; }
constexpr int layer_out(int l) { return l == N_LAYERS - 1 ? OUT_PAD : HID; }

// ---------------------------------------------------------------------------
// GEMM: C[M][N] = A(M x K) B(K x N) with an epilogue, BF16 operands, FP32
// accumulation.  A(m, k) = transA ? A[k lda + m] : A[m lda + k];
// B(k, n) = transB ? B[n ldb + k] : B[k ldb + n].  M, N multiples of 128,
// K a multiple of 32 (checked on the host).
// Block: 256 threads = 4 waves in 2 x 2, each wave 64 x 64 = 4 x 4 MFMA tiles
// of 16 x 16; K advances 32 per step through LDS tiles stored [row][k] with k
// contiguous (the operand layout of the instruction: lane l holds row l % 16,
// k = 8 (l / 16) .. + 7; the result holds rows 4 (l / 16) .. + 3, column
// l % 16).
// ---------------------------------------------------------------------------
constexpr int BM = 128, BN = 128, BK = 32, LDK = BK + 8;  // padded LDS row: 80 bytes
constexpr long GEMM_CUS = 256;  // compute units of the chip: the tile choice aims at >= 2 blocks each

enum Epi : int { EPI_FWD_GELU = 0, EPI_FWD_LINEAR = 1, EPI_BWD_GELU = 2, EPI_STORE_F32 = 3 };

struct GemmArgs {
  int M, N, K;
  int K_slice;         // K range of one blockIdx.z (split K); = K without splitting
  const bf16* A;
  long lda;
  int transA;
  const bf16* B;
  long ldb;
  int transB;
  long ldo;            // output row stride
  const float* bias;   // [N]            (forward)
  bf16* Zout;          // [M][N] BF16    (forward GELU: pre-activation)
  bf16* Aout;          // [M][N] BF16    (forward GELU: activation)
  float* Fout;         // [M][N] FP32    (forward linear, weight gradients)
  const bf16* Zin;     // [M][N] BF16    (backward: pre-activation of the layer below)
  bf16* Gout;          // [M][N] BF16    (backward: gradient w.r.t. that pre-activation)
  float* colsum;       // [splits][N] FP32 or null (weight gradients: column sums of B over each K
                       //                 slice, i.e. the bias gradient when B = dZ)
};

// GELU(z) = z Phi(z), Phi(z) = erfc(-z / sqrt 2) / 2, with erfc(u) for u >= 0
// from Abramowitz & Stegun 7.1.26 (erf to 1.5e-7 absolute):
//   erfc(u) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-u^2), t = 1 / (1 + p u),
// and erfc(-u) = 2 - erfc(u).  With the hardware reciprocal and exponential
// (about one ulp each) Phi stays within a few 1e-7, far below the BF16
// rounding the activations take, in about a third of the instructions of the
// library erff.  Training and inference share it.
__device__ __forceinline__ float phi_cdf(float z) {
  const float u = fabsf(z) * 0.70710678f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, u, 1.0f));
  const float poly =
      t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
  const float e = poly * __expf(-u * u);  // erfc(u)
  return z >= 0.f ? fmaf(-0.5f, e, 1.0f) : 0.5f * e;
}
__device__ __forceinline__ float gelu(float z) { return z * phi_cdf(z); }
__device__ __forceinline__ float gelu_grad(float z) { return phi_cdf(z) + z * 0.39894228f * __expf(-0.5f * z * z); }

// Global -> register staging of one K step of the A and B tiles (TM / 8 BF16
// of each per thread: NV = TM / 64 vectors of 8), and register -> LDS
// placement in the [row][k] layout.  Untransposed: 4 / NV threads a row, each
// NV vectors along k; transposed (k rows of TM): 8 threads a k row, each NV
// vectors along the row index.
template <int TM>
struct Stage {
  static constexpr int NV = TM / 64;
  bf16x8 a[NV], b[NV];
};

template <int TM>
__device__ __forceinline__ void stage_load(const GemmArgs& g, long m0, long n0, int k0, int t, Stage<TM>& r) {
  constexpr int NV = TM / 64, TPR = 4 / NV;
  if (!g.transA) {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(g.A + (m0 + t / TPR) * g.lda + k0 + (t % TPR) * NV * 8);
#pragma unroll
    for (int v = 0; v < NV; ++v) r.a[v] = src[v];
  } else {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(g.A + (long)(k0 + (t >> 3)) * g.lda + m0 + (t & 7) * NV * 8);
#pragma unroll
    for (int v = 0; v < NV; ++v) r.a[v] = src[v];
  }
  if (g.transB) {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(g.B + (n0 + t / TPR) * g.ldb + k0 + (t % TPR) * NV * 8);
#pragma unroll
    for (int v = 0; v < NV; ++v) r.b[v] = src[v];
  } else {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(g.B + (long)(k0 + (t >> 3)) * g.ldb + n0 + (t & 7) * NV * 8);
#pragma unroll
    for (int v = 0; v < NV; ++v) r.b[v] = src[v];
  }
}

template <int TM>
__device__ __forceinline__ void stage_store(const GemmArgs& g, int t, const Stage<TM>& r, bf16 (*As)[LDK],
                                            bf16 (*Bs)[LDK]) {
  constexpr int NV = TM / 64, TPR = 4 / NV;
  if (!g.transA) {
    const int row = t / TPR, kh = (t % TPR) * NV * 8;
#pragma unroll
    for (int v = 0; v < NV; ++v) *reinterpret_cast<bf16x8*>(&As[row][kh + 8 * v]) = r.a[v];
  } else {
    const int kk = t >> 3, mc = (t & 7) * NV * 8;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < 8; ++j) As[mc + 8 * v + j][kk] = r.a[v][j];
  }
  if (g.transB) {
    const int row = t / TPR, kh = (t % TPR) * NV * 8;
#pragma unroll
    for (int v = 0; v < NV; ++v) *reinterpret_cast<bf16x8*>(&Bs[row][kh + 8 * v]) = r.b[v];
  } else {
    const int kk = t >> 3, nc = (t & 7) * NV * 8;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < 8; ++j) Bs[nc + 8 * v + j][kk] = r.b[v][j];
  }
}

// Software-pipelined main loop: the next K step's tiles are loaded into
// registers while the matrix cores work on the current one from LDS, then
// placed into the other LDS buffer; one barrier per K step.  TM x TM block
// tiles (128, or 64 where 128 would leave the compute units short of blocks),
// 4 waves in 2 x 2, each (TM / 2)^2 = (TM / 32)^2 MFMA tiles.
template <int EPI, int TM>
__global__ void __launch_bounds__(256) k_gemm(const GemmArgs g) {
  static_assert(TM == 128 || (TM == 64 && EPI != EPI_STORE_F32), "64-wide tiles for the forward and backward products");
  constexpr int NT = TM / 32;  // MFMA tiles per wave and dimension
  __shared__ bf16 As[2][TM][LDK];
  __shared__ bf16 Bs[2][TM][LDK];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long m0 = (long)blockIdx.y * TM, n0 = (long)blockIdx.x * TM;
  f32x4 acc[NT][NT];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  float csum = 0.f;  // column sum of B over this block's K slice (weight-gradient products)
  const bool do_csum = EPI == EPI_STORE_F32 && g.colsum && blockIdx.y == 0;
  const int k_begin = blockIdx.z * g.K_slice, k_end = min(g.K, k_begin + g.K_slice);
  Stage<TM> r;
  stage_load<TM>(g, m0, n0, k_begin, t, r);
  stage_store<TM>(g, t, r, As[0], Bs[0]);
  __syncthreads();
  int cur = 0;
  for (int k0 = k_begin; k0 < k_end; k0 += BK) {
    const bool more = k0 + BK < k_end;
    if (more) stage_load<TM>(g, m0, n0, k0 + BK, t, r);
    if (do_csum) {
      // column sums of this K step of B, in a fixed order (two halves of k per column)
      const int n = t & 127, kh = (t >> 7) * 16;
#pragma unroll
      for (int j = 0; j < 16; ++j) csum += (float)Bs[cur][n][kh + j];
    }
    bf16x8 af[NT], bfr[NT];
    const int kq = 8 * (lane >> 4), rr = lane & 15;
#pragma unroll
    for (int i = 0; i < NT; ++i) af[i] = *reinterpret_cast<const bf16x8*>(&As[cur][wm * (TM / 2) + i * 16 + rr][kq]);
#pragma unroll
    for (int j = 0; j < NT; ++j) bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][wn * (TM / 2) + j * 16 + rr][kq]);
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    if (more) stage_store<TM>(g, t, r, As[cur ^ 1], Bs[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
  }
  if (do_csum) {
    float* red = reinterpret_cast<float*>(&As[cur][0][0]);  // no longer read
    red[t] = csum;
    __syncthreads();
    if (t < 128) g.colsum[(long)blockIdx.z * g.N + n0 + t] = red[t] + red[t + 128];
  }
  // epilogue
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int rr2 = 0; rr2 < 4; ++rr2) {
        const long row = m0 + wm * (TM / 2) + i * 16 + 4 * (lane >> 4) + rr2;
        const long col = n0 + wn * (TM / 2) + j * 16 + (lane & 15);
        const long o = row * g.ldo + col;
        const float v = acc[i][j][rr2];
        if (EPI == EPI_FWD_GELU) {
          const float z = v + g.bias[col];
          g.Zout[o] = (bf16)z;
          g.Aout[o] = (bf16)gelu(z);
        } else if (EPI == EPI_FWD_LINEAR) {
          g.Fout[o] = v + g.bias[col];
        } else if (EPI == EPI_BWD_GELU) {
          g.Gout[o] = (bf16)(v * gelu_grad((float)g.Zin[o]));
        } else {
          g.Fout[(long)blockIdx.z * g.M * g.ldo + o] = v;  // split-K partial
        }
      }
}

// ---------------------------------------------------------------------------
// Inference: every layer of a tile of MQ queries in one block, the activations
// held in LDS from the embedded inputs to the last hidden layer (they never
// reach HBM), the weights streamed from L2.  The products are the transposes
// of the GEMMs' (D[feature][query] = W^T(feature, k) X(query, k), weights as
// the instruction's A operand, activations as its B operand), so a lane's four
// accumulators are four consecutive features of one query: one 8-byte LDS
// store each after bias and GELU.  Every output element sums the same 32-wide
// products over the same k steps in the same order as k_gemm, with the same
// bias, GELU and BF16 rounding.  Wave w computes features [64 w, 64 w + 64) of
// every hidden layer for all MQ queries; the output layer's first 16 features
// (the four outputs and zero padding) go one query tile per wave.
// ---------------------------------------------------------------------------
constexpr int MQ = 128;                   // queries per block
constexpr int MLP_LDX = HID + 8;          // LDS row of one query's activations: 1040 bytes
constexpr int MLP_THREADS = 512;          // 8 waves
constexpr size_t MLP_LDS = (size_t)MQ * MLP_LDX * sizeof(bf16);
static_assert(MLP_THREADS / 64 * 64 == HID, "eight waves of 64 features cover a hidden layer");
static_assert(MLP_THREADS / 64 * 16 == MQ, "one query tile per wave in the output layer");

struct MlpWeights {
  const bf16* Wt[N_LAYERS];     // W^T[out][in] of each layer
  const float* bias[N_LAYERS];  // [out]
};

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(MLP_THREADS) k_mlp_infer(const bf16* X0, const MlpWeights P, float* out) {
  extern __shared__ __align__(16) unsigned char mlp_smem[];
  bf16(*X)[MLP_LDX] = reinterpret_cast<bf16(*)[MLP_LDX]>(mlp_smem);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const long q0 = (long)blockIdx.x * MQ;
  // the tile's embedded inputs, IN_PAD BF16 a query
  for (int i = t; i < MQ * IN_PAD / 8; i += MLP_THREADS) {
    const int r = i / (IN_PAD / 8), c = (i % (IN_PAD / 8)) * 8;
    *reinterpret_cast<bf16x8*>(&X[r][c]) = *reinterpret_cast<const bf16x8*>(X0 + (q0 + r) * IN_PAD + c);
  }
  __syncthreads();
  const int rr = lane & 15, kq = 8 * (lane >> 4);
  const int f0 = 64 * wave;
  for (int l = 0; l < N_HIDDEN; ++l) {
    const int K = layer_in(l);
    const bf16* W = P.Wt[l];
    f32x4 acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const bf16x8*>(W + (long)(f0 + 16 * i + rr) * K + kq);
    for (int k0 = 0; k0 < K; k0 += 32) {
      // the next k step's weight fragments are in flight during this one's products
      bf16x8 an[4];
      const int kn = k0 + 32 < K ? k0 + 32 : k0;
#pragma unroll
      for (int i = 0; i < 4; ++i) an[i] = *reinterpret_cast<const bf16x8*>(W + (long)(f0 + 16 * i + rr) * K + kn + kq);
      bf16x8 b[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&X[16 * j + rr][k0 + kq]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = an[i];
    }
    __syncthreads();  // every wave has read this layer's inputs
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int f = f0 + 16 * i + 4 * (lane >> 4);
      const float4 bb = *reinterpret_cast<const float4*>(P.bias[l] + f);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        bf16x4 v;
        v[0] = (bf16)gelu(acc[i][j][0] + bb.x);
        v[1] = (bf16)gelu(acc[i][j][1] + bb.y);
        v[2] = (bf16)gelu(acc[i][j][2] + bb.z);
        v[3] = (bf16)gelu(acc[i][j][3] + bb.w);
        *reinterpret_cast<bf16x4*>(&X[16 * j + rr][f]) = v;
      }
    }
    __syncthreads();
  }
  // output layer, features 0..15 of query tile `wave`
  {
    const bf16* W = P.Wt[N_LAYERS - 1];
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < HID; k0 += 32) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(W + (long)rr * HID + k0 + kq);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&X[16 * wave + rr][k0 + kq]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    const int f = 4 * (lane >> 4);
    const float4 bb = *reinterpret_cast<const float4*>(P.bias[N_LAYERS - 1] + f);
    float4 o;
    o.x = acc[0] + bb.x; o.y = acc[1] + bb.y; o.z = acc[2] + bb.z; o.w = acc[3] + bb.w;
    *reinterpret_cast<float4*>(out + (q0 + 16 * wave + rr) * OUT_PAD + f) = o;
  }
}

// ---------------------------------------------------------------------------
// element-wise kernels
// ---------------------------------------------------------------------------

// The fixed embedding of one feature row x = (b/a, c/a, ln k rbar, m, alpha,
// beta, gamma, theta, phi), angles in degrees, ZYZ Euler angles of the
// particle (lab = Rz(alpha) Ry(beta) Rz(gamma) body):
//   [0, 9)   (x - shift) / scale
//   [9, 21)  particle-frame unit vectors of the incident direction z, the two
//            polarisations x and y and the cell-centre direction s
//   [21, 23) cos phi, sin phi
// then BF16 and zero up to IN_PAD.  One thread per row.
__global__ void k_inputs(int n, int n_pad, const float* feats, const float* shift, const float* scale, bf16* X) {
  const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_pad) return;
  constexpr int E8 = (IN_EMB + 7) / 8 * 8;
  float e[E8];
#pragma unroll
  for (int c = 0; c < E8; ++c) e[c] = 0.0f;
  if (r < n) {
    const float* x = feats + r * IN_RAW;
#pragma unroll
    for (int c = 0; c < IN_RAW; ++c) e[c] = (x[c] - shift[c]) / scale[c];
    const float D2R = 0.017453292519943295f;
    float sa, ca, sb, cb, sg, cg, st, ct, sp, cp;
    sincosf(x[4] * D2R, &sa, &ca);
    sincosf(x[5] * D2R, &sb, &cb);
    sincosf(x[6] * D2R, &sg, &cg);
    sincosf(x[7] * D2R, &st, &ct);
    sincosf(x[8] * D2R, &sp, &cp);
    // rows of R: the particle-frame components of the lab axes
    const float R0[3] = {ca * cb * cg - sa * sg, -ca * cb * sg - sa * cg, ca * sb};
    const float R1[3] = {sa * cb * cg + ca * sg, -sa * cb * sg + ca * cg, sa * sb};
    const float R2[3] = {-sb * cg, sb * sg, cb};
    const float s0 = st * cp, s1 = st * sp, s2 = ct;
    float vz[3], vx[3], vy[3], vs[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      vz[i] = R2[i]; vx[i] = R0[i]; vy[i] = R1[i];
      vs[i] = s0 * R0[i] + s1 * R1[i] + s2 * R2[i];
      e[9 + i] = vz[i]; e[12 + i] = vx[i]; e[15 + i] = vy[i]; e[18 + i] = vs[i];
    }
    e[21] = cp; e[22] = sp;
  }
  bf16x8* dst = reinterpret_cast<bf16x8*>(X + r * IN_PAD);
#pragma unroll
  for (int c8 = 0; c8 < IN_PAD / 8; ++c8) {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = 8 * c8 + j < E8 ? (bf16)e[8 * c8 + j] : (bf16)0.0f;
    dst[c8] = v;
  }
}

// Loss of normalised targets y under N(mu, e^{2s}) per output pair, mean over
// rows < n and the two outputs: the beta-NLL of Seitzer et al. (ICLR 2022)
// with beta = 1, i.e. each element's Gaussian NLL 0.5 d^2 e^{-2s} + s
// (d = y - mu) weighted by w = e^{2s} held constant.  Its value is
// 0.5 d^2 + s w; its gradient is -d for mu (that of the squared error, so no
// small sigma can blow up the mean's step) and w - d^2 for s (stationary at
// sigma^2 = E d^2).  Writes the gradient w.r.t. the output pre-activations
// (zero in padded rows and columns) and per-block partial sums of the loss.
// The log-sigma enters as max(s, S_MIN) (sigma = 1e-4 in normalised units,
// far below the error bars of use); below the floor its gradient is zero.
__global__ void __launch_bounds__(256) k_nll(int n, int n_pad, const float* out, const float* targets,
                                             const float* t_shift, const float* t_scale, bf16* dZ, float* partial) {
  __shared__ float red[256];
  const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (r < n_pad) {
    float g[OUT_RAW] = {0.f, 0.f, 0.f, 0.f};
    if (r < n) {
      const float inv = 1.0f / (2.0f * (float)n);
      for (int o = 0; o < 2; ++o) {
        const float y = (targets[r * 2 + o] - t_shift[o]) / t_scale[o];
        const float mu = out[r * OUT_PAD + o], s_raw = out[r * OUT_PAD + 2 + o];
        const float s = fmaxf(s_raw, S_MIN);
        const float w = __expf(2.0f * s), d = y - mu;
        l += (0.5f * d * d + s * w) * inv;
        g[o] = -d * inv;
        g[2 + o] = s_raw > S_MIN ? (w - d * d) * inv : 0.0f;
      }
    }
    for (int c = 0; c < OUT_PAD; ++c) dZ[r * OUT_PAD + c] = (bf16)(c < OUT_RAW ? g[c] : 0.f);
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Ordered sum of the partial losses (one block).
__global__ void k_sum(const float* partial, int n, float* out) {
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = s;
  }
}

constexpr int DW_MAX_SPLITS = 32;  // split-K slices of a weight-gradient product

// Sum of split-K partial products [slices][n] in slice order.
__global__ void k_sum_slices(const float* part, int slices, long n, float* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int k = 0; k < slices; ++k) s += part[(long)k * n + i];
  out[i] = s;
}

// Adam on FP32 master parameters; refreshes the BF16 copies W[in][out] and
// W^T[out][in] of a weight matrix (rows = in, cols = out; none for biases).
__global__ void k_adam(float* w, float* m, float* v, const float* g, long n, float lr, float b1, float b2, float eps,
                       float c1, float c2, bf16* wb, bf16* wtb, int rows, int cols) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) {
    const long r = i / cols, c = i - r * cols;
    wb[i] = (bf16)wi;
    wtb[c * rows + r] = (bf16)wi;
  }
}

// BF16 copies of the master weights (after a host upload).
__global__ void k_to_bf16(const float* w, long n, bf16* wb, bf16* wtb, int rows, int cols) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long r = i / cols, c = i - r * cols;
  wb[i] = (bf16)w[i];
  wtb[c * rows + r] = (bf16)w[i];
}

// De-normalised predictions [n][4]: ln I_x, ln I_y, ln sigma_x, ln sigma_y
// (sigma of ln I).
__global__ void k_predict(int n, const float* out, const float* t_shift, const float* t_scale, float* pred) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int o = 0; o < 2; ++o) {
    pred[r * 4 + o] = out[(long)r * OUT_PAD + o] * t_scale[o] + t_shift[o];
    pred[r * 4 + 2 + o] = out[(long)r * OUT_PAD + 2 + o] + logf(t_scale[o]);
  }
}

// First index i in [0, n) with v[i] >= x (v ascending).
__device__ __forceinline__ int first_ge(const double* v, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (v[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ln of the mean over the nodes of each cell of a per-node intensity
// (inten [p][pol][node]), per particle and polarisation: out[p][cell][pol].
// Cell (tc, pc) holds the nodes with theta in [t0 + tc dt, t0 + (tc + 1) dt)
// and phi in [p0 + pc dp, ...).  One thread per output.
__global__ void k_cell_log_intensity(int n_part, const float* inten, int n_pol, int n_theta, const double* th,
                                     int n_phi, const double* ph, rtw_cells c, float* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n_cells = (long)c.n_theta_cells * c.n_phi_cells;
  const long n_out = (long)n_part * n_cells * n_pol;
  if (i >= n_out) return;
  const int pol = (int)(i % n_pol);
  const long cell = (i / n_pol) % n_cells;
  const long p = i / ((long)n_pol * n_cells);
  const int tc = (int)(cell / c.n_phi_cells), pc = (int)(cell - (long)tc * c.n_phi_cells);
  const int it0 = first_ge(th, n_theta, c.theta0_deg + tc * c.dtheta_deg);
  const int it1 = first_ge(th, n_theta, c.theta0_deg + (tc + 1) * c.dtheta_deg);
  const int ip0 = first_ge(ph, n_phi, c.phi0_deg + pc * c.dphi_deg);
  const int ip1 = first_ge(ph, n_phi, c.phi0_deg + (pc + 1) * c.dphi_deg);
  const float* I = inten + (p * n_pol + pol) * (long)n_theta * n_phi;
  double s = 0.0;
  int cnt = 0;
  for (int it = it0; it < it1; ++it)
    for (int ip = ip0; ip < ip1; ++ip) {
      s += (double)I[(long)it * n_phi + ip];
      ++cnt;
    }
  out[i] = cnt > 0 ? (float)log(fmax(s / cnt, 1e-30)) : 0.f;
}

__global__ void k_zero_int(int* p, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Queries whose sigma exceeds tau (either polarisation) use the fallback; the
// particle of such a query is marked.
__global__ void k_flag(int n, const float* pred, float log_tau, const int* q_part, int* used, int* need) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const bool fb = pred[r * 4 + 2] > log_tau || pred[r * 4 + 3] > log_tau;
  used[r] = fb ? 1 : 0;
  if (fb) need[q_part[r]] = 1;
}

// Final answers: surrogate means, or the RTW cell values of the re-computed
// particles (fb_slot[particle] = its index in the fallback batch).
__global__ void k_answer(int n, const float* pred, const int* used, const int* q_part, const int* q_cell,
                         const int* fb_slot, const float* cell_I, int n_cells, float* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int o = 0; o < 2; ++o) {
    float v = pred[r * 4 + o];
    if (used[r]) v = cell_I[((long)fb_slot[q_part[r]] * n_cells + q_cell[r]) * 2 + o];
    out[r * 2 + o] = v;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct rtw_surrogate {
  int max_rows;
  long step;
  float* master[N_LAYERS];  // W[in][out] FP32
  float* bias[N_LAYERS];    // [out] FP32
  float* mW[N_LAYERS];
  float* vW[N_LAYERS];
  float* mb[N_LAYERS];
  float* vb[N_LAYERS];
  float* gW[N_LAYERS];
  float* gb[N_LAYERS];
  bf16* Wb[N_LAYERS];   // [in][out]
  bf16* Wtb[N_LAYERS];  // [out][in]
  bf16* X0;             // [rows][IN_PAD]
  bf16* Z[N_HIDDEN];    // [rows][HID]
  bf16* A[N_HIDDEN];    // [rows][HID]
  bf16* dZa;            // [rows][HID] gradient buffers (ping-pong)
  bf16* dZb;
  bf16* dZout;          // [rows][OUT_PAD]
  float* out;           // [rows][OUT_PAD]
  float* partial;       // loss partial sums
  float* colpart;       // split-K partial bias gradients [DW_MAX_SPLITS][512]
  float* wpart;         // split-K partial weight gradients [DW_MAX_SPLITS][512][512]
  float* norm;          // feature shift[9], scale[9], target shift[2], scale[2]
  std::vector<void*> allocs;
};

namespace {

int dmalloc(rtw_surrogate* h, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) return mfail(RTW_ERR_DEVICE, "device allocation of %zu bytes failed", bytes);
  h->allocs.push_back(*p);
  return RTW_OK;
}

int gemm(int epi, GemmArgs g, hipStream_t st, int splits = 1, int* used_splits = nullptr) {
  if (g.M % BM || g.N % BN || g.K % BK) return mfail(RTW_ERR_INVALID_ARG, "gemm shape %d x %d x %d", g.M, g.N, g.K);
  const int steps = g.K / BK;
  splits = std::max(1, std::min(splits, steps));
  g.K_slice = (steps + splits - 1) / splits * BK;
  splits = (g.K + g.K_slice - 1) / g.K_slice;
  if (splits > 1 && epi != EPI_STORE_F32) return mfail(RTW_ERR_INVALID_ARG, "split K only for weight gradients");
  if (used_splits) *used_splits = splits;
  // 64-wide tiles where 128-wide ones would give fewer than two blocks a compute unit
  const bool small = epi != EPI_STORE_F32 && (long)(g.N / BN) * (g.M / BM) < 2L * GEMM_CUS;
  const int tm = small ? 64 : 128;
  dim3 grid(g.N / tm, g.M / tm, splits);
  switch (epi * 2 + (small ? 1 : 0)) {
    case 2 * EPI_FWD_GELU: hipLaunchKernelGGL((k_gemm<EPI_FWD_GELU, 128>), grid, dim3(256), 0, st, g); break;
    case 2 * EPI_FWD_GELU + 1: hipLaunchKernelGGL((k_gemm<EPI_FWD_GELU, 64>), grid, dim3(256), 0, st, g); break;
    case 2 * EPI_FWD_LINEAR: hipLaunchKernelGGL((k_gemm<EPI_FWD_LINEAR, 128>), grid, dim3(256), 0, st, g); break;
    case 2 * EPI_FWD_LINEAR + 1: hipLaunchKernelGGL((k_gemm<EPI_FWD_LINEAR, 64>), grid, dim3(256), 0, st, g); break;
    case 2 * EPI_BWD_GELU: hipLaunchKernelGGL((k_gemm<EPI_BWD_GELU, 128>), grid, dim3(256), 0, st, g); break;
    case 2 * EPI_BWD_GELU + 1: hipLaunchKernelGGL((k_gemm<EPI_BWD_GELU, 64>), grid, dim3(256), 0, st, g); break;
    default: hipLaunchKernelGGL((k_gemm<EPI_STORE_F32, 128>), grid, dim3(256), 0, st, g); break;
  }
  return RTW_OK;
}

GemmArgs gargs(int M, int N, int K) {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.M = M; g.N = N; g.K = K;
  return g;
}

// Forward pass of rows [0, n_pad) from X0; the output pre-activations land in h->out.
int forward(rtw_surrogate* h, int n_pad, hipStream_t st) {
  const bf16* x = h->X0;
  for (int l = 0; l < N_LAYERS; ++l) {
    GemmArgs g = gargs(n_pad, layer_out(l), layer_in(l));
    g.A = x; g.lda = layer_in(l); g.transA = 0;
    g.B = h->Wtb[l]; g.ldb = layer_in(l); g.transB = 1;
    g.ldo = layer_out(l);
    g.bias = h->bias[l];
    int rc;
    if (l < N_HIDDEN) {
      g.Zout = h->Z[l]; g.Aout = h->A[l];
      rc = gemm(EPI_FWD_GELU, g, st);
      x = h->A[l];
    } else {
      g.Fout = h->out;
      rc = gemm(EPI_FWD_LINEAR, g, st);
    }
    if (rc) return rc;
  }
  return RTW_OK;
}

// Forward pass for inference (no pre-activations kept): k_mlp_infer over the
// n_pad / MQ query tiles; the output pre-activations land in h->out (columns
// 0..15 written).
int infer(rtw_surrogate* h, int n_pad, hipStream_t st) {
  // the kernel's dynamic LDS beyond 64 KB, allowed once per device with that device current
  {
    static std::mutex mu;
    static bool set[64] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return mfail(RTW_ERR_DEVICE, "no current device");
    std::lock_guard<std::mutex> lk(mu);
    if (!set[dev]) {
      if (hipFuncSetAttribute((const void*)k_mlp_infer, hipFuncAttributeMaxDynamicSharedMemorySize, (int)MLP_LDS) !=
          hipSuccess)
        return mfail(RTW_ERR_DEVICE, "inference kernel needs %zu bytes of LDS", MLP_LDS);
      set[dev] = true;
    }
  }
  if (n_pad % MQ) return mfail(RTW_ERR_INVALID_ARG, "inference rows %d not a multiple of %d", n_pad, MQ);
  MlpWeights P;
  for (int l = 0; l < N_LAYERS; ++l) { P.Wt[l] = h->Wtb[l]; P.bias[l] = h->bias[l]; }
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)(n_pad / MQ)), dim3(MLP_THREADS), MLP_LDS, st, h->X0, P, h->out);
  return RTW_OK;
}

int upload_inputs(rtw_surrogate* h, int n, int n_pad, const float* feats, hipStream_t st) {
  hipLaunchKernelGGL(k_inputs, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0, st, n, n_pad, feats, h->norm,
                     h->norm + IN_RAW, h->X0);
  return RTW_OK;
}

int pad_rows(int n) { return (n + BM - 1) / BM * BM; }

// SplitMix64 (Steele, Lea, Flood 2014) for the seeded initialisation.
struct Mix {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

int refresh_bf16(rtw_surrogate* h, hipStream_t st) {
  for (int l = 0; l < N_LAYERS; ++l) {
    const long n = (long)layer_in(l) * layer_out(l);
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, h->master[l], n, h->Wb[l],
                       h->Wtb[l], layer_in(l), layer_out(l));
  }
  return RTW_OK;
}

}  // namespace

extern "C" {

const char* rtw_surrogate_last_error(void) { return m_err.c_str(); }

int rtw_surrogate_param_count(size_t* n) {
  if (!n) return mfail(RTW_ERR_INVALID_ARG, "NULL count");
  size_t c = 0;
  for (int l = 0; l < N_LAYERS; ++l) c += (size_t)layer_in(l) * layer_out(l) + layer_out(l);
  *n = c;
  return RTW_OK;
}

int rtw_surrogate_create(uint64_t seed, int max_rows, rtw_surrogate** out) {
  if (!out) return mfail(RTW_ERR_INVALID_ARG, "NULL handle");
  if (max_rows < 1 || max_rows > (1 << 22)) return mfail(RTW_ERR_INVALID_ARG, "max_rows must be in [1, 2^22]");
  rtw_surrogate* h = new rtw_surrogate();
  h->max_rows = pad_rows(max_rows);
  h->step = 0;
  const long R = h->max_rows;
  int rc = RTW_OK;
  auto A = [&](void** p, size_t b) { if (!rc) rc = dmalloc(h, p, b); };
  for (int l = 0; l < N_LAYERS; ++l) {
    const size_t nw = (size_t)layer_in(l) * layer_out(l), nb = layer_out(l);
    A((void**)&h->master[l], 4 * nw); A((void**)&h->bias[l], 4 * nb);
    A((void**)&h->mW[l], 4 * nw); A((void**)&h->vW[l], 4 * nw);
    A((void**)&h->mb[l], 4 * nb); A((void**)&h->vb[l], 4 * nb);
    A((void**)&h->gW[l], 4 * nw); A((void**)&h->gb[l], 4 * nb);
    A((void**)&h->Wb[l], 2 * nw); A((void**)&h->Wtb[l], 2 * nw);
  }
  A((void**)&h->X0, 2 * R * IN_PAD);
  for (int l = 0; l < N_HIDDEN; ++l) { A((void**)&h->Z[l], 2 * R * HID); A((void**)&h->A[l], 2 * R * HID); }
  A((void**)&h->dZa, 2 * R * HID); A((void**)&h->dZb, 2 * R * HID);
  A((void**)&h->dZout, 2 * R * OUT_PAD);
  A((void**)&h->out, 4 * R * OUT_PAD);
  A((void**)&h->partial, 4 * (R / 256 + 1));
  A((void**)&h->colpart, 4 * (size_t)DW_MAX_SPLITS * HID);
  A((void**)&h->wpart, 4 * (size_t)DW_MAX_SPLITS * HID * HID);
  A((void**)&h->norm, 4 * 22);
  if (rc) { rtw_surrogate_destroy(h); return rc; }
  // seeded initialisation: uniform(-b, b) with b = sqrt(6 / fan_in) (He, for GELU),
  // output layer scaled by 0.1; biases zero; padded input rows and output columns zero
  Mix mx{seed};
  std::vector<float> w, z;
  for (int l = 0; l < N_LAYERS; ++l) {
    const int fi = l == 0 ? IN_EMB : HID;
    const double b = std::sqrt(6.0 / fi) * (l == N_LAYERS - 1 ? 0.1 : 1.0);
    w.assign((size_t)layer_in(l) * layer_out(l), 0.f);
    for (int i = 0; i < layer_in(l); ++i)
      for (int o = 0; o < layer_out(l); ++o) {
        const double u = (2.0 * mx.uniform() - 1.0) * b;
        const bool live = (l > 0 || i < IN_EMB) && (l < N_LAYERS - 1 || o < OUT_RAW);
        w[(size_t)i * layer_out(l) + o] = live ? (float)u : 0.f;
      }
    z.assign(w.size(), 0.f);
    hipMemcpy(h->master[l], w.data(), 4 * w.size(), hipMemcpyHostToDevice);
    hipMemcpy(h->mW[l], z.data(), 4 * z.size(), hipMemcpyHostToDevice);
    hipMemcpy(h->vW[l], z.data(), 4 * z.size(), hipMemcpyHostToDevice);
    z.assign(layer_out(l), 0.f);
    hipMemcpy(h->bias[l], z.data(), 4 * z.size(), hipMemcpyHostToDevice);
    hipMemcpy(h->mb[l], z.data(), 4 * z.size(), hipMemcpyHostToDevice);
    hipMemcpy(h->vb[l], z.data(), 4 * z.size(), hipMemcpyHostToDevice);
  }
  float norm[22];
  for (int i = 0; i < IN_RAW; ++i) { norm[i] = 0.f; norm[IN_RAW + i] = 1.f; }
  norm[18] = norm[19] = 0.f;
  norm[20] = norm[21] = 1.f;
  hipMemcpy(h->norm, norm, sizeof(norm), hipMemcpyHostToDevice);
  refresh_bf16(h, nullptr);
  if (hipDeviceSynchronize() != hipSuccess) { rtw_surrogate_destroy(h); return mfail(RTW_ERR_DEVICE, "init failed"); }
  *out = h;
  return RTW_OK;
}

int rtw_surrogate_destroy(rtw_surrogate* h) {
  if (!h) return RTW_OK;
  hipDeviceSynchronize();
  for (void* p : h->allocs) hipFree(p);
  delete h;
  return RTW_OK;
}

int rtw_surrogate_set_normalization(rtw_surrogate* h, const float* feat_shift, const float* feat_scale,
                                    const float* target_shift, const float* target_scale) {
  if (!h || !feat_shift || !feat_scale || !target_shift || !target_scale)
    return mfail(RTW_ERR_INVALID_ARG, "NULL argument");
  float norm[22];
  for (int i = 0; i < IN_RAW; ++i) {
    if (!(feat_scale[i] > 0.f)) return mfail(RTW_ERR_INVALID_ARG, "feature scale %d must be positive", i);
    norm[i] = feat_shift[i];
    norm[IN_RAW + i] = feat_scale[i];
  }
  for (int o = 0; o < 2; ++o) {
    if (!(target_scale[o] > 0.f)) return mfail(RTW_ERR_INVALID_ARG, "target scale must be positive");
    norm[18 + o] = target_shift[o];
    norm[20 + o] = target_scale[o];
  }
  if (hipMemcpy(h->norm, norm, sizeof(norm), hipMemcpyHostToDevice) != hipSuccess)
    return mfail(RTW_ERR_DEVICE, "upload failed");
  return RTW_OK;
}

// Trained network to and from a file: magic "RTWS", format version, parameter
// count, the 22 normalisation floats, then the FP32 parameters (host byte order).
namespace {
constexpr uint32_t WEIGHTS_MAGIC = 0x53575452u;  // "RTWS"
constexpr uint32_t WEIGHTS_VERSION = 1;
}  // namespace

int rtw_surrogate_save(rtw_surrogate* h, const char* path) {
  if (!h || !path) return mfail(RTW_ERR_INVALID_ARG, "NULL argument");
  size_t n = 0;
  rtw_surrogate_param_count(&n);
  std::vector<float> par(n);
  int rc = rtw_surrogate_get_params(h, par.data(), n);
  if (rc) return rc;
  float norm[22];
  if (hipMemcpy(norm, h->norm, sizeof(norm), hipMemcpyDeviceToHost) != hipSuccess)
    return mfail(RTW_ERR_DEVICE, "normalisation read failed");
  FILE* f = std::fopen(path, "wb");
  if (!f) return mfail(RTW_ERR_INVALID_ARG, "cannot open %s for writing", path);
  const uint32_t head[2] = {WEIGHTS_MAGIC, WEIGHTS_VERSION};
  const uint64_t cnt = n;
  bool ok = std::fwrite(head, sizeof(head), 1, f) == 1 && std::fwrite(&cnt, sizeof(cnt), 1, f) == 1 &&
            std::fwrite(norm, sizeof(norm), 1, f) == 1 && std::fwrite(par.data(), sizeof(float), n, f) == n;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? RTW_OK : mfail(RTW_ERR_INVALID_ARG, "write to %s failed", path);
}

int rtw_surrogate_load(rtw_surrogate* h, const char* path) {
  if (!h || !path) return mfail(RTW_ERR_INVALID_ARG, "NULL argument");
  size_t n = 0;
  rtw_surrogate_param_count(&n);
  FILE* f = std::fopen(path, "rb");
  if (!f) return mfail(RTW_ERR_INVALID_ARG, "cannot open %s", path);
  uint32_t head[2] = {0, 0};
  uint64_t cnt = 0;
  float norm[22];
  std::vector<float> par(n);
  const bool ok = std::fread(head, sizeof(head), 1, f) == 1 && std::fread(&cnt, sizeof(cnt), 1, f) == 1 &&
                  head[0] == WEIGHTS_MAGIC && head[1] == WEIGHTS_VERSION && cnt == n &&
                  std::fread(norm, sizeof(norm), 1, f) == 1 && std::fread(par.data(), sizeof(float), n, f) == n;
  std::fclose(f);
  if (!ok) return mfail(RTW_ERR_INVALID_ARG, "%s is not a weights file of this network", path);
  int rc = rtw_surrogate_set_normalization(h, norm, norm + IN_RAW, norm + 18, norm + 20);
  if (rc) return rc;
  return rtw_surrogate_set_params(h, par.data(), n);
}

// Parameters in a fixed order, FP32: for each layer l = 0..6, W[in][out] then
// bias[out], with in = 128 for layer 0 (rows >= 23 unused) and out = 128 for
// the last layer (columns >= 4 unused).
int rtw_surrogate_get_params(rtw_surrogate* h, float* host, size_t n) {
  size_t need = 0;
  rtw_surrogate_param_count(&need);
  if (!h || !host || n < need) return mfail(RTW_ERR_INVALID_ARG, "need %zu floats", need);
  hipDeviceSynchronize();
  size_t off = 0;
  for (int l = 0; l < N_LAYERS; ++l) {
    const size_t nw = (size_t)layer_in(l) * layer_out(l);
    hipMemcpy(host + off, h->master[l], 4 * nw, hipMemcpyDeviceToHost);
    off += nw;
    hipMemcpy(host + off, h->bias[l], 4 * (size_t)layer_out(l), hipMemcpyDeviceToHost);
    off += layer_out(l);
  }
  return RTW_OK;
}

int rtw_surrogate_set_params(rtw_surrogate* h, const float* host, size_t n) {
  size_t need = 0;
  rtw_surrogate_param_count(&need);
  if (!h || !host || n < need) return mfail(RTW_ERR_INVALID_ARG, "need %zu floats", need);
  hipDeviceSynchronize();
  size_t off = 0;
  for (int l = 0; l < N_LAYERS; ++l) {
    const size_t nw = (size_t)layer_in(l) * layer_out(l);
    hipMemcpy(h->master[l], host + off, 4 * nw, hipMemcpyHostToDevice);
    off += nw;
    hipMemcpy(h->bias[l], host + off, 4 * (size_t)layer_out(l), hipMemcpyHostToDevice);
    off += layer_out(l);
  }
  refresh_bf16(h, nullptr);
  if (hipDeviceSynchronize() != hipSuccess) return mfail(RTW_ERR_DEVICE, "upload failed");
  return RTW_OK;
}

static int predict(rtw_surrogate* h, int n, const float* feats, float* pred, void* hip_stream, bool layered) {
  if (!h || !feats || !pred) return mfail(RTW_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || n > h->max_rows) return mfail(RTW_ERR_INVALID_ARG, "n must be in [1, %d]", h->max_rows);
  hipStream_t st = (hipStream_t)hip_stream;
  const int n_pad = pad_rows(n);
  int rc = upload_inputs(h, n, n_pad, feats, st);
  if (!rc) rc = layered ? forward(h, n_pad, st) : infer(h, n_pad, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_predict, dim3((n + 255) / 256), dim3(256), 0, st, n, h->out, h->norm + 18, h->norm + 20, pred);
  if (hipGetLastError() != hipSuccess) return mfail(RTW_ERR_DEVICE, "launch failed");
  return RTW_OK;
}

int rtw_surrogate_forward(rtw_surrogate* h, int n, const float* feats, float* pred, void* hip_stream) {
  return predict(h, n, feats, pred, hip_stream, false);
}

int rtw_surrogate_forward_layered(rtw_surrogate* h, int n, const float* feats, float* pred, void* hip_stream) {
  return predict(h, n, feats, pred, hip_stream, true);
}

int rtw_surrogate_grad(rtw_surrogate* h, int n, const float* feats, const float* targets, float* loss,
                       void* hip_stream);

int rtw_surrogate_train_step(rtw_surrogate* h, int n, const float* feats, const float* targets, float lr,
                             float* loss, void* hip_stream) {
  int rc = rtw_surrogate_grad(h, n, feats, targets, loss, hip_stream);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  h->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - std::pow(b1, (float)h->step), c2 = 1.f - std::pow(b2, (float)h->step);
  for (int l = 0; l < N_LAYERS; ++l) {
    const long nw = (long)layer_in(l) * layer_out(l), nb = layer_out(l);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, h->master[l], h->mW[l],
                       h->vW[l], h->gW[l], nw, lr, b1, b2, eps, c1, c2, h->Wb[l], h->Wtb[l], layer_in(l),
                       layer_out(l));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, h->bias[l], h->mb[l], h->vb[l],
                       h->gb[l], nb, lr, b1, b2, eps, c1, c2, (bf16*)nullptr, (bf16*)nullptr, 1, (int)nb);
  }
  if (hipGetLastError() != hipSuccess) return mfail(RTW_ERR_DEVICE, "launch failed");
  return RTW_OK;
}

// Loss and gradients (no update): forward, NLL, backward through all layers.
// Gradients are left in the handle (rtw_surrogate_get_grads).
int rtw_surrogate_grad(rtw_surrogate* h, int n, const float* feats, const float* targets, float* loss,
                       void* hip_stream) {
  if (!h || !feats || !targets || !loss) return mfail(RTW_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || n > h->max_rows) return mfail(RTW_ERR_INVALID_ARG, "n must be in [1, %d]", h->max_rows);
  hipStream_t st = (hipStream_t)hip_stream;
  const int n_pad = pad_rows(n);
  int rc = upload_inputs(h, n, n_pad, feats, st);
  if (!rc) rc = forward(h, n_pad, st);
  if (rc) return rc;
  const int nblk = n_pad / 256 + 1;
  hipLaunchKernelGGL(k_nll, dim3((unsigned)nblk), dim3(256), 0, st, n, n_pad, h->out, targets, h->norm + 18,
                     h->norm + 20, h->dZout, h->partial);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, st, h->partial, nblk, loss);
  const bf16* dz = h->dZout;
  bf16* bufs[2] = {h->dZa, h->dZb};
  for (int l = N_LAYERS - 1; l >= 0; --l) {
    const int in = layer_in(l), out = layer_out(l);
    const bf16* xin = l == 0 ? h->X0 : h->A[l - 1];
    // dW = X^T dZ  [in][out]
    GemmArgs g = gargs(in, out, n_pad);
    g.A = xin; g.lda = in; g.transA = 1;
    g.B = dz; g.ldb = out; g.transB = 0;
    g.ldo = out; g.Fout = h->wpart; g.colsum = h->colpart;
    // split the batch dimension so that the small weight matrix fills the
    // chip; the slices are added in a fixed order
    const int tiles = (in / BM) * (out / BN);
    const int splits = std::max(1, std::min(DW_MAX_SPLITS, 512 / tiles));
    int used = 1;
    if ((rc = gemm(EPI_STORE_F32, g, st, splits, &used))) return rc;
    const long nw = (long)in * out;
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, h->wpart, used, nw,
                       h->gW[l]);
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((out + 255) / 256)), dim3(256), 0, st, h->colpart, used,
                       (long)out, h->gb[l]);
    if (l > 0) {
      // dZ_{l-1} = (dZ W^T) * gelu'(Z_{l-1})
      bf16* dn = bufs[l & 1];
      GemmArgs b = gargs(n_pad, in, out);
      b.A = dz; b.lda = out; b.transA = 0;
      b.B = h->Wb[l]; b.ldb = out; b.transB = 1;
      b.ldo = in; b.Zin = h->Z[l - 1]; b.Gout = dn;
      if ((rc = gemm(EPI_BWD_GELU, b, st))) return rc;
      dz = dn;
    }
  }
  if (hipGetLastError() != hipSuccess) return mfail(RTW_ERR_DEVICE, "launch failed");
  return RTW_OK;
}

// Gradients of the last rtw_surrogate_grad / train_step, in the parameter order.
int rtw_surrogate_get_grads(rtw_surrogate* h, float* host, size_t n) {
  size_t need = 0;
  rtw_surrogate_param_count(&need);
  if (!h || !host || n < need) return mfail(RTW_ERR_INVALID_ARG, "need %zu floats", need);
  hipDeviceSynchronize();
  size_t off = 0;
  for (int l = 0; l < N_LAYERS; ++l) {
    const size_t nw = (size_t)layer_in(l) * layer_out(l);
    hipMemcpy(host + off, h->gW[l], 4 * nw, hipMemcpyDeviceToHost);
    off += nw;
    hipMemcpy(host + off, h->gb[l], 4 * (size_t)layer_out(l), hipMemcpyDeviceToHost);
    off += layer_out(l);
  }
  return RTW_OK;
}

int rtw_cell_log_intensity(int n_part, const float* intensity, int n_pol, const rtw_grid* grid, const rtw_cells* cells,
                           float* out, void* hip_stream) {
  if (!intensity || !grid || !cells || !out || n_part < 1 || (n_pol != 1 && n_pol != 2))
    return mfail(RTW_ERR_INVALID_ARG, "bad arguments");
  if (grid->n_theta < 1 || grid->n_phi < 1 || !grid->theta_deg || !grid->phi_deg)
    return mfail(RTW_ERR_INVALID_ARG, "empty node grid");
  if (cells->n_theta_cells < 1 || cells->n_phi_cells < 1 || !(cells->dtheta_deg > 0.0) || !(cells->dphi_deg > 0.0))
    return mfail(RTW_ERR_INVALID_ARG, "empty cell grid");
  hipStream_t st = (hipStream_t)hip_stream;
  const long n_out = (long)n_part * cells->n_theta_cells * cells->n_phi_cells * n_pol;
  hipLaunchKernelGGL(k_cell_log_intensity, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st, n_part,
                     intensity, n_pol, grid->n_theta, grid->theta_deg, grid->n_phi, grid->phi_deg, *cells,
                     out);
  if (hipGetLastError() != hipSuccess) return mfail(RTW_ERR_DEVICE, "launch failed");
  return RTW_OK;
}

int rtw_surrogate_features(int n_part, const rtw_particle* parts, const rtw_incident* inc, int n_cell,
                           const double* cell_theta_deg, const double* cell_phi_deg, float* feats) {
  if (n_part < 1 || !parts || !inc || n_cell < 1 || !cell_theta_deg || !cell_phi_deg || !feats)
    return mfail(RTW_ERR_INVALID_ARG, "bad arguments");
  if (!(inc->wavelength > 0.0)) return mfail(RTW_ERR_INVALID_ARG, "wavelength must be positive");
  if (inc->source_distance != 0.0) return mfail(RTW_ERR_UNSUPPORTED, "the surrogate models plane-wave incidence");
  if (inc->observation_radius != 0.0) return mfail(RTW_ERR_UNSUPPORTED, "the surrogate models the far field");
  const double k = 2.0 * 3.14159265358979323846 / inc->wavelength;
  for (int p = 0; p < n_part; ++p) {
    const double* s = parts[p].semi_axes;
    if (!(s[0] > 0 && s[1] > 0 && s[2] > 0)) return mfail(RTW_ERR_INVALID_ARG, "particle %d: bad semi-axes", p);
    if (parts[p].m_im != 0.0) return mfail(RTW_ERR_UNSUPPORTED, "particle %d: the surrogate models real indices", p);
    const double rbar = std::cbrt(s[0] * s[1] * s[2]);
    for (int c = 0; c < n_cell; ++c) {
      float* f = feats + ((size_t)p * n_cell + c) * IN_RAW;
      f[0] = (float)(s[1] / s[0]);
      f[1] = (float)(s[2] / s[0]);
      f[2] = (float)std::log(k * rbar);
      f[3] = (float)parts[p].m;
      f[4] = (float)parts[p].euler_deg[0];
      f[5] = (float)parts[p].euler_deg[1];
      f[6] = (float)parts[p].euler_deg[2];
      f[7] = (float)cell_theta_deg[c];
      f[8] = (float)cell_phi_deg[c];
    }
  }
  return RTW_OK;
}

namespace {
size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr double FALLBACK_HITS_PER_NODE = 12.0;  // generous hit-pool sizing of the fallback batch
}

int rtw_surrogate_query_scratch_size(int n_part, const rtw_particle* parts, const int* grid_n,
                                     const rtw_incident* inc, const rtw_trace_opts* opts, const rtw_grid* grid,
                                     const rtw_cells* cells, size_t* bytes) {
  if (!bytes || !cells || !grid) return mfail(RTW_ERR_INVALID_ARG, "NULL argument");
  size_t ws = 0;
  const rtw_batch_opts bo{0, FALLBACK_HITS_PER_NODE};
  int rc = rtw_batch_workspace_size(n_part, parts, grid_n, inc, opts, grid, &bo, &ws);
  if (rc) return mfail(rc, "%s", rtw_last_error());
  const size_t n_cells = (size_t)cells->n_theta_cells * cells->n_phi_cells;
  const size_t nodes = (size_t)grid->n_theta * grid->n_phi;
  *bytes = 256 + a256(8 * (size_t)n_part) + a256(sizeof(float) * n_part * n_cells * 2) + a256(ws) +
           a256((size_t)n_part * 2 * 2 * nodes * 2 * sizeof(float)) + (size_t)n_part * 2 * nodes * sizeof(float);
  return RTW_OK;
}

int rtw_surrogate_query(rtw_surrogate* h, int n_query, const float* feats, const int32_t* q_part,
                        const int32_t* q_cell, float tau, int n_part, const rtw_particle* parts, const int* grid_n,
                        const rtw_incident* inc, const rtw_trace_opts* opts, const rtw_grid* grid,
                        const rtw_cells* cells, const rtw_tune* tune, float* pred, float* answer,
                        int32_t* used_fallback, void* scratch, size_t scratch_bytes, int* n_recomputed,
                        void* hip_stream) {
  if (!h || !feats || !q_part || !q_cell || !parts || !grid_n || !inc || !opts || !grid || !cells || !pred ||
      !answer || !used_fallback || !scratch)
    return mfail(RTW_ERR_INVALID_ARG, "NULL argument");
  if (n_query < 1 || n_part < 1) return mfail(RTW_ERR_INVALID_ARG, "need queries and particles");
  if (!(tau > 0.f)) return mfail(RTW_ERR_INVALID_ARG, "tau must be positive");
  if (opts->precision != RTW_MIXED || inc->n_pol != 2)
    return mfail(RTW_ERR_UNSUPPORTED, "the fallback runs the mixed path with two polarisations");
  if (inc->source_distance != 0.0) return mfail(RTW_ERR_UNSUPPORTED, "the surrogate models plane-wave incidence");
  if (inc->observation_radius != 0.0) return mfail(RTW_ERR_UNSUPPORTED, "the surrogate models the far field");
  size_t need_bytes = 0;
  int rc = rtw_surrogate_query_scratch_size(n_part, parts, grid_n, inc, opts, grid, cells, &need_bytes);
  if (rc) return rc;
  if (scratch_bytes < need_bytes) return mfail(RTW_ERR_WORKSPACE, "query needs %zu scratch bytes", need_bytes);
  hipStream_t st = (hipStream_t)hip_stream;
  const int n_cells = cells->n_theta_cells * cells->n_phi_cells;
  char* base = (char*)(((uintptr_t)scratch + 255) & ~(uintptr_t)255);
  int* need = (int*)base;
  int* dslot = need + n_part;
  float* cellI = (float*)(base + a256(8 * (size_t)n_part));
  char* ws = (char*)cellI + a256(sizeof(float) * (size_t)n_part * n_cells * 2);
  // 1. surrogate, in chunks of the handle's row capacity
  for (int q0 = 0; q0 < n_query; q0 += h->max_rows) {
    const int nq = std::min(h->max_rows, n_query - q0);
    rc = rtw_surrogate_forward(h, nq, feats + (size_t)q0 * IN_RAW, pred + (size_t)q0 * 4, hip_stream);
    if (rc) return rc;
  }
  // 2. which particles need the RTW answer
  hipLaunchKernelGGL(k_zero_int, dim3((n_part + 255) / 256), dim3(256), 0, st, need, (long)n_part);
  hipLaunchKernelGGL(k_flag, dim3((n_query + 255) / 256), dim3(256), 0, st, n_query, pred, std::log(tau), q_part,
                     used_fallback, need);
  std::vector<int> hneed(n_part);
  hipMemcpyAsync(hneed.data(), need, sizeof(int) * (size_t)n_part, hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) return mfail(RTW_ERR_DEVICE, "surrogate pass failed");
  std::vector<rtw_particle> fp;
  std::vector<int> fg, slot(n_part, 0);
  for (int p = 0; p < n_part; ++p)
    if (hneed[p]) { slot[p] = (int)fp.size(); fp.push_back(parts[p]); fg.push_back(grid_n[p]); }
  if (n_recomputed) *n_recomputed = (int)fp.size();
  hipMemcpyAsync(dslot, slot.data(), sizeof(int) * (size_t)n_part, hipMemcpyHostToDevice, st);
  // 3. RTW for those particles.  The batch workspace is not monotone in the
  // particle set (a subset can group into chunks that need more than the whole
  // set), so each batch is checked against the scratch left after the cell
  // values and split in halves until it fits; one particle always fits, its
  // workspace being at most that of the whole set the scratch was sized for.
  // A batch whose hit pool overflows is run again with twice the pool per
  // node where that fits the scratch, else split.
  const size_t avail = scratch_bytes - (size_t)(ws - (char*)scratch);
  const size_t nodes = (size_t)grid->n_theta * grid->n_phi;
  struct Piece {
    int first, count;
    double hits_per_node;
  };
  std::vector<Piece> todo;  // ranges of fp
  if (!fp.empty()) todo.push_back({0, (int)fp.size(), FALLBACK_HITS_PER_NODE});
  auto fits = [&](int f0, int nf, double hpn, size_t* wsb_out) -> int {
    const rtw_batch_opts b{0, hpn};
    size_t wsb = 0;
    const int r = rtw_batch_workspace_size(nf, fp.data() + f0, fg.data() + f0, inc, opts, grid, &b, &wsb);
    if (r) return -1;
    *wsb_out = a256(wsb);
    const size_t ffb = a256((size_t)nf * 2 * 2 * nodes * 2 * sizeof(float));
    return *wsb_out + ffb + (size_t)nf * 2 * nodes * sizeof(float) <= avail ? 1 : 0;
  };
  while (!todo.empty()) {
    const Piece pc = todo.back();
    todo.pop_back();
    const int f0 = pc.first, nf = pc.count;
    size_t wsb = 0;
    const int fit = fits(f0, nf, pc.hits_per_node, &wsb);
    if (fit < 0) return mfail(RTW_ERR_INVALID_ARG, "%s", rtw_last_error());
    if (!fit) {
      if (nf == 1) return mfail(RTW_ERR_WORKSPACE, "fallback particle does not fit the query scratch");
      todo.push_back({f0 + nf / 2, nf - nf / 2, pc.hits_per_node});
      todo.push_back({f0, nf / 2, pc.hits_per_node});
      continue;
    }
    const rtw_batch_opts bo{0, pc.hits_per_node};
    const size_t ffb = a256((size_t)nf * 2 * 2 * nodes * 2 * sizeof(float));
    char* ff = ws + wsb;
    float* incoh = (float*)(ff + ffb);
    rc = rtw_batch(nf, fp.data() + f0, fg.data() + f0, inc, opts, grid, ff, nullptr, incoh, tune, &bo, ws, wsb,
                   hip_stream);
    if (!rc) rc = rtw_farfield_status(ws, hip_stream, nullptr);
    if (rc == RTW_ERR_WORKSPACE) {  // hit pool overflow: a larger pool, or halves
      size_t w2 = 0;
      if (pc.hits_per_node < 1e4 && fits(f0, nf, 2.0 * pc.hits_per_node, &w2) == 1) {
        todo.push_back({f0, nf, 2.0 * pc.hits_per_node});
        continue;
      }
      if (nf > 1) {
        todo.push_back({f0 + nf / 2, nf - nf / 2, pc.hits_per_node});
        todo.push_back({f0, nf / 2, pc.hits_per_node});
        continue;
      }
    }
    if (rc) return mfail(rc, "fallback: %s", rtw_last_error());
    rc = rtw_cell_log_intensity(nf, incoh, 2, grid, cells, cellI + (size_t)f0 * n_cells * 2, hip_stream);
    if (rc) return rc;
  }
  // 4. answers (dslot was uploaded synchronously before its first use by hipMemcpyAsync ordering)
  hipLaunchKernelGGL(k_answer, dim3((n_query + 255) / 256), dim3(256), 0, st, n_query, pred, used_fallback, q_part,
                     q_cell, dslot, cellI, n_cells, answer);
  if (hipGetLastError() != hipSuccess) return mfail(RTW_ERR_DEVICE, "launch failed");
  if (hipStreamSynchronize(st) != hipSuccess) return mfail(RTW_ERR_DEVICE, "query failed");
  return RTW_OK;
}

}  // extern "C"
