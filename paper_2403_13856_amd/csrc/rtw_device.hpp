// rtw_device.hpp -- device-side building blocks of the RTW hot path on gfx950.
//
// One thread traces one incident ray through the ellipsoid (Ren et al., Ray
// Theory of Waves): at each interaction the incidence-plane basis is formed,
// the carried state is rotated into it, vector Snell (Eq. 4) gives both
// outgoing directions, Eq. 8 the Fresnel coefficients, and the wavefront
// equation (Eq. 3) the WFC of both branches.  With the surface basis chosen
// as (e_perp, n x e_perp) both projection matrices of Eq. 3 are diagonal,
// diag(1, n.k_hat), so the equation reduces to a handful of multiply-adds.
//
// Precision policy (template parameter G = type of the wave quantities):
//   G = double : every step in FP64.
//   G = float  : Fresnel coefficients, Jones matrix and the emitted fields in
//                FP32; the polyline (positions, directions, normals, Snell),
//                chord lengths, optical path, phase reduction, the
//                wavefront-curvature recursion, the divergence product and the
//                propagation Jacobian I + L Q (which vanishes at caustics) stay
//                in FP64.  Records and the far-field assembly are FP32.  An
//                FP64 FMA issues at the rate of an unpacked FP32 one on this
//                chip, so the curvature costs registers, not time, in FP64,
//                while in FP32 its rounding, amplified where det(I + L Q)
//                cancels, sent 15% of the rays to an FP64 re-trace.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtw {

// ---------------------------------------------------------------------------
// scalar helpers with one spelling for both precisions
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rsq(float x) { return __frsqrt_rn(x); }

// FP64 1 / b and 1 / sqrt(x) from the hardware estimates refined by two
// Newton steps (each squares the relative error: a few ulp from the estimate,
// about one ulp after them), cheaper than IEEE division and square root.
// Where the estimate is infinite or zero (b = 0, x = 0, infinities) it is
// returned as is, so that those cases give what 1 / b and 1 / sqrt(x) give.
__device__ __forceinline__ double rcp_d(double b) {
  double r = __builtin_amdgcn_rcp(b);
  if (!(fabs(r) < 1.79e308) || r == 0.0) return r;
  double e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  e = fma(-b, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsq_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
  if (!(fabs(y) < 1.79e308) || y == 0.0) return y;
  const double h = 0.5 * x;
  double e = fma(-h * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsq(double x) { return rsq_d(x); }
// sqrt(x) = x / sqrt(x) for x >= 0 from rsq_d (0 for x = 0)
__device__ __forceinline__ double sqrt_d(double x) { return x > 0.0 ? x * rsq_d(x) : 0.0; }
// 1 / x of the wave quantities: the hardware reciprocal in FP32 (1 ulp; the
// arguments here are normal numbers of order 1 to 10), rcp_d in FP64
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return rcp_d(x); }
__device__ __forceinline__ float sqr_t(float x) { return __fsqrt_rn(x); }
__device__ __forceinline__ double sqr_t(double x) { return sqrt(x); }
__device__ __forceinline__ void sincos_t(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_t(double x, double* s, double* c) { sincos(x, s, c); }

// sin and cos of an FP32 angle already reduced to about [-pi, pi] (a phase
// reduced modulo 2 pi): quadrant j = rint(2 x / pi), r = x - j pi / 2 with pi / 2
// in two parts (j pi_hi is exact for |j| <= 4, so r is exact but for the
// last rounding), then the Taylor series of sin to r^9 and cos to r^10 on
// |r| <= pi / 4 (truncation below 2e-9) and the quadrant's signs and swap:
// about a fifth of the instructions of the general sincosf, to ~1 ulp.
__device__ __forceinline__ void sincos_red(float x, float* s, float* c) {
  const float j = rintf(x * 0.63661977236758134f);
  float r = fmaf(-j, 1.57079637050628662f, x);   // pi / 2 rounded to FP32
  r = fmaf(-j, -4.37113900018624284e-8f, r);     // pi / 2 minus that
  const float r2 = r * r;
  const float sr = fmaf(r * r2, fmaf(r2, fmaf(r2, fmaf(r2, 2.75573192e-6f, -1.98412698e-4f), 8.33333333e-3f),
                                     -1.66666667e-1f), r);
  const float cr = fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -2.75573192e-7f, 2.48015873e-5f), -1.38888889e-3f),
                                          4.16666667e-2f), -0.5f), 1.0f);
  const int q = (int)j & 3;
  const float ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}
__device__ __forceinline__ void sincos_red(double x, double* s, double* c) { sincos(x, s, c); }

// atan2(y, x) in FP32, within a few 1e-7 rad: a = min / max of |x|, |y|; above
// tan(pi / 12), atan a = pi / 6 + atan t with t = (a sqrt 3 - 1) / (a + sqrt 3),
// so |t| <= tan(pi / 12) and the Taylor series of atan to t^11 leaves below
// 2e-9; then the octant and the quadrant.  atan2(0, 0) = 0.
// q / d for 0 <= q, 1 <= d, q + d < 2^31 and a quotient below 2^15 (grid
// indices: ray or quad -> row, key offset -> order slot).  q and d rounded to
// FP32, the hardware reciprocal (1 ulp) and the product put the estimate
// within a few 2^-24 relative of q / d, i.e. within 2^-7 for such quotients,
// so the truncated estimate is off by at most one and one correction step
// makes it exact (checked with the reciprocal 2 ulp off either way).  It
// replaces an integer division sequence several times as long.
__device__ __forceinline__ int div_quot15(int q, int d) {
  int r = (int)((float)q * __builtin_amdgcn_rcpf((float)d));
  if (r * d > q) --r;
  else if ((r + 1) * d <= q) ++r;
  return r;
}

__device__ __forceinline__ float atan2_f32(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float a = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  const bool big = a > 0.267949192f;  // tan(pi / 12)
  const float t = big ? (a * 1.73205081f - 1.0f) * __builtin_amdgcn_rcpf(a + 1.73205081f) : a;
  const float t2 = t * t;
  float p = fmaf(t * t2, fmaf(t2, fmaf(t2, fmaf(t2, fmaf(t2, -9.09090909e-2f, 1.11111111e-1f), -1.42857143e-1f),
                                       2.0e-1f), -3.33333333e-1f), t);
  if (big) p += 0.523598776f;                  // pi / 6
  if (ay > ax) p = 1.57079633f - p;            // pi / 2 - atan(1 / a)
  if (x < 0.0f) p = 3.14159265f - p;
  return copysignf(p, y);
}

template <typename T>
struct v3 {
  T x, y, z;
};
template <typename T>
__host__ __device__ __forceinline__ v3<T> mk3(T x, T y, T z) {
  v3<T> r;
  r.x = x; r.y = y; r.z = z;
  return r;
}
template <typename T>
__host__ __device__ __forceinline__ T dot(const v3<T>& a, const v3<T>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__host__ __device__ __forceinline__ v3<T> cross(const v3<T>& a, const v3<T>& b) {
  return mk3<T>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <typename T>
__device__ __forceinline__ v3<T> axpy(T s, const v3<T>& a, const v3<T>& b) {  // s a + b
  return mk3<T>(s * a.x + b.x, s * a.y + b.y, s * a.z + b.z);
}
template <typename T>
__host__ __device__ __forceinline__ v3<T> scl(T s, const v3<T>& a) {
  return mk3<T>(s * a.x, s * a.y, s * a.z);
}
template <typename T, typename U>
__device__ __forceinline__ v3<T> cvt(const v3<U>& a) {
  return mk3<T>((T)a.x, (T)a.y, (T)a.z);
}

template <typename T>
struct cx {
  T re, im;
};
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  cx<T> r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  T den = b.re * b.re + b.im * b.im;
  cx<T> r;
  r.re = (a.re * b.re + a.im * b.im) / den;
  r.im = (a.im * b.re - a.re * b.im) / den;
  return r;
}

// ---------------------------------------------------------------------------
// per-particle constants, prepared on the host
// ---------------------------------------------------------------------------
struct ParticleConst {
  double A[3];   // 1/a^2, 1/b^2, 1/c^2
  double R[9];   // body -> lab rotation, row-major
  double k;      // 2 pi / lambda
  double m;      // relative index (real part)
  double m_im;   // its imaginary part: attenuation exp(-k m_im L) per internal segment
  double L, h;   // grid half-width and ray spacing (um)
  int N;         // rays per side
  int p_min, p_max, n_pol;
  double amplif_limit;  // mixed path: FP64 re-trace above this error amplification
  double zs;     // point-source distance on the lab -z axis (um); 0: plane wave
  double robs;   // observation radius (um); 0: far field
};

// Phase a wave leaving the exit point r (kr = k r) gains between the
// directions x and y: in the far field (kappa = 0) kr.(x - y); on the
// observation sphere of radius R (kappa = k R) |kappa y' - kr| -
// |kappa x' - kr| between its points R x' and R y' in those directions
// (x' = x / |x|: a direction rounded to FP32 names the point of the sphere
// along it), formed as kr.(x' - y') 2 kappa / (|kappa y' - kr| + |kappa x' - kr|),
// the same difference of squares over the sum, without the cancellation of
// the plain difference (exact for unit x', y', also where one distance vanishes).
__device__ __forceinline__ double near_carry(double kappa, double krx, double kry, double krz, double xx, double xy,
                                             double xz, double yx, double yy, double yz) {
  if (kappa == 0.0) return krx * (xx - yx) + kry * (xy - yy) + krz * (xz - yz);
  const double sx = rsq_d(xx * xx + xy * xy + xz * xz), sy = rsq_d(yx * yx + yy * yy + yz * yz);
  xx *= sx; xy *= sx; xz *= sx;
  yx *= sy; yy *= sy; yz *= sy;
  const double ax = kappa * yx - krx, ay = kappa * yy - kry, az = kappa * yz - krz;
  const double bx = kappa * xx - krx, by = kappa * xy - kry, bz = kappa * xz - krz;
  return (krx * (xx - yx) + kry * (xy - yy) + krz * (xz - yz)) * 2.0 * kappa /
         (sqrt(ax * ax + ay * ay + az * az) + sqrt(bx * bx + by * by + bz * bz));
}

// Two-constant Cody-Waite reduction of x modulo 2 pi in FP64 (Cody & Waite,
// Software Manual for the Elementary Functions, 1980).  TWO_PI_HI keeps 31
// significant bits, so n * TWO_PI_HI is exact for |n| < 2^22 (|x| < 2.6e7 rad).
__device__ __forceinline__ double reduce_2pi(double x) {
  const double INV_TWO_PI = 0.15915494309189535;
  const double TWO_PI_HI = 6.2831853069365025;
  const double TWO_PI_LO = 2.430840202602477e-10;
  double n = rint(x * INV_TWO_PI);
  return (x - n * TWO_PI_HI) - n * TWO_PI_LO;
}

// Ai(-z) and Ai'(-z) for z >= 0 (FP64).  Up to z = 10 the Airy equation
// y'' = x y is marched from x = 0 (Ai(0) = 3^(-2/3) / Gamma(2/3), Ai'(0) =
// -3^(-1/3) / Gamma(1/3), Abramowitz & Stegun 10.4.4-5) to x = -z in equal
// steps of at most 1/2, each by its Taylor series about the current point,
// whose coefficients follow from (j + 2)(j + 1) a_{j+2} = x0 a_j + a_{j-1};
// from z = 10 on, the asymptotic expansions A&S 10.4.60 and 10.4.62 in
// xi = (2/3) z^{3/2} (their twelfth term is below 1e-13 there).
__device__ inline void airy_neg(double z, double& ai, double& aip) {
  if (z < 10.0) {
    double y = 0.35502805388781723926, yp = -0.25881940379280679840;
    const int n = (int)ceil(2.0 * z);
    const double h = n > 0 ? -z / n : 0.0;
    double x0 = 0.0;
    for (int s = 0; s < n; ++s) {
      double am1 = 0.0, a0 = y, a1 = yp;  // a_{j-1}, a_j, a_{j+1} for j = 0
      double py = a0, pyp = a1, hp = 1.0;   // sums of a_j h^j and (j + 1) a_{j+1} h^j
      for (int j = 0; j < 48; ++j) {
        const double a2 = (x0 * a0 + am1) / ((double)(j + 2) * (double)(j + 1));
        hp *= h;
        py += a1 * hp;
        pyp += (double)(j + 2) * a2 * hp;
        am1 = a0; a0 = a1; a1 = a2;
      }
      y = py;
      yp = pyp;
      x0 += h;
    }
    ai = y;
    aip = yp;
    return;
  }
  const double xi = (2.0 / 3.0) * z * sqrt(z);
  const double ixi = 1.0 / xi;
  // c_k of Ai (d_k of Ai' = -(6k + 1) / (6k - 1) c_k), summed as the alternating
  // even and odd series of both
  double c = 1.0, pw = 1.0, se = 0.0, so = 0.0, de = 0.0, dd = 0.0;
  for (int k = 0; k < 12; ++k) {
    if (k > 0) c *= (6.0 * k - 5.0) * (6.0 * k - 3.0) * (6.0 * k - 1.0) / ((2.0 * k - 1.0) * 216.0 * k);
    const double d = k > 0 ? -c * (6.0 * k + 1.0) / (6.0 * k - 1.0) : 1.0;
    const double sg = (k & 2) ? -1.0 : 1.0;
    if (k & 1) { so += sg * c * pw; dd += sg * d * pw; }
    else { se += sg * c * pw; de += sg * d * pw; }
    pw *= ixi;
  }
  double sn, cs;
  sincos(xi + 0.78539816339744830962, &sn, &cs);
  const double q = sqrt(sqrt(z)), isp = 0.56418958354775628695;  // z^{1/4}, 1/sqrt(pi)
  ai = isp / q * (sn * se - cs * so);
  aip = -isp * q * (cs * de + sn * dd);
}

// J1(x), FP64: below 25, downward recurrence J_{n-1} = (2n / x) J_n - J_{n+1}
// from a start far above x (Miller), normalised by J_0 + 2 sum J_{2m} = 1;
// from 25 on, Hankel's asymptotic expansion (A&S 9.2.5 with 9.2.9-10), 14 terms.
__device__ inline double bessel_j1(double x) {
  const double ax = fabs(x);
  if (ax < 1e-8) return 0.5 * x;
  double r;
  if (ax < 25.0) {
    const int top = 2 * ((int)(ax + 15.0 + sqrt(40.0 * ax)) / 2);
    double jn1 = 0.0, jn = 1e-30, keep1 = 0.0, even = 0.0;
    for (int nn = top; nn > 0; --nn) {
      const double jm = 2.0 * nn / ax * jn - jn1;  // J_{nn-1}
      jn1 = jn;
      jn = jm;
      if (nn == 2) keep1 = jn;
      if (((nn - 1) & 1) == 0 && nn > 1) even += jn;
      if (fabs(jn) > 1e200) { jn *= 1e-200; jn1 *= 1e-200; keep1 *= 1e-200; even *= 1e-200; }
    }
    r = keep1 / (jn + 2.0 * even);
  } else {
    double a = 1.0, pw = 1.0, P = 0.0, Q = 0.0;
    const double ix = 1.0 / ax;
    for (int k = 0; k < 14; ++k) {
      if (k > 0) a *= (4.0 - (2.0 * k - 1.0) * (2.0 * k - 1.0)) / (8.0 * k);
      const double sg = (k & 2) ? -1.0 : 1.0;
      if (k & 1) Q += sg * a * pw; else P += sg * a * pw;
      pw *= ix;
    }
    double sn, cs;
    sincos(ax - 2.35619449019234492885, &sn, &cs);
    r = sqrt(0.63661977236758134308 * ix) * (P * cs - Q * sn);
  }
  return x < 0.0 ? -r : r;
}

// Number of negative eigenvalues of the symmetric matrix [[a, b], [b, c]].
__device__ __forceinline__ int neg_eigs(double a, double b, double c) {
  double det = a * c - b * b;
  if (det < 0.0) return 1;
  double tr = a + c;
  if (det > 0.0) return tr < 0.0 ? 2 : 0;
  return tr < 0.0 ? 1 : 0;
}

// One emitted order of one ray, lab frame.
template <typename G>
struct Emission {
  int slot;            // order slot p - p_min
  int nf;              // focal lines, far-field leg included
  int det_neg;         // det Q' < 0
  v3<G> dir;           // lab exit direction (the phase is computed with exactly this vector)
  v3<G> obs;           // node-space direction: dir in the far field, else the direction of the
                       // point M where the ray meets the observation sphere (the phase refers
                       // to exactly this vector)
  v3<double> obs64;    // the same direction before its rounding to G (interpolation weights)
  v3<double> rexit;    // lab exit point (um)
  double phase;        // OPL - k dir.rexit - nf pi/2, unreduced; at radius R: OPL + k (d_M - R) - nf pi/2
  double amp;          // sqrt(D / |det Q'|); at radius R: R sqrt(D / |det(I + d_M Q')|)
  double amplif;       // error amplification of the divergence factor along this ray (>= 1)
  double drift;        // growth of a direction perturbation along the ray: prod of the largest |eig(I + L Q)|
  cx<G> f[2][3];       // lab field vectors amp e^{i phase} (J_perp e_perp + J_par e_par)
};

// ---------------------------------------------------------------------------
// the per-ray trace: Eqs. 3, 4, 6, 8, 9, 10
//
// The polyline (positions, directions, normals, incidence-plane bases, Snell)
// is FP64 in both paths; the wave quantities carried along it (Fresnel
// coefficients, Jones matrix, wavefront-curvature recursion, emitted fields)
// are in G.  FP32 directions drift: each curved reflection multiplies a
// direction error by ~3-5, which after three bounces moves the far-field
// interpolation by ~1e-4; FP64 multiply-adds cost the same as FP32 ones on
// this chip, so the polyline stays FP64.
// ---------------------------------------------------------------------------
// GEN = false compiles out the finite observation radius and absorption (for
// particles with !needs_general_trace): the plain far field then fits three
// waves per SIMD without spilling.
__host__ __device__ inline bool needs_general_trace(const ParticleConst& P) { return P.robs > 0.0 || P.m_im > 0.0; }

// The state a ray carries between interactions.
template <typename G>
struct RayState {
  v3<double> r, d, u1, u2;  // position on the surface, direction, polarisation basis (u2 = d x u1)
  double q11, q12, q22;     // WFC in (u1, u2)
  cx<G> J[2][2];            // J[component along u_a][incident pol]
  double D;                 // divergence product of the internal segments
  double opl;               // optical path (phase), referenced to the particle centre
  double amplif;            // largest error amplification of the divergence factor so far
  double drift;             // growth of a direction perturbation so far
  double n_cur, n_oth;      // index of the current and of the other medium
  int nf;                   // focal lines crossed so far
};

// Entry of the incident ray of grid cell (ix, iy) into the particle (the
// initial state at its first interaction); false if the ray misses.
template <typename G>
__device__ __forceinline__ bool ray_init(const ParticleConst& P, int ix, int iy, RayState<G>& s) {
  typedef v3<double> V;
  const double* R = P.R;
  const double x = -P.L + (ix + 0.5) * P.h;
  const double y = -P.L + (iy + 0.5) * P.h;
  // plane wave: lab ray x*ex + y*ey + t ez in body coordinates
  V o = mk3(R[0] * x + R[3] * y, R[1] * x + R[4] * y, R[2] * x + R[5] * y);
  V d = mk3(R[6], R[7], R[8]);
  V u1 = mk3(R[0], R[1], R[2]);  // body image of lab x
  V u2 = mk3(R[3], R[4], R[5]);  // body image of lab y = d x u1
  double t0 = 0.0;
  if (P.zs > 0.0) {
    // point source at lab (0, 0, -zs): the ray toward the lab point (x, y, 0),
    // polarisation u1 = lab x made transverse to it, u2 = d x u1
    const double il = rsq_d(x * x + y * y + P.zs * P.zs);
    const double lx = x * il, ly = y * il, lz = P.zs * il;
    const double iu = rsq_d(1.0 - lx * lx);
    const double ux = (1.0 - lx * lx) * iu, uy = -lx * ly * iu, uz = -lx * lz * iu;
    d = mk3(R[0] * lx + R[3] * ly + R[6] * lz, R[1] * lx + R[4] * ly + R[7] * lz, R[2] * lx + R[5] * ly + R[8] * lz);
    u1 = mk3(R[0] * ux + R[3] * uy + R[6] * uz, R[1] * ux + R[4] * uy + R[7] * uz, R[2] * ux + R[5] * uy + R[8] * uz);
    u2 = cross(d, u1);
    // start at the closest approach to the centre: the entry quadratic solved
    // from the source itself would lose digits as the square of its distance
    o = mk3(-P.zs * R[6], -P.zs * R[7], -P.zs * R[8]);
    t0 = -dot(o, d);
    o = axpy(t0, d, o);
  }
  const V Ad0 = mk3(P.A[0] * d.x, P.A[1] * d.y, P.A[2] * d.z);
  const V Ao = mk3(P.A[0] * o.x, P.A[1] * o.y, P.A[2] * o.z);
  double qa = dot(d, Ad0), qb = 2.0 * dot(d, Ao), qc = dot(o, Ao) - 1.0;
  double disc = qb * qb - 4.0 * qa * qc;
  if (!(disc > 0.0)) return false;
  double qq = -0.5 * (qb + copysign(sqrt_d(disc), qb));
  if (qq == 0.0) return false;
  double t = fmin(qq / qa, qc / qq);

  s.r = axpy(t, d, o);
  s.d = d;
  s.u1 = u1;
  s.u2 = u2;
  s.q11 = s.q12 = s.q22 = 0;   // plane wave
  s.J[0][0].re = 1; s.J[0][0].im = 0; s.J[0][1].re = 0; s.J[0][1].im = 0;
  s.J[1][0].re = 0; s.J[1][0].im = 0; s.J[1][1].re = 1; s.J[1][1].im = 0;
  s.D = 1.0;
  s.nf = 0;
  s.opl = P.k * dot(d, s.r);  // incident phase, referenced to the particle centre
  if (P.zs > 0.0) {
    // spherical wave rho = t0 + t from the source: WFC I / rho, amplitude
    // zs / rho, phase k (rho - zs) (both referenced to the particle centre)
    const double rho = t0 + t;
    const double irho = rcp_d(rho);
    s.q11 = s.q22 = irho;
    s.J[0][0].re = s.J[1][1].re = (G)(P.zs * irho);
    s.opl = P.k * (rho - P.zs);
  }
  // Largest relative-error amplification met so far by the divergence factor:
  // the cancellation in det(I + L Q) per propagation (a focal line close to an
  // interface).  Each emission adds the cancellation of its own exit wavefront
  // equation (a flat exit wavefront: a far-field caustic).
  s.amplif = 1.0;
  s.drift = 1.0;
  s.n_cur = 1.0;
  s.n_oth = P.m;
  return true;
}

// Interaction q (1 = entry) of a ray in state s.  An order in [p_min, p_max]
// emitted here goes to sink.emit at once.  Returns bit 0 when it emits, bit 1
// when the ray goes on to interaction q + 1 (s then holds its state there).
template <typename G, bool GEN, typename Sink>
__device__ __forceinline__ int ray_interact(const ParticleConst& P, int q, RayState<G>& s, Sink& sink) {
  typedef v3<double> V;
  const double* R = P.R;
  int status = 0;
  // outward normal and incidence-plane basis (FP64)
  V Ar = mk3(P.A[0] * s.r.x, P.A[1] * s.r.y, P.A[2] * s.r.z);
  const double inA = rsq_d(dot(Ar, Ar));
  V nh = scl(inA, Ar);
  const double dn = dot(s.d, nh);  // n . k_hat (signed)
  const double sgn = dn > 0 ? 1.0 : -1.0;
  const double ci = sgn * dn;    // cos(theta_i)
  V c = scl(sgn, cross(s.d, nh));  // d x nu
  const double c2 = dot(c, c);
  V ep = c2 < 1e-24 ? s.u1 : scl(rsq_d(c2), c);
  // rotate the carried state into (e_perp, e_par): e_perp = cs u1 + sn u2
  const G cs = (G)dot(ep, s.u1), sn = (G)dot(ep, s.u2);
  cx<G> Jl[2][2];
  for (int k = 0; k < 2; ++k) {
    Jl[0][k].re = cs * s.J[0][k].re + sn * s.J[1][k].re;
    Jl[0][k].im = cs * s.J[0][k].im + sn * s.J[1][k].im;
    Jl[1][k].re = -sn * s.J[0][k].re + cs * s.J[1][k].re;
    Jl[1][k].im = -sn * s.J[0][k].im + cs * s.J[1][k].im;
  }
  const double csd = dot(ep, s.u1), snd = dot(ep, s.u2);
  const double t11 = csd * csd * s.q11 + 2 * csd * snd * s.q12 + snd * snd * s.q22;
  const double t12 = (csd * csd - snd * snd) * s.q12 + csd * snd * (s.q22 - s.q11);
  const double t22 = snd * snd * s.q11 - 2 * csd * snd * s.q12 + csd * csd * s.q22;

  // surface curvature in (s1, s2) = (e_perp, n x e_perp), shape operator of r^T A r = 1
  V s2 = cross(nh, ep);
  const double C11 = (P.A[0] * ep.x * ep.x + P.A[1] * ep.y * ep.y + P.A[2] * ep.z * ep.z) * inA;
  const double C12 = (P.A[0] * ep.x * s2.x + P.A[1] * ep.y * s2.y + P.A[2] * ep.z * s2.z) * inA;
  const double C22 = (P.A[0] * s2.x * s2.x + P.A[1] * s2.y * s2.y + P.A[2] * s2.z * s2.z) * inA;

  // Snell (Eq. 4), FP64
  const double n_cur = s.n_cur, n_oth = s.n_oth;
  const double mrel = n_oth / n_cur;
  const double st2 = 1.0 - ci * ci;
  const double ct2 = 1.0 - st2 / (mrel * mrel);
  const bool tir = ct2 < 0.0;
  V dr = axpy(-2.0 * dn, nh, s.d);
  const double gr = -dn;  // n . k_hat of the reflected wave
  double ct = 0.0, gt = 0.0;
  V dt = s.d;
  if (!tir) {
    ct = sqrt_d(ct2);
    const double sct = sgn * ct, im = rcp_d(mrel);
    dt = mk3((s.d.x - dn * nh.x) * im + sct * nh.x, (s.d.y - dn * nh.y) * im + sct * nh.y,
             (s.d.z - dn * nh.z) * im + sct * nh.z);
    gt = dot(dt, nh);
  }
  // Fresnel (Eq. 8) in units of n_cur k, in G
  cx<G> rp, rl, tp, tl;
  {
    const G cig = (G)ci, mg = (G)mrel, m2 = mg * mg;
    if (!tir) {
      const G b = (G)(mrel * ct);  // k_rn / (n_cur k)
      const G inv1 = rcp_t(cig + b), inv2 = rcp_t(m2 * cig + b);
      rp.re = (cig - b) * inv1;  rp.im = 0;
      rl.re = (m2 * cig - b) * inv2;  rl.im = 0;
      tp.re = 2 * cig * inv1;  tp.im = 0;
      tl.re = 2 * mg * cig * inv2;  tl.im = 0;
    } else {
      // evanescent transmitted wave, k_rn = +i n_cur k sqrt(sin^2 - m_rel^2)
      const G beta = (G)sqrt(st2 - mrel * mrel);
      cx<G> a1, b1, a2, b2;
      a1.re = cig; a1.im = -beta; b1.re = cig; b1.im = beta;
      a2.re = m2 * cig; a2.im = -beta; b2.re = m2 * cig; b2.im = beta;
      rp = cdiv(a1, b1);
      rl = cdiv(a2, b2);
      tp.re = tp.im = tl.re = tl.im = 0;
    }
  }

  // wavefront equation (Eq. 3) with diagonal projections P = diag(1, n.k_hat):
  //   k' P' Q' P' = k_i P_i Q~ P_i + C n.(k' - k_i)
  const double ki = n_cur * P.k;
  const double M11i = ki * t11, M12i = ki * dn * t12, M22i = ki * dn * dn * t22;

  // ---- emission of an order, if this interaction emits one ----
  int p_emit = -1;
  bool emit_t = false;
  if (q == 1) p_emit = 0;  // external reflection
  else if (!tir) { p_emit = q - 1; emit_t = true; }
  if (p_emit >= P.p_min && p_emit <= P.p_max) {
    status |= 1;
    const double kod = emit_t ? n_oth * P.k : n_cur * P.k;
    const double god = emit_t ? gt : gr;
    const double w = emit_t ? (kod * gt - n_cur * P.k * dn) : (n_cur * P.k * (gr - dn));
    const V dout = emit_t ? dt : dr;
    const double inko = rcp_d(kod), igo = rcp_d(god);
    const double a11 = M11i + w * C11, a12 = M12i + w * C12, a22 = M22i + w * C22;
    double Q11 = a11 * inko;
    double Q12 = a12 * inko * igo;
    double Q22 = a22 * inko * igo * igo;
    double detQ = Q11 * Q22 - Q12 * Q12;
    int nft = s.nf + neg_eigs(Q11, Q12, Q22);
    double e_amplif = s.amplif;
    {
      // cancellation in det of the Eq. 3 sum M = k_i P Q~ P + w C: a flat exit
      // wavefront (far-field caustic) makes det M small against its terms;
      // first-order bound of the relative error of det M for entry-wise errors
      double t11a = fabs((double)M11i) + fabs((double)(w * C11)), t12a = fabs((double)M12i) + fabs((double)(w * C12));
      double t22a = fabs((double)M22i) + fabs((double)(w * C22));
      double b11 = a11, b12 = a12, b22 = a22;
      e_amplif = fmax(e_amplif, (t11a * fabs(b22) + fabs(b11) * t22a + 2.0 * t12a * fabs(b12)) /
                                    fmax(fabs(b11 * b22 - b12 * b12), 1e-300));
    }
    double amp = sqrt_d(s.D * rcp_d(fabs(detQ)));
    v3<G> ul;
    V epo = cross(dout, ep);  // e_par' of the outgoing wave
    // lab vectors: direction rounded once to G; the phase uses exactly that vector
    const V dl64 = mk3(R[0] * dout.x + R[1] * dout.y + R[2] * dout.z, R[3] * dout.x + R[4] * dout.y + R[5] * dout.z,
                       R[6] * dout.x + R[7] * dout.y + R[8] * dout.z);
    v3<G> dl = mk3<G>((G)dl64.x, (G)dl64.y, (G)dl64.z);
    V ul64 = dl64;
    V rl_lab = mk3(R[0] * s.r.x + R[1] * s.r.y + R[2] * s.r.z, R[3] * s.r.x + R[4] * s.r.y + R[5] * s.r.z,
                   R[6] * s.r.x + R[7] * s.r.y + R[8] * s.r.z);
    double phase = s.opl - P.k * dot(cvt<double>(dl), rl_lab) - nft * 1.5707963267948966;
    ul = dl;
    if (GEN && P.robs > 0.0) {
      // finite observation radius: continue the ray by d_M to M on the
      // sphere; the last leg's divergence factor is 1 / det(I + d_M Q')
      // d_M - R without the cancellation of the plain difference at large R
      const double drr = dot(dout, s.r);
      const double rp2 = dot(s.r, s.r) - drr * drr;
      const double dMR = -drr - rp2 * rcp_d(sqrt_d(P.robs * P.robs - rp2) + P.robs);
      const double dM = P.robs + dMR;
      const double g11 = 1.0 + dM * Q11, g12 = dM * Q12, g22 = 1.0 + dM * Q22;
      const double detG = g11 * g22 - g12 * g12;
      nft = s.nf + neg_eigs(g11, g12, g22);
      amp = P.robs * sqrt_d(s.D * rcp_d(fabs(detG)));
      // Q' carries the error amplified so far; det(I + d_M Q') scales its
      // entries' rounding by half its entry-wise condition.  Far from the
      // particle that tends to det Q''s own condition, which e_amplif
      // already holds, so only the excess over it multiplies e_amplif (it
      // grows where a caustic meets the observation sphere)
      const double cg = 0.5 * (fabs(dM * Q11) * fabs(g22) + fabs(g11) * fabs(dM * Q22) + 2.0 * dM * dM * Q12 * Q12) /
                        fmax(fabs(detG), 1e-300);
      const double cq = (fabs(Q11 * Q22) + Q12 * Q12) / fmax(fabs(detQ), 1e-300);
      e_amplif *= fmax(1.0, cg / cq);
      phase = s.opl + P.k * dMR - nft * 1.5707963267948966;
      const V Mb = mk3(s.r.x + dM * dout.x, s.r.y + dM * dout.y, s.r.z + dM * dout.z);
      const double ir = rcp_d(P.robs);
      const V u = mk3((R[0] * Mb.x + R[1] * Mb.y + R[2] * Mb.z) * ir, (R[3] * Mb.x + R[4] * Mb.y + R[5] * Mb.z) * ir,
                      (R[6] * Mb.x + R[7] * Mb.y + R[8] * Mb.z) * ir);
      ul = mk3<G>((G)u.x, (G)u.y, (G)u.z);
      ul64 = u;
      // refer the phase to the rounded direction, as the far field does: the
      // phase gained from R u to the sphere's point along (G)u (exact, also
      // where d_M vanishes)
      if (sizeof(G) < 8)
        phase += near_carry(P.k * P.robs, P.k * rl_lab.x, P.k * rl_lab.y, P.k * rl_lab.z, u.x, u.y, u.z,
                            (double)ul.x, (double)ul.y, (double)ul.z);
    }
    G sph, cph;
    if (sizeof(G) == 8) sincos_t((G)phase, &sph, &cph);
    else sincos_red((G)reduce_2pi(phase), &sph, &cph);
    G ga = (G)amp;
    cx<G> pa;
    pa.re = ga * cph; pa.im = ga * sph;
    v3<G> epl = mk3<G>((G)(R[0] * ep.x + R[1] * ep.y + R[2] * ep.z), (G)(R[3] * ep.x + R[4] * ep.y + R[5] * ep.z),
                       (G)(R[6] * ep.x + R[7] * ep.y + R[8] * ep.z));
    v3<G> eql = mk3<G>((G)(R[0] * epo.x + R[1] * epo.y + R[2] * epo.z),
                       (G)(R[3] * epo.x + R[4] * epo.y + R[5] * epo.z),
                       (G)(R[6] * epo.x + R[7] * epo.y + R[8] * epo.z));
    cx<G> c0 = emit_t ? tp : rp, c1 = emit_t ? tl : rl;
    Emission<G> e;
    e.slot = p_emit - P.p_min;
    e.nf = nft;
    e.det_neg = detQ < 0.0;
    e.dir = dl;
    e.obs = ul;
    e.obs64 = ul64;
    e.rexit = rl_lab;
    e.phase = phase;
    e.amp = amp;
    e.amplif = e_amplif;
    e.drift = s.drift;
    for (int k = 0; k < 2; ++k) {
      cx<G> jp = cmul(pa, cmul(c0, Jl[0][k]));
      cx<G> jq = cmul(pa, cmul(c1, Jl[1][k]));
      e.f[k][0].re = jp.re * epl.x + jq.re * eql.x; e.f[k][0].im = jp.im * epl.x + jq.im * eql.x;
      e.f[k][1].re = jp.re * epl.y + jq.re * eql.y; e.f[k][1].im = jp.im * epl.y + jq.im * eql.y;
      e.f[k][2].re = jp.re * epl.z + jq.re * eql.z; e.f[k][2].im = jp.im * epl.z + jq.im * eql.z;
    }
    sink.emit(e);
  }
  if (q == P.p_max + 1) return status;

  // ---- continuing branch: transmitted at q = 1, reflected afterwards ----
  const bool cont_t = (q == 1);
  if (cont_t && tir) return status;
  const double kod = cont_t ? n_oth * P.k : n_cur * P.k;
  const double god = cont_t ? gt : gr;
  const double w = cont_t ? (kod * gt - n_cur * P.k * dn) : (n_cur * P.k * (gr - dn));
  const double inko = rcp_d(kod), igo = rcp_d(god);
  const double Q11 = (M11i + w * C11) * inko;
  const double Q12 = (M12i + w * C12) * inko * igo;
  const double Q22 = (M22i + w * C22) * inko * igo * igo;
  cx<G> c0 = cont_t ? tp : rp, c1 = cont_t ? tl : rl;
  for (int k = 0; k < 2; ++k) {
    s.J[0][k] = cmul(c0, Jl[0][k]);
    s.J[1][k] = cmul(c1, Jl[1][k]);
  }
  const V d = cont_t ? dt : dr;
  s.d = d;
  s.u1 = ep;
  s.u2 = cross(d, ep);
  if (cont_t) { s.n_cur = n_oth; s.n_oth = 1.0; }

  // free propagation along the chord (FP64): G = I + L Q, Q <- Q G^-1
  const V r = s.r;
  const double L = -2.0 * (P.A[0] * d.x * r.x + P.A[1] * d.y * r.y + P.A[2] * d.z * r.z) /
                   (P.A[0] * d.x * d.x + P.A[1] * d.y * d.y + P.A[2] * d.z * d.z);
  double g11 = 1.0 + L * (double)Q11, g12 = L * (double)Q12, g22 = 1.0 + L * (double)Q22;
  double detG = g11 * g22 - g12 * g12;
  {
    double mid = 0.5 * (g11 + g22), rad = sqrt(0.25 * (g11 - g22) * (g11 - g22) + g12 * g12);
    s.drift *= fmax(1.0, fmax(fabs(mid + rad), fabs(mid - rad)));
  }
  // cancellation in det(I + L Q) (relative errors enter through L Q only)
  s.amplif = fmax(s.amplif, (fabs(L * (double)Q11) * fabs(g22) + fabs(g11) * fabs(L * (double)Q22) + 2.0 * g12 * g12) /
                                fmax(fabs(detG), 1e-300));
  s.D *= rcp_d(fabs(detG));
  s.nf += neg_eigs(g11, g12, g22);
  double idg = rcp_d(detG);
  // Q G^-1 with G^-1 = [[g22, -g12], [-g12, g11]] / det G  (symmetric result)
  double n11 = ((double)Q11 * g22 - (double)Q12 * g12) * idg;
  double n12 = ((double)Q12 * g11 - (double)Q11 * g12) * idg;
  double n22 = ((double)Q22 * g11 - (double)Q12 * g12) * idg;
  s.q11 = n11; s.q12 = n12; s.q22 = n22;
  s.opl += s.n_cur * P.k * L;
  if (GEN && s.n_cur != 1.0 && P.m_im > 0.0) {
    // weak absorption along the internal segment
    const G att = (G)exp(-P.k * P.m_im * L);
    for (int k = 0; k < 2; ++k)
      for (int a = 0; a < 2; ++a) { s.J[a][k].re *= att; s.J[a][k].im *= att; }
  }
  s.r = axpy(L, d, r);
  return status | 2;
}

template <typename G, bool GEN = true, typename Sink>
__device__ void trace_ray(const ParticleConst& P, int ix, int iy, Sink& sink) {
  RayState<G> s;
  if (!ray_init(P, ix, iy, s)) return;
  for (int q = 1; q <= P.p_max + 1; ++q)
    if (!(ray_interact<G, GEN>(P, q, s, sink) & 2)) break;
}

}  // namespace rtw
