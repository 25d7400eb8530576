/*
 * rtw_oracle.c -- plain FP64 CPU oracle of the Ray Theory of Waves far-field
 * path (Ren et al., arXiv 2403.13856).
 *
 * TEST INFRASTRUCTURE ONLY (see rtw_oracle.h).  Written for readability, not
 * speed: every step follows the paper's order and notation, with no blocking,
 * fusion or reordering.  All arithmetic is IEEE double; build with
 * -ffp-contract=off.
 *
 * Readings of the paper used here (the paper is silent or garbled on them):
 *  R1  Q > 0 means a diverging wavefront (Q = 1/R, R measured from the
 *      virtual source) and the surface curvature matrix C is positive for a
 *      convex surface with the outward normal n; both follow from the
 *      appendix construction (the wavefront lies upstream of its tangent
 *      plane by delta = t Q t^T / 2, the surface lies below its tangent plane
 *      along -n by t C t^T / 2).
 *  R2  Projection matrices are P_ab = s_a . (wavefront basis)_b, and the
 *      tangent vectors are row vectors, t_i = t_c P_i (appendix Eq. A2-A3;
 *      the printed "t_i = P_i t_c" is read as the row-vector form).
 *  R3  Eq. 8 is applied at every interface with the relative index
 *      m_rel = n_other / n_current, k_in = n_current k cos(theta_i) and
 *      k_rn = n_other k cos(theta_t); under total internal reflection
 *      k_rn = +i k sqrt(n_cur^2 sin^2 theta_i - n_oth^2) (evanescent decay for
 *      exp(-i w t)), and the transmitted order is absent.
 *  R4  The parallel unit vector is e_par = khat x e_perp for the incident and
 *      for each outgoing wave, e_perp = unit(d x nu) with nu the normal on the
 *      transmission side; at exact normal incidence e_perp is the first
 *      vector of the carried basis.
 *  R5  Eq. 9 is read as Phi_P = +k1.r1 + sum_q k_q.(r_q - r_{q-1}) + k'.(r_M -
 *      r_{p+1}); the far field drops k r, leaving -k dir.r_exit.  The
 *      incident phase is referenced to the particle centre.
 *  R6  Each focal line adds -pi/2 under exp(-i w t) (opposite sign to the path
 *      phase).  N_f counts the eigenvalues of I + L Q' that are negative on
 *      each internal segment plus the negative eigenvalues of Q' on the
 *      far-field leg.
 *  R7  Eq. 6 for the far field: D = prod over internal segments of
 *      1/|det(I + L Q')|, and the far-field amplitude is sqrt(D/|det Q'|)
 *      (the last Gaussian-curvature ratio times r^2).
 *  R8  Eq. 7 interactions are numbered 1..p+1 as in Eqs. 6 and 9.  Order p=0
 *      is the external reflection at interaction 1; order p>=1 is the
 *      transmission out at interaction p+1 after p-1 internal reflections.
 *  R9  Interpolation (RTW strategy section): per order, each incident-grid
 *      quad is split along its (i,j)-(i+1,j+1) diagonal; a triangle is used
 *      when its three rays emit the order with equal focal-line counts (the
 *      direction map folds exactly where N_f changes); a node direction inside the spherical triangle
 *      receives the barycentric (central projection) interpolation of the
 *      three ray fields, each carried to the node direction with the
 *      stationary-phase gradient dPhi/d(dir) = -k r_exit.
 *  R10 Non-plane incidence (the Phi_i term of Eq. 10): a point source S on
 *      the lab axis at z = -z_s sends a spherical wave toward +z.  The ray
 *      of grid point (x, y) runs from S through the lab point (x, y, 0);
 *      at its first interaction point r_1, rho_1 = |r_1 - S| from S, the
 *      incident WFC is Q_i = I / rho_1 (diverging, reading R1), the amplitude
 *      A_0 = z_s / rho_1 (unit at the distance of the particle centre) and
 *      Phi_i = k (rho_1 - z_s) (phase referenced to the particle centre, so
 *      that z_s -> infinity gives back the plane wave's k z_1).  Its
 *      polarisation vectors are lab x made transverse to the ray and
 *      normalised, u_1, and u_2 = d x u_1.  The grid's half-width is the
 *      largest extent along x or y of the particle's tangent cone from S on
 *      the plane z = 0 (rtwo_grid_halfwidth_source).
 *  R11 Observation at a finite distance (the point M of Eqs. 6 and 9): the
 *      nodes lie on the sphere of radius R about the particle centre.  A ray
 *      leaving r_exit along d meets it after d_M (|r_exit + d_M d| = R); the
 *      last Gaussian-curvature ratio of Eq. 6 is 1/det(I + d_M Q'), so the
 *      field there is A_0 |eps| sqrt(D / |det(I + d_M Q')|); N_f counts the
 *      negative eigenvalues of I + d_M Q' on that leg; the path phase of Eq. 9
 *      ends with k d_M.  The output is R e^{-ikR} E(M) (tending to the far
 *      field F as R grows), so its phase is OPL + k (d_M - R) - N_f pi/2.
 *      The ray's node-space direction is u = M / R; interpolation (R9) runs on
 *      u, and each vertex field is carried to a node n along the sphere as a
 *      wave leaving the ray's exit point, phase k (|R n - r_exit| - |R u -
 *      r_exit|) (its gradient on the sphere at u is the ray's, and for
 *      R -> infinity it tends to R9's -k r_exit.(n - u)).  Only the part of
 *      E(M) tangent to the sphere at M is an output (the radial part, of
 *      relative size |r_exit| / R, is dropped at the vertex); the output is its
 *      projection on the node's (e_theta, e_phi).
 *  R12 Correction at fold caustics (the wave correction near caustics that the
 *      paper names without formulas): where an order's two branches coalesce
 *      at a fold their focal-line counts differ by one.  At a node holding
 *      exactly two contributions of one order, a with N_f = n and b with
 *      N_f = n + 1, their geometric-optics sum is replaced by the uniform
 *      asymptotic (Airy) form of Chester, Friedman and Ursell (1957) in
 *      Ludwig's (1966) two-ray form: with the branches' interpolated fields
 *      f_a, f_b and their carried phases phi_a, phi_b (each the barycentric
 *      mean of its rays' phases carried to the node, focal lines included),
 *      Delta = (phi_b - phi_a) / 2 + pi / 4 is half their path-phase
 *      difference, (2/3) zeta^{3/2} = Delta, and
 *        u = sqrt(pi) e^{-i pi/4} [ (f_a e^{i Delta} + i f_b e^{-i Delta}) zeta^{1/4} Ai(-zeta)
 *                                - i (f_a e^{i Delta} - i f_b e^{-i Delta}) zeta^{-1/4} Ai'(-zeta) ],
 *      which tends to f_a + f_b far from the fold (large zeta).  Nodes with
 *      Delta <= 0 keep the sum; the dark side of the fold gets no field.
 *  R13 Forward diffraction (not in the paper's ray path; plane wave, far
 *      field): by Babinet's principle the particle's shadow diffracts like an
 *      aperture of its shape.  The shadow of the ellipsoid on the plane
 *      z = 0 is the ellipse rho^T S2^-1 rho <= 1, S2 the x-y block of
 *      R diag(a^2, b^2, c^2) R^T; its Fraunhofer amplitude in direction n is
 *      F_d = (i k / 2 pi) pi sqrt(det S2) 2 J1(k s) / (k s), s = sqrt(n_t^T S2 n_t),
 *      n_t the projection of n on the plane (F_d(0) = i k area / 2 pi, the
 *      forward amplitude the optical theorem pairs with the shadow), carried
 *      by the incident polarisation in the frame (e_theta, e_phi) that turns
 *      with phi: x gives (cos phi, -sin phi), y gives (sin phi, cos phi).
 *  R14 Absorbing particles (not in the paper): for m = m_r + i m_im with
 *      m_im << m_r, the weak-absorption reading of geometric optics: Snell,
 *      Eq. 8 and Eq. 3 use m_r, and every internal segment of length L
 *      scales the carried field by exp(-k m_im L) (a homogeneous wave of index
 *      m_r + i m_im; the inhomogeneous-wave corrections of strong absorption
 *      are left out).  Parity unpinned against the paper; pinned to the
 *      chord lengths of the sphere.
 */
#include "rtw_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double PI = 3.14159265358979323846;
static int g_threads = 0;

void rtwo_set_threads(int n) { g_threads = n; }
int rtwo_get_threads(void) {
#ifdef _OPENMP
  return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* small vector helpers                                               */
/* ------------------------------------------------------------------ */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c) {
  double x = a[1] * b[2] - a[2] * b[1];
  double y = a[2] * b[0] - a[0] * b[2];
  double z = a[0] * b[1] - a[1] * b[0];
  c[0] = x; c[1] = y; c[2] = z;
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }
static void scale3(double s, const double* a, double* c) { c[0] = s * a[0]; c[1] = s * a[1]; c[2] = s * a[2]; }
static void copy3(const double* a, double* c) { c[0] = a[0]; c[1] = a[1]; c[2] = a[2]; }
static void matvec(const double M[3][3], const double* v, double* o) {
  double t[3];
  for (int i = 0; i < 3; i++) t[i] = M[i][0] * v[0] + M[i][1] * v[1] + M[i][2] * v[2];
  copy3(t, o);
}
static void matTvec(const double M[3][3], const double* v, double* o) {
  double t[3];
  for (int i = 0; i < 3; i++) t[i] = M[0][i] * v[0] + M[1][i] * v[1] + M[2][i] * v[2];
  copy3(t, o);
}

/* Rotation body -> lab, R = Rz(alpha) Ry(beta) Rz(gamma). */
static void euler_zyz(const double* deg, double R[3][3]) {
  double a = deg[0] * PI / 180.0, b = deg[1] * PI / 180.0, g = deg[2] * PI / 180.0;
  double Za[3][3] = {{cos(a), -sin(a), 0}, {sin(a), cos(a), 0}, {0, 0, 1}};
  double Yb[3][3] = {{cos(b), 0, sin(b)}, {0, 1, 0}, {-sin(b), 0, cos(b)}};
  double Zg[3][3] = {{cos(g), -sin(g), 0}, {sin(g), cos(g), 0}, {0, 0, 1}};
  double T[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      T[i][j] = 0;
      for (int k = 0; k < 3; k++) T[i][j] += Za[i][k] * Yb[k][j];
    }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      R[i][j] = 0;
      for (int k = 0; k < 3; k++) R[i][j] += T[i][k] * Zg[k][j];
    }
}

/* ------------------------------------------------------------------ */
/* 2x2 real matrices                                                   */
/* ------------------------------------------------------------------ */
typedef struct { double m[2][2]; } mat2;

static mat2 m2mul(mat2 A, mat2 B) {
  mat2 C;
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) C.m[i][j] = A.m[i][0] * B.m[0][j] + A.m[i][1] * B.m[1][j];
  return C;
}
static mat2 m2T(mat2 A) {
  mat2 C;
  C.m[0][0] = A.m[0][0]; C.m[0][1] = A.m[1][0]; C.m[1][0] = A.m[0][1]; C.m[1][1] = A.m[1][1];
  return C;
}
static double m2det(mat2 A) { return A.m[0][0] * A.m[1][1] - A.m[0][1] * A.m[1][0]; }
static mat2 m2inv(mat2 A) {
  double d = m2det(A);
  mat2 C;
  C.m[0][0] = A.m[1][1] / d; C.m[0][1] = -A.m[0][1] / d;
  C.m[1][0] = -A.m[1][0] / d; C.m[1][1] = A.m[0][0] / d;
  return C;
}
static mat2 m2add(mat2 A, mat2 B) {
  mat2 C;
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) C.m[i][j] = A.m[i][j] + B.m[i][j];
  return C;
}
static mat2 m2scale(double s, mat2 A) {
  mat2 C;
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) C.m[i][j] = s * A.m[i][j];
  return C;
}
/* Number of negative eigenvalues of a symmetric 2x2 matrix (explicit eigenvalues). */
static int m2neg(mat2 A) {
  double a = A.m[0][0], c = A.m[1][1], b = 0.5 * (A.m[0][1] + A.m[1][0]);
  double mid = 0.5 * (a + c), rad = sqrt(0.25 * (a - c) * (a - c) + b * b);
  return (mid - rad < 0.0) + (mid + rad < 0.0);
}

/* ------------------------------------------------------------------ */
/* Eq. 8 (Fresnel coefficients from normal wave-vector components)      */
/* ------------------------------------------------------------------ */
static void fresnel_eq8(cplx kin, cplx krn, double m, cplx* rperp, cplx* rpar, cplx* tperp, cplx* tpar) {
  *rperp = (kin - krn) / (kin + krn);
  *rpar = (m * m * kin - krn) / (m * m * kin + krn);
  *tperp = 2.0 * kin / (kin + krn);
  *tpar = 2.0 * m * kin / (m * m * kin + krn);
}

void rtwo_fresnel(double m_rel, double ci, double* out) {
  /* unit wave number in the current medium: k_in = ci, k_rn = m_rel cos(theta_t) */
  double ct2 = 1.0 - (1.0 - ci * ci) / (m_rel * m_rel);
  cplx kin = ci, krn;
  if (ct2 >= 0.0) krn = m_rel * sqrt(ct2);
  else krn = I * sqrt((1.0 - ci * ci) - m_rel * m_rel);
  cplx rp, rl, tp, tl;
  fresnel_eq8(kin, krn, m_rel, &rp, &rl, &tp, &tl);
  out[0] = creal(rp); out[1] = cimag(rp);
  out[2] = creal(rl); out[3] = cimag(rl);
  out[4] = creal(tp); out[5] = cimag(tp);
  out[6] = creal(tl); out[7] = cimag(tl);
  cplx ratio = krn / kin;
  out[8] = creal(ratio); out[9] = cimag(ratio);
}

/* ------------------------------------------------------------------ */
/* geometry of the ellipsoid r^T A r = 1, A = diag(a^-2, b^-2, c^-2)   */
/* ------------------------------------------------------------------ */
typedef struct {
  double A[3];      /* diagonal of A */
  double R[3][3];   /* body -> lab */
  double k;         /* 2 pi / lambda */
  double m;
  double m_im;      /* imaginary part of the index (R14) */
  double zs;        /* point-source distance (0: plane wave) */
  double robs;      /* observation radius (0: far field) */
  int n_pol, p_min, p_max;
  int corr;         /* RTWO_CAUSTIC | RTWO_DIFFRACTION */
} ctx_t;

static void Avec(const ctx_t* c, const double* v, double* o) {
  o[0] = c->A[0] * v[0]; o[1] = c->A[1] * v[1]; o[2] = c->A[2] * v[2];
}

/* Surface basis (s1, s2) of the tangent plane at the outward normal n: the
 * wavefront equation holds in any orthonormal tangent basis; the oracle takes
 * s1 along the tangential part of the body axis least aligned with n. */
static void surface_basis(const double* n, double* s1, double* s2) {
  double ax[3] = {0, 0, 0};
  int best = 0;
  double bestv = fabs(n[0]);
  for (int i = 1; i < 3; i++)
    if (fabs(n[i]) < bestv) { bestv = fabs(n[i]); best = i; }
  ax[best] = 1.0;
  double t[3];
  double an = dot3(ax, n);
  for (int i = 0; i < 3; i++) t[i] = ax[i] - an * n[i];
  scale3(1.0 / norm3(t), t, s1);
  cross3(n, s1, s2);
}

/* Curvature matrix of the ellipsoid in (s1, s2): C_ab = s_a^T A s_b / |A r|
 * (second fundamental form of the level set r^T A r = 1 for the outward
 * normal; positive for this convex surface, reading R1). */
static mat2 curvature_matrix(const ctx_t* c, const double* r, const double* s1, const double* s2) {
  double Ar[3], As1[3], As2[3];
  Avec(c, r, Ar);
  double nA = norm3(Ar);
  Avec(c, s1, As1);
  Avec(c, s2, As2);
  mat2 C;
  C.m[0][0] = dot3(s1, As1) / nA;
  C.m[0][1] = dot3(s1, As2) / nA;
  C.m[1][0] = dot3(s2, As1) / nA;
  C.m[1][1] = dot3(s2, As2) / nA;
  return C;
}

/* Projection matrix P_ab = s_a . v_b (appendix Eq. A3, reading R2). */
static mat2 projection(const double* s1, const double* s2, const double* v1, const double* v2) {
  mat2 P;
  P.m[0][0] = dot3(s1, v1); P.m[0][1] = dot3(s1, v2);
  P.m[1][0] = dot3(s2, v1); P.m[1][1] = dot3(s2, v2);
  return P;
}

/* Wavefront equation (Eq. 3): k' P' Q' P'^T = k_i P_i Q_i P_i^T + C n.(k' - k_i),
 * solved for Q'.  kvec_i and kvec_o are the full wave vectors. */
static mat2 wavefront_equation(mat2 Qi, double ki, mat2 Pi, double ko, mat2 Po, mat2 C,
                               const double* n, const double* kvec_i, const double* kvec_o) {
  double dk[3] = {kvec_o[0] - kvec_i[0], kvec_o[1] - kvec_i[1], kvec_o[2] - kvec_i[2]};
  mat2 rhs = m2add(m2scale(ki, m2mul(m2mul(Pi, Qi), m2T(Pi))), m2scale(dot3(n, dk), C));
  mat2 Poinv = m2inv(Po);
  return m2scale(1.0 / ko, m2mul(m2mul(Poinv, rhs), m2T(Poinv)));
}

/* State of a ray between interactions, body frame. */
typedef struct {
  double r[3], d[3];    /* position on the surface, unit direction */
  double u1[3], u2[3];  /* wavefront basis, u2 = d x u1 */
  mat2 Q;               /* WFC matrix in (u1, u2) */
  cplx J[2][2];         /* field components along (u1,u2) for each incident polarisation */
  double D;             /* divergence product (Eq. 6) */
  int nf;               /* focal lines so far */
  double opl;           /* path phase so far (rad) */
  double n_cur;         /* index of the medium the ray travels in */
  int tir_any;
} ray_state;

static void emit_order(const ctx_t* c, const ray_state* s, const double* dir, const double* eperp,
                       const double* epar, mat2 Qx, cplx Jx[2][2], rtwo_emit* e) {
  int nf_total = s->nf + m2neg(Qx);
  double detQ = m2det(Qx);
  double S = sqrt(s->D / fabs(detQ));
  double phase = s->opl - c->k * dot3(dir, s->r) - nf_total * (PI / 2.0);
  if (c->robs > 0.0) {
    /* finite observation radius (reading R11) */
    /* d_M - R = -d.r - |r_perp|^2 / (sqrt(R^2 - |r_perp|^2) + R): the root of
       |r + d_M d| = R written without the cancellation of d_M - R at large R */
    double dr = dot3(dir, s->r);
    double rp2 = dot3(s->r, s->r) - dr * dr;
    double dMR = -dr - rp2 / (sqrt(c->robs * c->robs - rp2) + c->robs);
    double dM = c->robs + dMR;
    mat2 G;
    G.m[0][0] = 1.0 + dM * Qx.m[0][0];
    G.m[0][1] = dM * Qx.m[0][1];
    G.m[1][0] = dM * Qx.m[1][0];
    G.m[1][1] = 1.0 + dM * Qx.m[1][1];
    nf_total = s->nf + m2neg(G);
    S = c->robs * sqrt(s->D / fabs(m2det(G)));
    phase = s->opl + c->k * dMR - nf_total * (PI / 2.0);
    double M[3] = {s->r[0] + dM * dir[0], s->r[1] + dM * dir[1], s->r[2] + dM * dir[2]};
    double Ml[3];
    matvec(c->R, M, Ml);
    scale3(1.0 / c->robs, Ml, e->obs);
  }
  e->valid = 1;
  e->nf = nf_total;
  e->det_neg = detQ < 0.0;
  e->tir_any = s->tir_any;
  matvec(c->R, dir, e->dir);
  matvec(c->R, s->r, e->rexit);
  e->opl = s->opl;
  e->phase = phase;
  e->amp = S;
  e->D = s->D;
  e->q[0] = Qx.m[0][0]; e->q[1] = 0.5 * (Qx.m[0][1] + Qx.m[1][0]); e->q[2] = Qx.m[1][1];
  matvec(c->R, eperp, e->eperp);
  matvec(c->R, epar, e->epar);
  cplx ph = cexp(I * phase);
  for (int a = 0; a < 2; a++)
    for (int p = 0; p < 2; p++) {
      e->jones[a][p][0] = creal(Jx[a][p]);
      e->jones[a][p][1] = cimag(Jx[a][p]);
    }
  for (int p = 0; p < 2; p++)
    for (int x = 0; x < 3; x++) {
      cplx f = S * ph * (Jx[0][p] * e->eperp[x] + Jx[1][p] * e->epar[x]);
      e->field[p][x][0] = creal(f);
      e->field[p][x][1] = cimag(f);
    }
}

/* Trace one ray through the lab point (x, y, 0): a plane-wave ray along +z,
 * or the ray from the point source (reading R10). */
static void trace_one(const ctx_t* c, double x, double y, rtwo_ray* out) {
  memset(out, 0, sizeof(*out));
  double zl[3] = {0, 0, 1}, xl[3] = {1, 0, 0}, yl[3] = {0, 1, 0};
  double o_lab[3] = {x, y, 0.0};
  if (c->zs > 0.0) {
    /* origin at S, direction toward (x, y, 0), x made transverse to it */
    double v[3] = {x, y, c->zs};
    scale3(1.0 / norm3(v), v, zl);
    double xt[3];
    for (int i = 0; i < 3; i++) xt[i] = xl[i] - zl[0] * zl[i];
    scale3(1.0 / norm3(xt), xt, xl);
    cross3(zl, xl, yl);
    o_lab[0] = 0.0; o_lab[1] = 0.0; o_lab[2] = -c->zs;
  }
  ray_state s;
  memset(&s, 0, sizeof(s));
  double o[3];
  matTvec(c->R, o_lab, o);
  matTvec(c->R, zl, s.d);
  matTvec(c->R, xl, s.u1);
  matTvec(c->R, yl, s.u2);

  /* a distant source: restart the ray at its closest approach to the centre,
     so that the quadratic below is not solved from far away (its rounding
     grows with the square of the distance) */
  double t0 = 0.0;
  if (c->zs > 0.0) {
    t0 = -dot3(o, s.d);
    for (int i = 0; i < 3; i++) o[i] += t0 * s.d[i];
  }
  /* entry point: smaller root of (o + t d)^T A (o + t d) = 1, stable form */
  double Ad[3], Ao[3];
  Avec(c, s.d, Ad);
  Avec(c, o, Ao);
  double qa = dot3(s.d, Ad), qb = 2.0 * dot3(s.d, Ao), qc = dot3(o, Ao) - 1.0;
  double disc = qb * qb - 4.0 * qa * qc;
  if (!(disc > 0.0)) return;
  double qq = -0.5 * (qb + copysign(sqrt(disc), qb));
  if (qq == 0.0) return;
  double t1 = qq / qa, t2 = qc / qq;
  double t = t1 < t2 ? t1 : t2;
  for (int i = 0; i < 3; i++) s.r[i] = o[i] + t * s.d[i];
  out->active = 1;

  /* initial state: plane wave (Q = 0), J = identity, incident phase k (khat . r1);
     point source: Q = I / rho_1, J = (z_s / rho_1) identity, phase k (rho_1 - z_s) */
  s.Q.m[0][0] = s.Q.m[0][1] = s.Q.m[1][0] = s.Q.m[1][1] = 0.0;
  s.J[0][0] = 1; s.J[0][1] = 0; s.J[1][0] = 0; s.J[1][1] = 1;
  s.D = 1.0;
  s.nf = 0;
  s.opl = c->k * dot3(s.d, s.r);
  if (c->zs > 0.0) {
    double rho = t0 + t; /* |d| = 1 and the ray starts at S */
    s.Q.m[0][0] = s.Q.m[1][1] = 1.0 / rho;
    s.J[0][0] = s.J[1][1] = c->zs / rho;
    s.opl = c->k * (rho - c->zs);
  }
  s.n_cur = 1.0;
  s.tir_any = 0;

  for (int q = 1; q <= c->p_max + 1; q++) {
    matvec(c->R, s.r, out->hit[q - 1]);
    out->n_hits = q;
    double n_oth = (q == 1) ? c->m : 1.0;

    /* local geometry */
    double Ar[3], nhat[3];
    Avec(c, s.r, Ar);
    scale3(1.0 / norm3(Ar), Ar, nhat);
    double dn = dot3(s.d, nhat);
    double nu[3];
    scale3(dn > 0.0 ? 1.0 : -1.0, nhat, nu);
    double ci = dot3(s.d, nu);
    double cr[3], eperp[3], epar_i[3];
    cross3(s.d, nu, cr);
    double sn = norm3(cr);
    if (sn < 1e-12) copy3(s.u1, eperp);
    else scale3(1.0 / sn, cr, eperp);
    cross3(s.d, eperp, epar_i);

    /* Snell (Eq. 4): tangential wave-vector components are continuous */
    double mrel = n_oth / s.n_cur;
    double ct2 = 1.0 - (1.0 - ci * ci) / (mrel * mrel);
    int tir = ct2 < 0.0;
    double dr[3], dt[3] = {0, 0, 0};
    for (int i = 0; i < 3; i++) dr[i] = s.d[i] - 2.0 * ci * nu[i];
    double ct = 0.0;
    if (!tir) {
      ct = sqrt(ct2);
      for (int i = 0; i < 3; i++) dt[i] = (s.d[i] - ci * nu[i]) / mrel + ct * nu[i];
    }

    /* Fresnel (Eq. 8) with the relative index */
    cplx kin = s.n_cur * c->k * ci;
    cplx krn = tir ? I * c->k * sqrt(s.n_cur * s.n_cur * (1.0 - ci * ci) - n_oth * n_oth)
                   : (cplx)(n_oth * c->k * ct);
    cplx rperp, rpar, tperp, tpar;
    fresnel_eq8(kin, krn, mrel, &rperp, &rpar, &tperp, &tpar);
    if (tir) s.tir_any = 1;

    /* Jones: carried (u1,u2) components -> (e_perp, e_par) -> per-branch coefficients */
    double Rot[2][2] = {{dot3(eperp, s.u1), dot3(eperp, s.u2)}, {dot3(epar_i, s.u1), dot3(epar_i, s.u2)}};
    cplx Jl[2][2], Jr[2][2], Jt[2][2];
    for (int a = 0; a < 2; a++)
      for (int p = 0; p < 2; p++) Jl[a][p] = Rot[a][0] * s.J[0][p] + Rot[a][1] * s.J[1][p];
    for (int p = 0; p < 2; p++) {
      Jr[0][p] = rperp * Jl[0][p];
      Jr[1][p] = rpar * Jl[1][p];
      Jt[0][p] = tperp * Jl[0][p];
      Jt[1][p] = tpar * Jl[1][p];
    }

    /* wavefront equation (Eq. 3) for both branches */
    double s1[3], s2[3];
    surface_basis(nhat, s1, s2);
    mat2 C = curvature_matrix(c, s.r, s1, s2);
    mat2 Pi = projection(s1, s2, s.u1, s.u2);
    double ki = s.n_cur * c->k;
    double kvec_i[3];
    scale3(ki, s.d, kvec_i);
    double epar_r[3], epar_t[3];
    cross3(dr, eperp, epar_r);
    mat2 Pr = projection(s1, s2, eperp, epar_r);
    double kvec_r[3];
    scale3(ki, dr, kvec_r);
    mat2 Qr = wavefront_equation(s.Q, ki, Pi, ki, Pr, C, nhat, kvec_i, kvec_r);
    mat2 Qt;
    double kt = n_oth * c->k;
    if (!tir) {
      cross3(dt, eperp, epar_t);
      mat2 Pt = projection(s1, s2, eperp, epar_t);
      double kvec_t[3];
      scale3(kt, dt, kvec_t);
      Qt = wavefront_equation(s.Q, ki, Pi, kt, Pt, C, nhat, kvec_i, kvec_t);
    }

    /* emission and choice of the continuing branch (reading R8) */
    int cont_is_t;
    if (q == 1) {
      if (0 >= c->p_min && 0 <= c->p_max) emit_order(c, &s, dr, eperp, epar_r, Qr, Jr, &out->emit[0]);
      if (tir) return;
      cont_is_t = 1;
    } else {
      int p = q - 1;
      if (!tir && p >= c->p_min && p <= c->p_max) emit_order(c, &s, dt, eperp, epar_t, Qt, Jt, &out->emit[p]);
      cont_is_t = 0;
    }

    /* record the continuing branch right after the interaction */
    const double* dnext = cont_is_t ? dt : dr;
    mat2 Qn = cont_is_t ? Qt : Qr;
    out->q_cont[q - 1][0] = Qn.m[0][0];
    out->q_cont[q - 1][1] = 0.5 * (Qn.m[0][1] + Qn.m[1][0]);
    out->q_cont[q - 1][2] = Qn.m[1][1];
    matvec(c->R, eperp, out->eperp_cont[q - 1]);
    matvec(c->R, dnext, out->dir_cont[q - 1]);
    if (q == c->p_max + 1) break;

    /* take the continuing branch */
    copy3(dnext, s.d);
    copy3(eperp, s.u1);
    cross3(s.d, s.u1, s.u2);
    s.Q = Qn;
    for (int a = 0; a < 2; a++)
      for (int p = 0; p < 2; p++) s.J[a][p] = cont_is_t ? Jt[a][p] : Jr[a][p];
    if (cont_is_t) s.n_cur = n_oth;

    /* free propagation to the next interaction (chord of the ellipsoid) */
    double Ar2[3], Ad2[3];
    Avec(c, s.r, Ar2);
    Avec(c, s.d, Ad2);
    double L = -2.0 * dot3(s.d, Ar2) / dot3(s.d, Ad2);
    mat2 G;
    G.m[0][0] = 1.0 + L * s.Q.m[0][0];
    G.m[0][1] = L * s.Q.m[0][1];
    G.m[1][0] = L * s.Q.m[1][0];
    G.m[1][1] = 1.0 + L * s.Q.m[1][1];
    s.D /= fabs(m2det(G));         /* Eq. 6: ratio of Gaussian curvatures */
    s.nf += m2neg(G);              /* focal lines crossed on this segment */
    s.Q = m2mul(s.Q, m2inv(G));    /* Q(L) = Q (I + L Q)^{-1} */
    s.opl += s.n_cur * c->k * L;   /* Eq. 9 path term */
    if (s.n_cur != 1.0 && c->m_im > 0.0) {
      /* R14: attenuation along an internal segment */
      double att = exp(-c->k * c->m_im * L);
      for (int a = 0; a < 2; a++)
        for (int p = 0; p < 2; p++) s.J[a][p] *= att;
    }
    for (int i = 0; i < 3; i++) s.r[i] += L * s.d[i];
  }
}

static int setup_ctx(const rtwo_particle* part, const rtwo_setup* st, ctx_t* c) {
  if (!part || !st) return -1;
  for (int i = 0; i < 3; i++)
    if (!(part->semi_axes[i] > 0.0)) return -1;
  if (!(part->m > 0.0) || part->m == 1.0) return -1;
  if (!(part->m_im >= 0.0) || !isfinite(part->m_im)) return -1;
  if (!(st->wavelength > 0.0)) return -1;
  if (st->n_pol < 1 || st->n_pol > 2) return -1;
  if (st->p_min < 0 || st->p_max < st->p_min || st->p_max > RTWO_MAX_ORDER) return -1;
  double amax = fmax(part->semi_axes[0], fmax(part->semi_axes[1], part->semi_axes[2]));
  if (!(st->source_distance == 0.0 || st->source_distance > amax)) return -1;
  if (!(st->observation_radius == 0.0 || st->observation_radius > amax)) return -1;
  if (st->corrections & ~(RTWO_CAUSTIC | RTWO_DIFFRACTION)) return -1;
  /* the Fraunhofer term of R13 is that of a plane wave in the far field */
  if ((st->corrections & RTWO_DIFFRACTION) && (st->source_distance != 0.0 || st->observation_radius != 0.0))
    return -1;
  c->corr = st->corrections;
  c->zs = st->source_distance;
  c->robs = st->observation_radius;
  for (int i = 0; i < 3; i++) c->A[i] = 1.0 / (part->semi_axes[i] * part->semi_axes[i]);
  euler_zyz(part->euler_deg, c->R);
  c->k = 2.0 * PI / st->wavelength;
  c->m = part->m;
  c->m_im = part->m_im;
  c->n_pol = st->n_pol;
  c->p_min = st->p_min;
  c->p_max = st->p_max;
  return 0;
}

int rtwo_trace_rays(const rtwo_particle* part, const rtwo_setup* setup, int n, const double* xy, rtwo_ray* out) {
  ctx_t c;
  if (setup_ctx(part, setup, &c) != 0 || n < 0 || (n > 0 && (!xy || !out))) return -1;
#pragma omp parallel for schedule(static) num_threads(rtwo_get_threads())
  for (int i = 0; i < n; i++) trace_one(&c, xy[2 * i], xy[2 * i + 1], &out[i]);
  return 0;
}

double rtwo_grid_halfwidth(const rtwo_particle* part) {
  double R[3][3];
  euler_zyz(part->euler_deg, R);
  double Sxx = 0, Syy = 0;
  for (int k = 0; k < 3; k++) {
    double s2 = part->semi_axes[k] * part->semi_axes[k];
    Sxx += R[0][k] * R[0][k] * s2;
    Syy += R[1][k] * R[1][k] * s2;
  }
  double L = sqrt(Sxx);
  if (sqrt(Syy) > L) L = sqrt(Syy);
  return L;
}

/* Point source S = (0, 0, -z_s): the rays from S that touch the particle form
 * its tangent cone; the grid's half-width is the cone's largest extent along
 * lab x or y on the plane z = 0.  With D = X - S, the line S + t D meets
 * X^T M X = 1 (M = R diag(1/a^2) R^T) in a double root exactly when
 * (D^T M S)^2 = (D^T M D)(S^T M S - 1), i.e. D^T K D = 0 with
 * K = z_s^2 (m m^T - m_z M) + M, m = M e_z (so S^T M S = z_s^2 m_z).  On z = 0,
 * D = (x, y, z_s); the extreme x = c of that conic is where the quadratic in
 * y has a double root, a quadratic in c (likewise for y). */
double rtwo_grid_halfwidth_source(const rtwo_particle* part, double source_distance) {
  if (!(source_distance > 0.0)) return rtwo_grid_halfwidth(part);
  double zs = source_distance, R[3][3], M[3][3], K[3][3];
  euler_zyz(part->euler_deg, R);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      M[i][j] = 0.0;
      for (int k = 0; k < 3; k++) M[i][j] += R[i][k] * R[j][k] / (part->semi_axes[k] * part->semi_axes[k]);
    }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) K[i][j] = zs * zs * (M[i][2] * M[j][2] - M[2][2] * M[i][j]) + M[i][j];
  double L = 0.0;
  for (int i = 0; i < 2; i++) {
    int j = 1 - i;
    double A = K[i][j] * K[i][j] - K[j][j] * K[i][i];
    double B = 2.0 * zs * (K[i][j] * K[j][2] - K[j][j] * K[i][2]);
    double C = zs * zs * (K[j][2] * K[j][2] - K[j][j] * K[2][2]);
    double sq = sqrt(B * B - 4.0 * A * C);
    L = fmax(L, fmax(fabs((-B + sq) / (2.0 * A)), fabs((-B - sq) / (2.0 * A))));
  }
  return L;
}

/* Compact per-ray record used by the far-field assembly. */
typedef struct {
  int valid, nf, det_neg;
  double dir[3], kr[3];
  double phase;  /* path and focal-line phase at dir (rad), unreduced */
  cplx f[2][3];
} cray;

int rtwo_trace_grid(const rtwo_particle* part, const rtwo_setup* setup, int* flags, double* dir, double* rexit,
                    double* phase, double* amp, double* field) {
  ctx_t c;
  if (setup_ctx(part, setup, &c) != 0 || setup->grid_n < 2) return -1;
  int N = setup->grid_n, n_ord = c.p_max - c.p_min + 1;
  long NN = (long)N * N;
  double L = rtwo_grid_halfwidth_source(part, setup->source_distance), h = 2.0 * L / N;
#pragma omp parallel for schedule(static) num_threads(rtwo_get_threads())
  for (int iy = 0; iy < N; iy++) {
    rtwo_ray ray;
    for (int ix = 0; ix < N; ix++) {
      long id = (long)iy * N + ix;
      trace_one(&c, -L + (ix + 0.5) * h, -L + (iy + 0.5) * h, &ray);
      for (int o = 0; o < n_ord; o++) {
        const rtwo_emit* e = &ray.emit[c.p_min + o];
        int valid = ray.active && e->valid;
        if (flags) flags[o * NN + id] = valid ? (1 | (e->nf << 1) | (e->det_neg << 8)) : 0;
        for (int x = 0; x < 3; x++) {
          if (dir) dir[(o * 3 + x) * NN + id] = valid ? e->dir[x] : 0.0;
          if (rexit) rexit[(o * 3 + x) * NN + id] = valid ? e->rexit[x] : 0.0;
        }
        if (phase) phase[o * NN + id] = valid ? e->phase : 0.0;
        if (amp) amp[o * NN + id] = valid ? e->amp : 0.0;
        if (field)
          for (int p = 0; p < c.n_pol; p++)
            for (int x = 0; x < 3; x++)
              for (int ri = 0; ri < 2; ri++)
                field[((((long)o * c.n_pol + p) * 3 + x) * 2 + ri) * NN + id] = valid ? e->field[p][x][ri] : 0.0;
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* far-field assembly (RTW strategy: parametrise by incident ray,       */
/* interpolate, sum coherently)                                         */
/* ------------------------------------------------------------------ */

/* indices [lo, hi) of sorted v[] with lo_val <= v < = hi_val */
static int lower_idx(const double* v, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (v[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}
static int upper_idx(const double* v, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (v[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

typedef struct {
  int n_theta, n_phi;
  const double* th;  /* radians */
  const double* ph;  /* radians */
  double* nvec;      /* [n_nodes][3] */
  double* etheta;    /* [n_nodes][3] */
  double* ephi;      /* [n_nodes][3] */
} nodes_t;

/* Visit every node whose direction lies in the spherical cap of angular radius
 * rho about the unit vector cdir (a conservative superset of a triangle). */
typedef void (*node_fn)(int node, void* user);
static void for_nodes_in_cap(const nodes_t* nd, const double* cdir, double rho, node_fn fn, void* user) {
  double cz = cdir[2];
  if (cz > 1.0) cz = 1.0;
  if (cz < -1.0) cz = -1.0;
  double thc = acos(cz);
  double phc = atan2(cdir[1], cdir[0]);
  if (phc < 0) phc += 2.0 * PI;
  double tlo = thc - rho, thi = thc + rho;
  int full_phi = 0;
  double dphi = 0.0;
  if (tlo <= 0.0 || thi >= PI || rho >= PI / 2) full_phi = 1;
  else {
    double sr = sin(rho) / sin(thc);
    if (sr >= 1.0) full_phi = 1;
    else dphi = asin(sr);
  }
  int i0 = lower_idx(nd->th, nd->n_theta, tlo);
  int i1 = upper_idx(nd->th, nd->n_theta, thi);
  for (int it = i0; it < i1; it++) {
    if (full_phi) {
      for (int ip = 0; ip < nd->n_phi; ip++) fn(it * nd->n_phi + ip, user);
      continue;
    }
    /* phi interval [phc - dphi, phc + dphi] on the circle, split at 0/2pi */
    double plo = phc - dphi, phi_hi = phc + dphi;
    double seg[2][2];
    int nseg = 0;
    if (plo < 0) { seg[nseg][0] = plo + 2 * PI; seg[nseg][1] = 2 * PI; nseg++; seg[nseg][0] = 0; seg[nseg][1] = phi_hi; nseg++; }
    else if (phi_hi >= 2 * PI) { seg[nseg][0] = plo; seg[nseg][1] = 2 * PI; nseg++; seg[nseg][0] = 0; seg[nseg][1] = phi_hi - 2 * PI; nseg++; }
    else { seg[nseg][0] = plo; seg[nseg][1] = phi_hi; nseg++; }
    for (int sg = 0; sg < nseg; sg++) {
      int j0 = lower_idx(nd->ph, nd->n_phi, seg[sg][0]);
      int j1 = upper_idx(nd->ph, nd->n_phi, seg[sg][1]);
      for (int ip = j0; ip < j1; ip++) fn(it * nd->n_phi + ip, user);
    }
  }
}

typedef struct {
  const nodes_t* nd;
  const cray* v[3];      /* vertices in triangle order */
  double kappa;          /* k R at a finite observation radius, 0 in the far field */
  long vid[3];           /* global ray ids (canonical edge orientation) */
  int n_pol;
  double* field;         /* accumulators */
  double* incoh;
  int* nflags;
  int* ncontrib;
  double* uncancelled;
  long n_nodes;
  struct clist* list;    /* R12: contributions kept per node instead of summed (NULL: summed) */
  int slot;              /* order slot of the triangle */
} tri_job;

/* One triangle's contribution to one node, kept for the fold-caustic form. */
typedef struct {
  long node, seq;
  int nf;
  double phi;      /* barycentric mean of the rays' phases carried to the node */
  cplx f[2][2];    /* [pol][theta|phi] */
} centry;
struct clist {
  centry* e;
  long n, cap;
};
static void clist_push(struct clist* L, const centry* x) {
  if (L->n == L->cap) {
    L->cap = L->cap ? 2 * L->cap : 4096;
    L->e = realloc(L->e, sizeof(centry) * (size_t)L->cap);
  }
  L->e[L->n] = *x;
  L->e[L->n].seq = L->n;
  L->n++;
}

/* Edge function of the canonical edge (lower ray id first): (d_i x d_j) . n */
static double edge_fn(const double* di, const double* dj, const double* n) {
  double cr[3];
  cross3(di, dj, cr);
  return dot3(cr, n);
}

static void tri_node(int node, void* user) {
  tri_job* J = (tri_job*)user;
  const double* n = &J->nd->nvec[3 * (long)node];
  double w[3];
  int inside = 1;
  for (int k = 0; k < 3; k++) {
    int a = (k + 1) % 3, b = (k + 2) % 3;   /* edge opposite vertex k */
    const cray *vi = J->v[a], *vj = J->v[b];
    if (J->vid[a] > J->vid[b]) { const cray* t = vi; vi = vj; vj = t; }
    double e = edge_fn(vi->dir, vj->dir, n);
    double side = edge_fn(vi->dir, vj->dir, J->v[k]->dir);
    w[k] = e / side;
    int ok = (e * side > 0.0) || (e == 0.0 && side > 0.0);
    if (!ok) inside = 0;
  }
  double sw = w[0] + w[1] + w[2];
  /* tie detection (watertight rule decides; the flag only marks closeness) */
  if (sw > 0.0) {
    double l0 = w[0] / sw, l1 = w[1] / sw, l2 = w[2] / sw;
    double mn = l0 < l1 ? l0 : l1;
    if (l2 < mn) mn = l2;
    if (mn > -1e-9 && mn < 1e-9) J->nflags[node] |= 1;
  }
  if (!inside) return;
  double lam[3] = {w[0] / sw, w[1] / sw, w[2] / sw};
  const double* et = &J->nd->etheta[3 * (long)node];
  const double* ep = &J->nd->ephi[3 * (long)node];
  centry ce;
  memset(&ce, 0, sizeof(ce));
  ce.node = node;
  ce.nf = J->v[0]->nf;
  for (int k = 0; k < 3; k++) {
    /* the ray's phase carried to the node (the argument of its carry) */
    const cray* v = J->v[k];
    double dn[3] = {n[0] - v->dir[0], n[1] - v->dir[1], n[2] - v->dir[2]}, carry;
    if (J->kappa > 0.0) {
      double a[3], b[3];
      for (int x = 0; x < 3; x++) {
        a[x] = J->kappa * n[x] - v->kr[x];
        b[x] = J->kappa * v->dir[x] - v->kr[x];
      }
      carry = -dot3(v->kr, dn) * 2.0 * J->kappa / (norm3(a) + norm3(b));
    } else {
      carry = -dot3(v->kr, dn);
    }
    ce.phi += lam[k] * (v->phase + carry);
  }
  for (int p = 0; p < J->n_pol; p++) {
    cplx ft = 0, fp = 0;
    double ut = 0, up = 0; /* magnitudes of the summed terms (before cancellation) */
    for (int k = 0; k < 3; k++) {
      const cray* v = J->v[k];
      double dn[3] = {n[0] - v->dir[0], n[1] - v->dir[1], n[2] - v->dir[2]};
      cplx carry;
      if (J->kappa > 0.0) {
        /* path difference from the exit point to R n and to R u (reading R11):
           |a| - |b| with a = kR n - k r, b = kR u - k r.  For unit n and u,
           |a|^2 - |b|^2 = 2 kR k r.(u - n), so |a| - |b| is that over |a| + |b|,
           which avoids subtracting two lengths near kR */
        double a[3], b[3];
        for (int x = 0; x < 3; x++) {
          a[x] = J->kappa * n[x] - v->kr[x];
          b[x] = J->kappa * v->dir[x] - v->kr[x];
        }
        carry = cexp(I * (-dot3(v->kr, dn) * 2.0 * J->kappa / (norm3(a) + norm3(b))));
      } else {
        carry = cexp(-I * dot3(v->kr, dn));  /* stationary-phase gradient */
      }
      cplx vt = 0, vp = 0;
      for (int x = 0; x < 3; x++) { vt += v->f[p][x] * et[x]; vp += v->f[p][x] * ep[x]; }
      ft += lam[k] * carry * vt;
      fp += lam[k] * carry * vp;
      ut += fabs(lam[k]) * cabs(vt);
      up += fabs(lam[k]) * cabs(vp);
    }
    if (J->uncancelled) J->uncancelled[node] += ut * ut + up * up;
    ce.f[p][0] = ft;
    ce.f[p][1] = fp;
    if (!J->list) {
      long base_t = ((long)(p * 2 + 0) * J->n_nodes + node) * 2;
      long base_p = ((long)(p * 2 + 1) * J->n_nodes + node) * 2;
      J->field[base_t] += creal(ft); J->field[base_t + 1] += cimag(ft);
      J->field[base_p] += creal(fp); J->field[base_p + 1] += cimag(fp);
    }
    J->incoh[node] += creal(ft * conj(ft)) + creal(fp * conj(fp));
  }
  if (J->list) clist_push(J->list, &ce);
  J->ncontrib[node] += 1;
}

/* ---- special functions of the corrections ---- */

/* Ai(-z), Ai'(-z) for z >= 0.  Below z = 10: Taylor steps of the Airy
 * equation y'' = x y toward x = -z (steps of at most 1/2; at x0 the series
 * y(x0 + t) = sum c_n t^n has (n + 2)(n + 1) c_{n+2} = x0 c_n + c_{n-1}),
 * started from Ai(0) = 3^{-2/3} / Gamma(2/3) and Ai'(0) = -3^{-1/3} / Gamma(1/3).
 * From z = 10 on: the asymptotic expansions of Abramowitz & Stegun 10.4.60 and
 * 10.4.62 in xi = (2/3) z^{3/2}, twelve terms (their error is below 1e-13 there). */
void rtwo_airy_neg(double z, double* ai, double* aip) {
  if (z < 10.0) {
    double y = 1.0 / (pow(3.0, 2.0 / 3.0) * tgamma(2.0 / 3.0));
    double yp = -1.0 / (pow(3.0, 1.0 / 3.0) * tgamma(1.0 / 3.0));
    double x0 = 0.0;
    int steps = (int)ceil(z / 0.5);
    double t = steps > 0 ? -z / steps : 0.0;
    for (int s = 0; s < steps; s++) {
      double c[64];
      c[0] = y;
      c[1] = yp;
      c[2] = x0 * c[0] / 2.0;
      for (int n = 1; n + 2 < 64; n++) c[n + 2] = (x0 * c[n] + c[n - 1]) / ((double)(n + 2) * (double)(n + 1));
      double ny = 0.0, nyp = 0.0, tp = 1.0;
      for (int n = 0; n < 64; n++) {
        ny += c[n] * tp;
        if (n + 1 < 64) nyp += (double)(n + 1) * c[n + 1] * tp;
        tp *= t;
      }
      y = ny;
      yp = nyp;
      x0 += t;
    }
    *ai = y;
    *aip = yp;
    return;
  }
  double xi = 2.0 / 3.0 * z * sqrt(z);
  double u[12], v[12];
  u[0] = v[0] = 1.0;
  for (int k = 1; k < 12; k++) {
    u[k] = u[k - 1] * (6.0 * k - 5.0) * (6.0 * k - 3.0) * (6.0 * k - 1.0) / ((2.0 * k - 1.0) * 216.0 * k);
    v[k] = -u[k] * (6.0 * k + 1.0) / (6.0 * k - 1.0);
  }
  double P = 0, Q = 0, Rr = 0, S = 0, xk = 1.0;
  for (int k = 0; k < 12; k++) {
    double sg = ((k / 2) % 2 == 0) ? 1.0 : -1.0;
    if (k % 2 == 0) { P += sg * u[k] / xk; Rr += sg * v[k] / xk; }
    else { Q += sg * u[k] / xk; S += sg * v[k] / xk; }
    xk *= xi;
  }
  double sn = sin(xi + PI / 4.0), cs = cos(xi + PI / 4.0);
  *ai = (sn * P - cs * Q) / (sqrt(PI) * pow(z, 0.25));
  *aip = -pow(z, 0.25) * (cs * Rr + sn * S) / sqrt(PI);
}

/* J1(x).  For |x| < 25 Miller's backward recurrence J_{n-1} = (2n / x) J_n -
 * J_{n+1}, normalised by J_0 + 2 (J_2 + J_4 + ...) = 1; beyond, Hankel's
 * asymptotic expansion (Abramowitz & Stegun 9.2.5, 9.2.9, 9.2.10) with
 * fourteen terms. */
double rtwo_bessel_j1(double x) {
  double ax = fabs(x), sg = x < 0 ? -1.0 : 1.0;
  if (ax < 1e-8) return 0.5 * x;
  if (ax < 25.0) {
    int M = 2 * ((int)(ax + 15.0 + sqrt(40.0 * ax)) / 2);
    double jp1 = 0.0, j = 1e-30, j1 = 0.0, norm = 0.0;
    for (int n = M; n >= 1; n--) {
      double jm1 = 2.0 * n / ax * j - jp1;
      jp1 = j;
      j = jm1;               /* j = J_{n-1} (unnormalised) */
      if (n - 1 == 1) j1 = j;
      if ((n - 1) % 2 == 0 && n - 1 > 0) norm += 2.0 * j;
      if (fabs(j) > 1e250) { j *= 1e-250; jp1 *= 1e-250; j1 *= 1e-250; norm *= 1e-250; }
    }
    norm += j;               /* J_0 */
    return sg * j1 / norm;
  }
  double P = 0, Q = 0, a = 1.0, xk = 1.0;
  for (int k = 0; k < 14; k++) {
    /* a_k(1) = prod_{j=1..k} (4 - (2j - 1)^2) / (k! 8^k) */
    if (k > 0) a *= (4.0 - (2.0 * k - 1.0) * (2.0 * k - 1.0)) / (8.0 * k);
    double sgn = ((k / 2) % 2 == 0) ? 1.0 : -1.0;
    if (k % 2 == 0) P += sgn * a / xk;
    else Q += sgn * a / xk;
    xk *= ax;
  }
  double chi = ax - 0.75 * PI;
  return sg * sqrt(2.0 / (PI * ax)) * (P * cos(chi) - Q * sin(chi));
}

static int centry_cmp(const void* pa, const void* pb) {
  const centry *a = pa, *b = pb;
  if (a->node != b->node) return a->node < b->node ? -1 : 1;
  return a->seq < b->seq ? -1 : (a->seq > b->seq ? 1 : 0);
}

/* R12: the kept contributions of one order, node by node: a pair of branches
 * with focal-line counts n, n + 1 becomes the uniform Airy form, everything
 * else is summed as it is. */
static void caustic_combine(struct clist* L, int n_pol, long n_nodes, double* field) {
  qsort(L->e, (size_t)L->n, sizeof(centry), centry_cmp);
  for (long i = 0; i < L->n;) {
    long j = i;
    while (j < L->n && L->e[j].node == L->e[i].node) j++;
    const long node = L->e[i].node;
    cplx out[2][2] = {{0, 0}, {0, 0}};
    int done = 0;
    if (j - i == 2 && abs(L->e[i].nf - L->e[i + 1].nf) == 1) {
      const centry* a = L->e[i].nf < L->e[i + 1].nf ? &L->e[i] : &L->e[i + 1];
      const centry* b = a == &L->e[i] ? &L->e[i + 1] : &L->e[i];
      double delta = 0.5 * (b->phi - a->phi) + PI / 4.0;
      if (delta > 0.0) {
        double zeta = pow(1.5 * delta, 2.0 / 3.0), ai, aip;
        rtwo_airy_neg(zeta, &ai, &aip);
        cplx ea = cexp(I * delta), eb = cexp(-I * delta);
        double z4 = pow(zeta, 0.25);
        cplx pre = sqrt(PI) * cexp(-I * PI / 4.0);
        for (int p = 0; p < n_pol; p++)
          for (int c = 0; c < 2; c++) {
            cplx sum = a->f[p][c] * ea + I * b->f[p][c] * eb;
            cplx dif = a->f[p][c] * ea - I * b->f[p][c] * eb;
            out[p][c] = pre * (sum * z4 * ai - I * dif * aip / z4);
          }
        done = 1;
      }
    }
    if (!done)
      for (long q = i; q < j; q++)
        for (int p = 0; p < n_pol; p++)
          for (int c = 0; c < 2; c++) out[p][c] += L->e[q].f[p][c];
    for (int p = 0; p < n_pol; p++)
      for (int c = 0; c < 2; c++) {
        long base = ((long)(p * 2 + c) * n_nodes + node) * 2;
        field[base] += creal(out[p][c]);
        field[base + 1] += cimag(out[p][c]);
      }
    i = j;
  }
  L->n = 0;
}

typedef struct { int* nflags; } band_job;
static void band_node(int node, void* user) { ((band_job*)user)->nflags[node] |= 2; }
static double ang(const double* a, const double* b);
/* nodes within `band` of the great-circle segment a-b (a == b: of the point a):
   the segment along which an order's field ends (bit 3) */
typedef struct { int* nflags; const nodes_t* nd; const double *a, *b; double band; } edge_job;
static void edge_node(int node, void* user) {
  const edge_job* E = (const edge_job*)user;
  const double* n = &E->nd->nvec[3 * (long)node];
  double c[3];
  cross3(E->a, E->b, c);
  double cn = norm3(c), dist;
  double da = ang(n, E->a), db = ang(n, E->b);
  dist = da < db ? da : db;
  if (cn > 0.0) {
    /* foot of the node on the great circle lies between a and b when it is on
       the inner side of both end planes */
    double pa[3], pb[3];
    cross3(c, E->a, pa); /* points from a toward b within the circle */
    cross3(E->b, c, pb); /* points from b toward a */
    if (dot3(n, pa) >= 0.0 && dot3(n, pb) >= 0.0) {
      double s = fabs(dot3(n, c)) / cn;
      double d = asin(s > 1.0 ? 1.0 : s);
      if (d < dist) dist = d;
    }
  }
  if (dist <= E->band) E->nflags[node] |= 8;
}

static void unit_centroid(const double* a, const double* b, const double* c, double* o) {
  double s[3] = {a[0] + b[0] + c[0], a[1] + b[1] + c[1], a[2] + b[2] + c[2]};
  scale3(1.0 / norm3(s), s, o);
}
/* Angle between two unit vectors from their chord (accurate for tiny angles). */
static double ang(const double* a, const double* b) {
  double df[3] = {a[0] - b[0], a[1] - b[1], a[2] - b[2]};
  double h = 0.5 * norm3(df);
  if (h > 1.0) h = 1.0;
  return 2.0 * asin(h);
}

int rtwo_farfield(const rtwo_particle* part, const rtwo_setup* setup, int n_theta, const double* theta_deg,
                  int n_phi, const double* phi_deg, double band_deg, double edge_band_deg, double* field,
                  double* incoh, int* nflags, int* ncontrib, double* uncancelled) {
  ctx_t c;
  if (setup_ctx(part, setup, &c) != 0 || setup->grid_n < 2 || n_theta < 1 || n_phi < 1 || !theta_deg ||
      !phi_deg || !field)
    return -1;
  for (int i = 1; i < n_theta; i++) if (!(theta_deg[i] > theta_deg[i - 1])) return -1;
  for (int i = 1; i < n_phi; i++) if (!(phi_deg[i] > phi_deg[i - 1])) return -1;
  if (theta_deg[0] < 0 || theta_deg[n_theta - 1] > 180 || phi_deg[0] < 0 || phi_deg[n_phi - 1] >= 360) return -1;

  int N = setup->grid_n, n_ord = c.p_max - c.p_min + 1, n_pol = c.n_pol;
  long NN = (long)N * N, n_nodes = (long)n_theta * n_phi;
  double L = rtwo_grid_halfwidth_source(part, setup->source_distance), h = 2.0 * L / N;
  double band = band_deg * PI / 180.0, edge_band = edge_band_deg * PI / 180.0;

  /* node directions and the lab (e_theta, e_phi) basis */
  double* th = malloc(sizeof(double) * n_theta);
  double* ph = malloc(sizeof(double) * n_phi);
  for (int i = 0; i < n_theta; i++) th[i] = theta_deg[i] * PI / 180.0;
  for (int i = 0; i < n_phi; i++) ph[i] = phi_deg[i] * PI / 180.0;
  nodes_t nd = {n_theta, n_phi, th, ph, malloc(sizeof(double) * 3 * n_nodes), malloc(sizeof(double) * 3 * n_nodes),
                malloc(sizeof(double) * 3 * n_nodes)};
  for (int i = 0; i < n_theta; i++)
    for (int j = 0; j < n_phi; j++) {
      long id = (long)i * n_phi + j;
      double st = sin(th[i]), ct = cos(th[i]), sp = sin(ph[j]), cp = cos(ph[j]);
      double* n = &nd.nvec[3 * id];
      n[0] = st * cp; n[1] = st * sp; n[2] = ct;
      double* et = &nd.etheta[3 * id];
      et[0] = ct * cp; et[1] = ct * sp; et[2] = -st;
      double* ep = &nd.ephi[3 * id];
      ep[0] = -sp; ep[1] = cp; ep[2] = 0.0;
    }

  double* inc_buf = incoh ? incoh : malloc(sizeof(double) * n_nodes);
  int* fl_buf = nflags ? nflags : malloc(sizeof(int) * n_nodes);
  int* nc_buf = ncontrib ? ncontrib : malloc(sizeof(int) * n_nodes);
  memset(field, 0, sizeof(double) * 2 * 2 * n_pol * n_nodes);
  memset(inc_buf, 0, sizeof(double) * n_nodes);
  memset(fl_buf, 0, sizeof(int) * n_nodes);
  memset(nc_buf, 0, sizeof(int) * n_nodes);
  if (uncancelled) memset(uncancelled, 0, sizeof(double) * n_nodes);

  /* per-ray records of every order */
  cray* rec = malloc(sizeof(cray) * (size_t)n_ord * NN);
#pragma omp parallel for schedule(static) num_threads(rtwo_get_threads())
  for (int iy = 0; iy < N; iy++) {
    rtwo_ray ray;
    for (int ix = 0; ix < N; ix++) {
      long id = (long)iy * N + ix;
      trace_one(&c, -L + (ix + 0.5) * h, -L + (iy + 0.5) * h, &ray);
      for (int o = 0; o < n_ord; o++) {
        const rtwo_emit* e = &ray.emit[c.p_min + o];
        cray* r = &rec[o * NN + id];
        memset(r, 0, sizeof(*r));
        r->valid = ray.active && e->valid;
        if (!r->valid) continue;
        r->nf = e->nf;
        r->phase = e->phase;
        r->det_neg = e->det_neg;
        for (int x = 0; x < 3; x++) {
          /* node-space direction: the exit direction, or at a finite radius
             (R11) the direction of M */
          r->dir[x] = c.robs > 0.0 ? e->obs[x] : e->dir[x];
          r->kr[x] = c.k * e->rexit[x];
        }
        for (int p = 0; p < 2; p++) {
          for (int x = 0; x < 3; x++) r->f[p][x] = e->field[p][x][0] + I * e->field[p][x][1];
          if (c.robs > 0.0) {
            /* the part tangent to the sphere at M */
            cplx fr = r->f[p][0] * r->dir[0] + r->f[p][1] * r->dir[1] + r->f[p][2] * r->dir[2];
            for (int x = 0; x < 3; x++) r->f[p][x] -= fr * r->dir[x];
          }
        }
      }
    }
  }

  /* rasterise every triangle of every order into the node grid */
  struct clist clist = {NULL, 0, 0};
  for (int o = 0; o < n_ord; o++) {
    for (int iy = 0; iy + 1 < N; iy++)
      for (int ix = 0; ix + 1 < N; ix++) {
        long v00 = (long)iy * N + ix, v10 = v00 + 1, v01 = v00 + N, v11 = v00 + N + 1;
        long tris[2][3] = {{v00, v10, v11}, {v00, v11, v01}};
        for (int t = 0; t < 2; t++) {
          const cray* V[3];
          int all_valid = 1;
          for (int k = 0; k < 3; k++) {
            V[k] = &rec[o * NN + tris[t][k]];
            if (!V[k]->valid) all_valid = 0;
          }
          if (!all_valid) {
            /* a triangle on the edge of the order's sheet (one or two of its
               rays do not emit the order): the field ends along the segment
               between its emitting rays, so mark the nodes within the band of
               that segment (or of a lone emitting ray) */
            int kv[3], nv = 0;
            for (int k = 0; k < 3; k++)
              if (V[k]->valid) kv[nv++] = k;
            if (nv == 0) continue;
            edge_job ej = {fl_buf, &nd, V[kv[0]]->dir, V[kv[nv - 1]]->dir, edge_band};
            double ce[3];
            if (nv == 1) copy3(ej.a, ce);
            else {
              double s2[3] = {ej.a[0] + ej.b[0], ej.a[1] + ej.b[1], ej.a[2] + ej.b[2]};
              scale3(1.0 / norm3(s2), s2, ce);
            }
            for_nodes_in_cap(&nd, ce, ang(ce, ej.a) + edge_band + 1e-9, edge_node, &ej);
            continue;
          }
          /* an edge of the incident grid (both rays in its first or last row
             or column) also ends the sheet: no ray lies beyond it, so mark the
             nodes within the band of its image as well */
          for (int k = 0; k < 3; k++) {
            long ra = tris[t][(k + 1) % 3], rb = tris[t][(k + 2) % 3];
            long ya = ra / N, xa = ra % N, yb = rb / N, xb = rb % N;
            int on_grid_edge = (ya == yb && (ya == 0 || ya == N - 1)) || (xa == xb && (xa == 0 || xa == N - 1));
            if (!on_grid_edge) continue;
            edge_job ej = {fl_buf, &nd, V[(k + 1) % 3]->dir, V[(k + 2) % 3]->dir, edge_band};
            double s2[3] = {ej.a[0] + ej.b[0], ej.a[1] + ej.b[1], ej.a[2] + ej.b[2]}, ce[3];
            scale3(1.0 / norm3(s2), s2, ce);
            for_nodes_in_cap(&nd, ce, ang(ce, ej.a) + edge_band + 1e-9, edge_node, &ej);
          }
          double cen[3];
          unit_centroid(V[0]->dir, V[1]->dir, V[2]->dir, cen);
          double rho = ang(cen, V[0]->dir);
          for (int k = 1; k < 3; k++) {
            double a2 = ang(cen, V[k]->dir);
            if (a2 > rho) rho = a2;
          }
          /* The direction map ray -> exit direction is orientation preserving
           * or reversing as (-1)^nf: a fold (caustic at infinity) changes nf by
           * one, whereas a focal line crossing the exit interface flips
           * sign(det Q') through infinity but leaves nf and the map unchanged. */
          int same = V[0]->nf == V[1]->nf && V[0]->nf == V[2]->nf;
          if (!same) {
            /* fold triangle: dropped; mark the caustic band around it */
            band_job bj = {fl_buf};
            for_nodes_in_cap(&nd, cen, rho + band + 1e-9, band_node, &bj);
            continue;
          }
          double cr[3];
          cross3(V[0]->dir, V[1]->dir, cr);
          if (dot3(cr, V[2]->dir) == 0.0) continue; /* degenerate */
          tri_job J;
          J.nd = &nd;
          for (int k = 0; k < 3; k++) { J.v[k] = V[k]; J.vid[k] = tris[t][k]; }
          J.n_pol = n_pol;
          J.kappa = c.robs > 0.0 ? c.k * c.robs : 0.0;
          J.field = field;
          J.incoh = inc_buf;
          J.nflags = fl_buf;
          J.ncontrib = nc_buf;
          J.uncancelled = uncancelled;
          J.n_nodes = n_nodes;
          J.list = (c.corr & RTWO_CAUSTIC) ? &clist : NULL;
          J.slot = o;
          for_nodes_in_cap(&nd, cen, rho * (1.0 + 1e-9) + 1e-12, tri_node, &J);
        }
      }
    if (c.corr & RTWO_CAUSTIC) caustic_combine(&clist, n_pol, n_nodes, field);
  }
  free(clist.e);
  if (c.corr & RTWO_DIFFRACTION) {
    /* R13: the shadow's Fraunhofer amplitude, S2 = x-y block of R diag(a^2) R^T */
    double S2[2][2];
    for (int i = 0; i < 2; i++)
      for (int j = 0; j < 2; j++) {
        S2[i][j] = 0.0;
        for (int q = 0; q < 3; q++)
          S2[i][j] += c.R[i][q] * c.R[j][q] * part->semi_axes[q] * part->semi_axes[q];
      }
    double area = PI * sqrt(S2[0][0] * S2[1][1] - S2[0][1] * S2[1][0]);
    for (long id = 0; id < n_nodes; id++) {
      double t = th[id / n_phi], f = ph[id % n_phi];
      double nx = sin(t) * cos(f), ny = sin(t) * sin(f);
      double s = sqrt(S2[0][0] * nx * nx + 2.0 * S2[0][1] * nx * ny + S2[1][1] * ny * ny);
      double u = c.k * s;
      double shape = u < 1e-8 ? 1.0 : 2.0 * rtwo_bessel_j1(u) / u;
      cplx Fd = I * c.k / (2.0 * PI) * area * shape;
      double pol[2][2] = {{cos(f), -sin(f)}, {sin(f), cos(f)}};
      for (int p = 0; p < n_pol; p++)
        for (int a = 0; a < 2; a++) {
          long base = ((long)(p * 2 + a) * n_nodes + id) * 2;
          field[base] += creal(Fd * pol[p][a]);
          field[base + 1] += cimag(Fd * pol[p][a]);
        }
    }
  }
  for (long id = 0; id < n_nodes; id++) {
    double t = th[id / n_phi];
    if (t < band || t > PI - band) fl_buf[id] |= 4;
  }

  free(rec);
  free(nd.nvec); free(nd.etheta); free(nd.ephi);
  free(th); free(ph);
  if (!incoh) free(inc_buf);
  if (!nflags) free(fl_buf);
  if (!ncontrib) free(nc_buf);
  return 0;
}
