/*
 * rtw_oracle.h -- plain FP64 CPU oracle of the Ray Theory of Waves far-field
 * path (Ren et al., "Ray Theory of Waves", arXiv 2403.13856).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the GPU path can be
 * checked against an obviously-correct, slow implementation written directly
 * from the paper.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header, table or constant
 * with the HIP library and must never be linked into the product path.
 *
 * Units: lengths in micrometres, angles in degrees at this interface.
 * Lab frame: the incident plane wave travels along +z (or a spherical wave
 * from a point source on the -z axis, see rtwo_setup), polarisation basis
 * (x, y).  Body frame: x_lab = R x_body with R = Rz(alpha) Ry(beta) Rz(gamma)
 * (intrinsic Z-Y-Z Euler angles).  Time dependence exp(-i w t), so the
 * propagation phase grows as +k * path.
 *
 * Every entry point is pinned by the CPU tests tests/test_oracle_*.py against
 * closed forms, identities, symmetries, finite differences and the paper's
 * Table 1, not against its own formulas.
 */
#ifndef RTW_ORACLE_H
#define RTW_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define RTWO_MAX_ORDER 15 /* p_max limit */

typedef struct {
  double semi_axes[3]; /* a, b, c > 0 along body x, y, z (um) */
  double euler_deg[3]; /* Z-Y-Z Euler angles (deg), body -> lab */
  double m;            /* real part of the relative refractive index, m > 0, m != 1 */
  double m_im;         /* its imaginary part, >= 0: weak absorption (reading R14) */
} rtwo_particle;

typedef struct {
  double wavelength; /* in the surrounding medium (um) */
  int n_pol;         /* 1: x-polarised incidence only, 2: x and y */
  int p_min, p_max;  /* orders emitted, 0 <= p_min <= p_max <= 15 */
  int grid_n;        /* incident ray grid is grid_n x grid_n, cell centred */
  double source_distance; /* 0: plane wave along +z; > largest semi-axis: point source
                             at lab (0, 0, -source_distance), spherical wave (reading R10) */
  double observation_radius; /* 0: far field; > largest semi-axis: the nodes lie on the
                                sphere of this radius and the output is R e^{-ikR} E(M)
                                (reading R11) */
  int corrections;   /* bit 0 (RTWO_CAUSTIC): uniform Airy form across fold caustics
                        (reading R12); bit 1 (RTWO_DIFFRACTION): forward Fraunhofer
                        diffraction of the particle's shadow (reading R13); plane wave
                        and far field only */
} rtwo_setup;

#define RTWO_CAUSTIC 1
#define RTWO_DIFFRACTION 2

/* Everything the oracle knows about one emitted order of one ray. */
typedef struct {
  int valid;       /* 1 if this order leaves the particle for this ray */
  int nf;          /* focal lines crossed, far-field leg included */
  int det_neg;     /* 1 if det Q' < 0 at the exit */
  int tir_any;     /* 1 if any interaction on the way was total internal reflection */
  double dir[3];   /* lab exit direction (unit) */
  double rexit[3]; /* lab exit point (um) */
  double opl;      /* accumulated path phase up to the exit point (rad), incident k z1 included */
  double phase;    /* opl - k dir.rexit - nf*pi/2 (rad), unreduced */
  double amp;      /* S = sqrt(D / |det Q'|) (um) */
  double D;        /* product of Gaussian-curvature ratios over internal segments */
  double q[3];     /* Q' at the exit in (e_perp, e_par'), entries q11, q12, q22 (1/um) */
  double eperp[3]; /* lab e_perp of the last interaction */
  double epar[3];  /* lab e_par' = dir x e_perp */
  double jones[2][2][2]; /* [perp|par][incident pol x|y][re|im], Fresnel product only */
  double field[2][3][2]; /* [pol][lab xyz][re|im] = amp e^{i phase} (J_perp e_perp + J_par e_par') */
  double obs[3];   /* finite observation radius R: unit vector of the point where the ray
                      meets the sphere of radius R (then amp, phase, nf and field refer to
                      that point: amp = R sqrt(D / |det(I + d_M Q')|), phase = OPL + k (d_M - R)
                      - nf pi/2); zero in the far field */
} rtwo_emit;

/* Per-ray trace: the interaction polyline and the WFC after each interaction. */
typedef struct {
  int active;                                /* ray meets the particle */
  int n_hits;                                /* interaction points recorded */
  double hit[RTWO_MAX_ORDER + 2][3];         /* lab interaction points r_1 .. */
  double q_cont[RTWO_MAX_ORDER + 2][3];      /* Q of the continuing branch right after each interaction */
  double eperp_cont[RTWO_MAX_ORDER + 2][3];  /* lab basis vector 1 of that branch */
  double dir_cont[RTWO_MAX_ORDER + 2][3];    /* lab direction of that branch */
  rtwo_emit emit[RTWO_MAX_ORDER + 1];        /* indexed by order p */
} rtwo_ray;

/* Trace n rays through lab-plane points xy[2*i], xy[2*i+1] (um); out[i]
 * receives the full diagnostic record.  Returns 0 on success, <0 on bad input. */
int rtwo_trace_rays(const rtwo_particle* part, const rtwo_setup* setup,
                    int n, const double* xy, rtwo_ray* out);

/* Half-width L of the square incident grid: the projected ellipse's extent
 * along lab x and y, L = max(sqrt(S_xx), sqrt(S_yy)), S = R diag(a^2,b^2,c^2) R^T. */
double rtwo_grid_halfwidth(const rtwo_particle* part);

/* Half-width of the grid for a point source at source_distance (> 0): the
 * largest extent along lab x or y, on the plane z = 0, of the particle's
 * tangent cone from the source; the plane-wave L at 0. */
double rtwo_grid_halfwidth_source(const rtwo_particle* part, double source_distance);

/* Trace the full cell-centred grid.  Ray index = iy*N + ix, lab point
 * (-L + (ix+1/2) 2L/N, -L + (iy+1/2) 2L/N) with
 * L = rtwo_grid_halfwidth_source(part, setup->source_distance).  Outputs are per order slot
 * o = p - p_min, SoA, all caller-owned host arrays:
 *   flags [n_ord][N*N]   bit0 valid, bits1..7 nf, bit8 det_neg
 *   dir   [n_ord][3][N*N]  rexit [n_ord][3][N*N]  phase [n_ord][N*N]  amp [n_ord][N*N]
 *   field [n_ord][n_pol][3][2][N*N]
 * Any output pointer may be NULL. */
int rtwo_trace_grid(const rtwo_particle* part, const rtwo_setup* setup,
                    int* flags, double* dir, double* rexit, double* phase,
                    double* amp, double* field);

/* Far field on the node grid theta_deg[n_theta] x phi_deg[n_phi] (both sorted
 * ascending, theta in [0,180], phi in [0,360)).  Outputs (caller-owned):
 *   field  [n_pol][2 (theta,phi)][n_theta][n_phi][2 (re,im)]
 *   incoh  [n_theta*n_phi]  sum over contributions b of |f_b|^2 (pols, comps)
 *   nflags [n_theta*n_phi]  bit0 tie node (a barycentric weight within 1e-9 of 0),
 *                           bit1 within band_deg of a dropped fold triangle,
 *                           bit2 within band_deg of theta = 0 or 180,
 *                           bit3 within edge_band_deg of the edge of an order's sheet:
 *                           the segment between the emitting rays of a triangle some
 *                           of whose rays do not emit the order, or an edge of the
 *                           incident grid (no ray lies beyond it)
 *   ncontrib[n_theta*n_phi] number of triangle contributions
 *   uncancelled[n_theta*n_phi] sum over contributions of (sum over the three
 *                           rays of |lambda_v| |F_v|)^2 (pols, comps): the size of
 *                           the interpolated terms before they cancel
 * incoh, nflags, ncontrib and uncancelled may be NULL. */
int rtwo_farfield(const rtwo_particle* part, const rtwo_setup* setup,
                  int n_theta, const double* theta_deg, int n_phi, const double* phi_deg,
                  double band_deg, double edge_band_deg, double* field, double* incoh, int* nflags, int* ncontrib,
                  double* uncancelled);

/* Airy function and its derivative on the negative axis: ai = Ai(-z), aip =
 * Ai'(-z) for z >= 0 (Taylor stepping of Ai'' = x Ai from the values at 0 below
 * z = 10, the asymptotic expansion beyond). */
void rtwo_airy_neg(double z, double* ai, double* aip);

/* Bessel function of the first kind of order one. */
double rtwo_bessel_j1(double x);

/* Fresnel coefficients of the paper's Eq. 8 for a real relative index m_rel =
 * n_other/n_current and the incidence cosine ci (0 < ci <= 1).  Outputs
 * complex r_perp, r_par, t_perp, t_par as (re,im) pairs in out[8], and the
 * transmitted normal wave-vector ratio k_rn/k_in (complex) in out[8..9]. */
void rtwo_fresnel(double m_rel, double ci, double* out10);

/* Threads the oracle's OpenMP loops may use (0 = library default). */
void rtwo_set_threads(int n);
int rtwo_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
