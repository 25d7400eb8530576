/*
 * rtw.h -- C ABI of the MI355X-native Ray Theory of Waves library (librtw.so).
 *
 * Method: Ren et al., "Ray Theory of Waves" (arXiv 2403.13856).  A plane wave
 * travelling along lab +z (or the spherical wave of a point source on the
 * -z axis, see rtw_incident) meets one smooth ellipsoid, or each ellipsoid of
 * a batch.  A cell-centred square
 * grid of incident rays is traced; every ray carries a 2x2 wavefront-curvature
 * (WFC) matrix updated at each reflection and refraction by the wavefront
 * equation (Eq. 3), its direction by vector Snell (Eq. 4) and its
 * polarisation by the Fresnel coefficients (Eq. 8) re-evaluated in each
 * incidence plane.  Each order p leaves the particle with the amplitude of
 * Eqs. 5-7 (divergence factor from the WFC) and the phase of Eqs. 9-10 (path,
 * Fresnel and focal-line phases).  The far field on a (theta, phi) grid is the
 * coherent sum of all orders, obtained by interpolating the per-ray fields as
 * functions of the incident ray (section "Strategy of Ray Theory of Waves").
 *
 * Conventions
 *   - lengths in micrometres; angles in degrees at this interface;
 *   - lab frame: incident wave along +z, incident polarisation x (pol 0) and
 *     y (pol 1); theta is measured from +z, phi from +x towards +y;
 *   - body frame: x_lab = R x_body, R = Rz(alpha) Ry(beta) Rz(gamma);
 *   - time dependence exp(-i w t); the far field F(theta, phi) is
 *     lim r exp(-ikr) E(r) / E0, in micrometres, projected on (e_theta, e_phi);
 *     |F|^2 is the differential cross-section (um^2/sr) of the summed orders;
 *   - ray grid: N x N cell-centred over [-L, L]^2 of the plane z = 0,
 *     L = max(sqrt(S_xx), sqrt(S_yy)), S = R diag(a^2, b^2, c^2) R^T, for the
 *     plane wave (for a point source: see rtw_incident); ray index iy*N + ix;
 *   - every device pointer is caller-owned; the library never allocates or
 *     frees caller memory.  All calls are asynchronous on the given HIP stream
 *     (NULL = default stream); argument errors are returned immediately.
 *
 * Return codes: 0 = RTW_OK, negative = error; rtw_last_error() returns the
 * calling thread's message for the last failing call.
 */
#ifndef RTW_H
#define RTW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTW_OK 0
#define RTW_ERR_INVALID_ARG (-1)
#define RTW_ERR_UNSUPPORTED (-2)
#define RTW_ERR_WORKSPACE (-3)
#define RTW_ERR_DEVICE (-4)

#define RTW_FP64 0  /* every step in double precision */
#define RTW_MIXED 1 /* FP32 wave quantities (Fresnel, Jones, WFC, fields) and far-field
                       assembly; FP64 polyline (positions, directions, Snell, chords),
                       path length, phase reduction, divergence factor and caustic
                       Jacobian; rays with an ill-conditioned divergence factor are
                       traced again in FP64 */

#define RTW_MAX_ORDER 15

/* One ellipsoid r^T diag(a^-2, b^-2, c^-2) r = 1 in its body frame.
 * Absorbing particles (m_im > 0; not in the paper): the weak-absorption form
 * of geometric optics -- Snell, Eq. 8 and Eq. 3 use m, and every internal
 * segment of length L scales the carried field by exp(-k m_im L) (the per-ray
 * amplitude record excludes it, the field record includes it). */
typedef struct {
  double semi_axes[3]; /* a, b, c > 0 (um) */
  double euler_deg[3]; /* Z-Y-Z Euler angles (deg), body -> lab */
  double m;            /* real part of the relative refractive index, m > 0, m != 1 */
  double m_im;         /* imaginary part, >= 0 (0: no absorption) */
} rtw_particle;

/* Incident wave (the paper's problem statement: wavelength and polarisation
 * of the incident wave; Eq. 10's incident phase Phi_i for a non-plane wave).
 *   source_distance = 0: plane wave along lab +z, polarisation basis (x, y).
 *   source_distance = z_s > largest semi-axis of every particle: spherical
 *     wave from a point source at lab (0, 0, -z_s).  The ray of grid point
 *     (x, y) runs from the source through the lab point (x, y, 0); at its
 *     first interaction, rho_1 from the source, it has the wavefront
 *     curvature I / rho_1 (diverging), amplitude z_s / rho_1 and phase
 *     k (rho_1 - z_s) (unit amplitude and zero phase at the distance of the
 *     particle centre, so z_s -> infinity gives the plane wave); its
 *     polarisation vectors are lab x made transverse to the ray, and the ray
 *     direction crossed with that.  The incident grid's half-width is the
 *     largest extent along lab x or y of the particle's tangent cone from the
 *     source on the plane z = 0.
 * Observation (Eqs. 6 and 9 at the observation point M):
 *   observation_radius = 0: far field; the nodes are directions and the
 *     output is the far-field amplitude F (um).
 *   observation_radius = R > largest semi-axis of every particle: the nodes
 *     lie on the sphere of radius R about the particle centre.  Each ray is
 *     continued from its exit point r to the point M where it meets the
 *     sphere (d_M further); its divergence factor there is
 *     R sqrt(D / |det(I + d_M Q')|), its focal-line count includes the
 *     negative eigenvalues of I + d_M Q', its phase is OPL + k (d_M - R)
 *     - N_f pi/2.  The output is R e^{-ikR} times the tangential part of E(M)
 *     on the node's (e_theta, e_phi) (R -> infinity gives F).  Triangles are
 *     interpolated over the directions of M, each vertex carried to a node n
 *     by k (|R n - r| - |R u - r|) (u the vertex's direction of M).  The
 *     per-ray records of rtw_trace report amp, phase, focal lines and field
 *     at M; dir and rexit stay the exit direction and point.
 * Other values of source_distance or observation_radius:
 * RTW_ERR_INVALID_ARG. */
typedef struct {
  double wavelength;      /* in the surrounding medium (um) */
  int n_pol;              /* 1: x polarisation only; 2: x and y */
  double source_distance; /* 0: plane wave; z_s (um): point source, see above */
  double observation_radius; /* 0: far field; R (um): nodes on the sphere of radius R */
} rtw_incident;

/* Corrections of the far field beyond the ray sum (rtw_trace_opts.corrections,
 * bit flags; they change rtw_farfield and rtw_batch, not the per-ray records):
 *   RTW_CAUSTIC: wave correction at fold caustics (the rainbows), which the
 *     paper applies near caustics without giving formulas.  Where a node holds
 *     exactly two contributions of one order whose focal-line counts differ by
 *     one (the two branches that coalesce at a fold), their sum is replaced by
 *     the uniform asymptotic Airy form of Chester, Friedman and Ursell (1957),
 *     in Ludwig's (1966) two-ray form: with the branches' fields f_a (N_f = n),
 *     f_b (N_f = n + 1) and their phases phi_a, phi_b carried to the node,
 *     Delta = (phi_b - phi_a) / 2 + pi / 4, (2/3) zeta^{3/2} = Delta,
 *       u = sqrt(pi) e^{-i pi/4} [ (f_a e^{i Delta} + i f_b e^{-i Delta}) zeta^{1/4} Ai(-zeta)
 *                               - i (f_a e^{i Delta} - i f_b e^{-i Delta}) zeta^{-1/4} Ai'(-zeta) ]
 *     (u -> f_a + f_b far from the fold).  Nodes with Delta <= 0 keep the
 *     sum; the dark side of a fold gets no field.
 *   RTW_DIFFRACTION: forward Fraunhofer diffraction of the particle's shadow
 *     (Babinet), added to every node: the shadow on z = 0 is the ellipse
 *     rho^T S2^-1 rho <= 1 (S2 the x-y block of R diag(a^2, b^2, c^2) R^T),
 *     F_d = (i k / 2 pi) pi sqrt(det S2) 2 J1(k s) / (k s), s = sqrt(n_t^T S2 n_t)
 *     with n_t = (sin th cos ph, sin th sin ph), along (cos ph, -sin ph) on
 *     (e_theta, e_phi) for x polarisation and (sin ph, cos ph) for y.  Plane
 *     wave and far field only (else RTW_ERR_UNSUPPORTED).
 * The incoherent sums of rtw_batch (out_incoh) stay those of the ray sum. */
#define RTW_CAUSTIC 1
#define RTW_DIFFRACTION 2

typedef struct {
  int p_min, p_max; /* orders emitted, 0 <= p_min <= p_max <= RTW_MAX_ORDER */
  int grid_n;       /* incident rays per side, >= 2 */
  int precision;    /* RTW_FP64 or RTW_MIXED */
  int corrections;  /* 0, or RTW_CAUSTIC | RTW_DIFFRACTION (far-field calls only) */
} rtw_trace_opts;

/* Observation grid: sorted node angles, DEVICE pointers (caller-owned),
 * theta in [0, 180], phi in [0, 360), both strictly increasing. */
typedef struct {
  int n_theta;
  const double* theta_deg;
  int n_phi;
  const double* phi_deg;
} rtw_grid;

/* Mixed path (RTW_MIXED): a ray whose divergence factor is ill-conditioned in
 * FP32 -- a focal line within a few per cent of an interface, or an exit
 * wavefront near flat (a far-field caustic) -- is traced again in FP64 inside
 * the same kernel; its records then carry FP64-accurate values.
 *
 * Per-ray records written by rtw_trace, all DEVICE pointers, FP64 whatever
 * the precision path (the mixed path converts on store).  o = p - p_min is the
 * order slot, NN = N*N the ray count.  Any pointer may be NULL (not written).
 *   flags [n_ord][NN]            bit0 order emitted, bits 1..7 focal lines N_f,
 *                                bit 8 det Q' < 0 at the exit
 *   dir   [n_ord][3][NN]         lab exit direction
 *   rexit [n_ord][3][NN]         lab exit point (um)
 *   phase [n_ord][NN]            path + focal-line phase, unreduced (rad):
 *                                OPL - k dir.rexit - N_f pi/2
 *   amp   [n_ord][NN]            amplitude sqrt(D/|det Q'|) (um)
 *   field [n_ord][n_pol][3][2][NN]  lab field vector amp e^{i phase}
 *                                (J_perp e_perp + J_par e_par), (re, im)
 *   cond  [n_ord][2][NN]         conditioning of the emission: [0] relative-error
 *                                amplification of the divergence factor (the
 *                                mixed path re-traces in FP64 above its limit),
 *                                [1] growth of a direction perturbation along the
 *                                ray (product of the largest |eig(I + L Q)|) */
typedef struct {
  int32_t* flags;
  double* dir;
  double* rexit;
  double* phase;
  double* amp;
  double* field;
  double* cond;
} rtw_ray_records;

/* Trace the incident grid and store every emitted order (Eqs. 3-10).
 * Errors: RTW_ERR_INVALID_ARG (bad sizes, NULL structs), RTW_ERR_UNSUPPORTED
 * (m == 1, p_max > 15), RTW_ERR_DEVICE (launch failure). */
int rtw_trace(const rtw_particle* part, const rtw_incident* inc, const rtw_trace_opts* opts,
              const rtw_ray_records* out, void* hip_stream);

/* Bytes of device workspace rtw_farfield needs for these arguments, with room
 * for hits_per_node contributions per node on average (0 = library default). */
int rtw_farfield_workspace_size(const rtw_particle* part, const rtw_incident* inc, const rtw_trace_opts* opts,
                                const rtw_grid* grid, double hits_per_node, size_t* bytes);

/* Far field of the summed orders p_min..p_max on the node grid (interpolation
 * of the RTW strategy section, coherent sum over orders and branches).
 *   out_field  DEVICE, [n_pol][2 (theta, phi)][n_theta][n_phi] complex,
 *              interleaved (re, im): double for RTW_FP64, float for RTW_MIXED.
 *   ncontrib   DEVICE int32 [n_theta*n_phi] or NULL: triangle contributions per node.
 * Node grids have fewer than 65536 angles per side (RTW_ERR_INVALID_ARG).
 *   workspace  DEVICE, >= rtw_farfield_workspace_size bytes, 256-byte aligned.
 * Errors as rtw_trace, plus RTW_ERR_UNSUPPORTED when 2 (p_max - p_min + 1)
 * (grid_n - 1)^2 >= 2^31 (triangle keys are 32-bit).
 * The per-node sum is taken in a fixed order (deterministic).  If the hit pool
 * in the workspace overflows, the result is incomplete and
 * rtw_farfield_status() reports RTW_ERR_WORKSPACE with the size needed.
 * The call only queues kernels on hip_stream (no allocation, copy, fill or
 * synchronisation while profiling is off), so it may be captured into a HIP
 * graph; calls that share a workspace must not overlap. */
int rtw_farfield(const rtw_particle* part, const rtw_incident* inc, const rtw_trace_opts* opts,
                 const rtw_grid* grid, void* out_field, int32_t* ncontrib, void* workspace,
                 size_t workspace_bytes, void* hip_stream);

/* ---- Far field without device allocation ---------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * computation and kernels as rtw_farfield, with the workspace taken from a
 * static device array of RTW_STATIC_WORKSPACE_MIB MiB inside the library (one
 * copy per GPU, held until the process ends).  The call allocates and frees
 * nothing; the caller passes the inputs and outputs as for rtw_farfield.
 *   status_out DEVICE int32 [1] or NULL: written on the stream after the sum,
 *              RTW_OK, or RTW_ERR_WORKSPACE if the hit pool overflowed (the
 *              result is then incomplete).
 * Every call on one GPU shares that GPU's array and overwrites what the last
 * call left there (the kernels clear what must start at zero): calls that
 * overlap on one GPU, on different streams or host threads, race.
 * Errors as rtw_farfield, plus RTW_ERR_WORKSPACE, on the host before anything
 * is launched, when the call needs more than the static array at the default
 * pool sizing (6 contributions per node); RTW_ERR_DEVICE when there is no
 * current device.  Profiling events (rtw_profile_enable) are not recorded. */
#define RTW_STATIC_WORKSPACE_MIB 128
int rtw_farfield_static(const rtw_particle* part, const rtw_incident* inc, const rtw_trace_opts* opts,
                        const rtw_grid* grid, void* out_field, int32_t* ncontrib, int32_t* status_out,
                        void* hip_stream);

/* ---- Batches of particles (many ellipsoids, one call) -------------------
 * The same far field for n particles that share the incident wave, the
 * orders, the precision and the node grid, each with its own shape,
 * orientation, index and ray-grid side grid_n[i].  Particles are taken
 * largest first and grouped into chunks of at most rays_per_chunk incident
 * rays; each chunk is traced by one persistent kernel whose blocks take work
 * items (tiles of tile_rays rays of one particle) from a queue, then
 * rasterised and summed like rtw_farfield.  Results are bitwise identical to
 * rtw_farfield of each particle alone with the same tuning.
 * With rtw_batch_opts.fused (RTW_MIXED, at most 6 orders, no RTW_CAUSTIC) one
 * persistent kernel traces, rasterises and forms the hit contributions of
 * 64 x (tile_rays / 64)-ray tiles in LDS (no per-ray records in the
 * workspace); its results are bitwise independent of the tuning and agree
 * with the staged pipeline's within the mixed path's rounding. */
typedef struct {
  int tile_rays;     /* incident rays per trace work item, multiple of 256 (0 = 2048) */
  int blocks_per_cu; /* persistent trace blocks per compute unit (0 = 8) */
  int cand_inline;   /* triangles whose bounding box holds more nodes are rasterised
                        row by row (0 = 4096, the largest allowed) */
} rtw_tune;

typedef struct {
  long long rays_per_chunk; /* incident rays per chunk; the workspace scales with it
                               (0 = 2^26; a larger particle is a chunk of its own) */
  double hits_per_node;     /* hit-pool sizing per node of a chunk (0 = 6) */
  int fused;                /* 1: the fused kernel where it applies (RTW_MIXED, at most 6
                               orders, no RTW_CAUSTIC): trace, rasterisation and hit
                               contributions per ray tile in one persistent kernel, with no
                               per-ray records in the workspace (about a third of the
                               workspace; slower on MI355X); 0: the staged pipeline */
} rtw_batch_opts;

/* Workspace bytes for rtw_batch with these arguments (bopts may be NULL). */
int rtw_batch_workspace_size(int n, const rtw_particle* parts, const int* grid_n, const rtw_incident* inc,
                             const rtw_trace_opts* opts, const rtw_grid* grid, const rtw_batch_opts* bopts,
                             size_t* bytes);

/* Far fields of n particles.  parts and grid_n are HOST arrays [n]; opts gives
 * the orders and precision (its grid_n is ignored).
 *   out_field  DEVICE [n][n_pol][2][n_theta][n_phi] complex (layout and type as
 *              rtw_farfield), particle i at index i.
 *   ncontrib   DEVICE int32 [n][n_theta*n_phi] or NULL.
 *   out_incoh  DEVICE [n][n_pol][n_theta*n_phi] (float for RTW_MIXED, double for
 *              RTW_FP64) or NULL: the incoherent intensity sum_b (|f_b,theta|^2 +
 *              |f_b,phi|^2) of each node's triangle contributions b.
 *   tune       NULL = defaults (see rtw_tune); rtw_batch_autotune picks one.
 * Synchronises hip_stream once to upload the per-particle metadata (a few
 * hundred bytes per particle) into the workspace, then queues the kernels and
 * returns.  Errors as rtw_farfield for any particle (the message names it), plus
 * RTW_ERR_UNSUPPORTED when n_ord grid_n^2 >= 2^30.  Overflow of the hit pool is
 * reported by rtw_farfield_status on the same workspace. */
int rtw_batch(int n, const rtw_particle* parts, const int* grid_n, const rtw_incident* inc,
              const rtw_trace_opts* opts, const rtw_grid* grid, void* out_field, int32_t* ncontrib, void* out_incoh,
              const rtw_tune* tune, const rtw_batch_opts* bopts, void* workspace, size_t workspace_bytes,
              void* hip_stream);

/* Project autotuner: times rtw_batch on a sample of up to 64 of the particles
 * (spread over the size range) for a coordinate search over tile_rays,
 * blocks_per_cu and then cand_inline, and returns the fastest in *best.
 * out_field and workspace are used as scratch (sized as for rtw_batch of all n
 * particles); the call synchronises hip_stream. */
int rtw_batch_autotune(int n, const rtw_particle* parts, const int* grid_n, const rtw_incident* inc,
                       const rtw_trace_opts* opts, const rtw_grid* grid, const rtw_batch_opts* bopts,
                       void* out_field, void* workspace, size_t workspace_bytes, void* hip_stream, rtw_tune* best);

/* Synchronises hip_stream and reports whether the last rtw_farfield or
 * rtw_batch that used this workspace fitted: RTW_OK, or RTW_ERR_WORKSPACE with
 * *bytes_needed set to a workspace size that fits.  bytes_needed may be NULL. */
int rtw_farfield_status(const void* workspace, void* hip_stream, size_t* bytes_needed);

/* Synchronises hip_stream and reads counters of the last rtw_farfield or
 * rtw_batch that used this workspace: the number of node contributions
 * (triangle hits) and, for RTW_MIXED, the number of rays traced again in FP64
 * because their divergence factor was ill-conditioned in FP32.  Either pointer
 * may be NULL. */
int rtw_farfield_stats(const void* workspace, void* hip_stream, uint64_t* hits, uint64_t* fp64_rays);

/* Per-kernel timing for benchmarks: while enabled, every kernel the library
 * launches is bracketed by HIP events on the caller's stream.
 * rtw_profile_read waits for the recorded events and returns, per kernel name,
 * the summed duration (ms) and launch count: names is a caller buffer of
 * max_kernels rows of 64 chars; *n_kernels receives the number of distinct
 * kernels (may exceed max_kernels).  The recorded events are then released. */
int rtw_profile_enable(int on);
int rtw_profile_read(int max_kernels, char* names, double* total_ms, int* launches, int* n_kernels);

/* Restricts the events of rtw_profile_enable to the kernels reported under
 * this name by rtw_profile_read, so that a benchmark timing one kernel inside
 * a timed loop adds two events a launch of it instead of two for every
 * kernel; NULL or "" records every kernel again.  The name is copied. */
int rtw_profile_only(const char* name);

const char* rtw_last_error(void);

/* Library version string. */
const char* rtw_version(void);

#ifdef __cplusplus
}
#endif
#endif
