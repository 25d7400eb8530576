/*
 * rtw_surrogate.h -- C ABI of the learned surrogate of the RTW far field
 * (part of librtw.so).
 *
 * The paper computes every far field by tracing (section "Strategy of Ray
 * Theory of Waves"); this surrogate is not in the paper.  It learns, from far
 * fields that rtw_batch computes, the log of the cell-averaged incoherent
 * intensity
 *     ln I_pol(cell) = ln mean_{nodes in cell} sum_b (|f_b,theta|^2 + |f_b,phi|^2)
 * of each incident polarisation (x, y), b running over the node's triangle
 * contributions (orders and branches).  Averaged over a cell many fringes
 * wide, the coherent intensity |sum_b f_b|^2 tends to this value; sampled at
 * the nodes of a cell it scatters around it by the fringe contrast over the
 * square root of the node count, too much to learn to 1%.  Features:
 *     (b/a, c/a, ln(k rbar), m, alpha, beta, gamma, theta_cell, phi_cell)
 * with rbar = (abc)^(1/3), Euler angles and cell centres in degrees.  The
 * network first maps them to a fixed 23-wide embedding: the 9 normalised
 * features; the particle-frame unit vectors of the incident direction, both
 * polarisations and the cell direction (ZYZ Euler angles, lab = Rz(alpha)
 * Ry(beta) Rz(gamma) body); cos and sin of phi.
 * Network: embedding -> 512 -> ... (6 hidden layers of width 512, GELU) -> 4 outputs:
 * the two means and ln(sigma) of each, sigma being the predicted standard
 * deviation of ln I.  BF16 weights and activations, FP32 accumulation on the
 * matrix cores; FP32 master weights; trained with Adam (b1 = 0.9, b2 =
 * 0.999, eps = 1e-8) on the beta-NLL with beta = 1 (Seitzer et al., ICLR
 * 2022): the Gaussian negative log-likelihood 0.5 (y - mu)^2 / sigma^2 +
 * ln sigma of each output, weighted by sigma^2 held constant, so that the
 * means get the squared-error gradient and sigma^2 tends to the expected
 * squared error; ln sigma is floored at ln 1e-4 (normalised units) in it.  Inputs and targets are normalised inside with the
 * shifts and scales set by rtw_surrogate_set_normalization.
 *
 * Queries whose predicted sigma exceeds a threshold tau (either polarisation)
 * are answered by the RTW path instead (rtw_batch on the query's particle,
 * then the same cell average): the trace is both the fallback and the
 * reference the surrogate's error is measured against.
 *
 * Device pointers are caller-owned except the handle's own parameters and
 * activation buffers, which rtw_surrogate_create allocates and
 * rtw_surrogate_destroy frees.  Calls are asynchronous on hip_stream unless
 * stated.  Errors: RTW_ERR_INVALID_ARG, RTW_ERR_UNSUPPORTED,
 * RTW_ERR_WORKSPACE, RTW_ERR_DEVICE; message in rtw_surrogate_last_error().
 */
#ifndef RTW_SURROGATE_H
#define RTW_SURROGATE_H

#include "rtw.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RTW_SURROGATE_INPUTS 9
#define RTW_SURROGATE_EMBED 23
#define RTW_SURROGATE_WIDTH 512
#define RTW_SURROGATE_DEPTH 6

typedef struct rtw_surrogate rtw_surrogate;

/* Uniform cells on the sphere: cell (tc, pc), tc < n_theta_cells, pc <
 * n_phi_cells, holds the nodes with theta in [theta0 + tc dtheta, theta0 +
 * (tc + 1) dtheta) and phi in [phi0 + pc dphi, phi0 + (pc + 1) dphi) (degrees);
 * cell index tc * n_phi_cells + pc. */
typedef struct {
  int n_theta_cells;
  double theta0_deg, dtheta_deg;
  int n_phi_cells;
  double phi0_deg, dphi_deg;
} rtw_cells;

const char* rtw_surrogate_last_error(void);

/* Number of FP32 parameters in the order of get/set_params: for each layer
 * l = 0..6, W[in][out] then bias[out], with in = 128 for layer 0 (rows >= 23,
 * past the embedding, are zero and stay zero) and out = 128 for the last
 * layer (columns >= 4). */
int rtw_surrogate_param_count(size_t* n);

/* New surrogate with seeded uniform He initialisation (SplitMix64 stream),
 * buffers for up to max_rows rows per forward or training call.  Synchronous. */
int rtw_surrogate_create(uint64_t seed, int max_rows, rtw_surrogate** h);
int rtw_surrogate_destroy(rtw_surrogate* h);

/* Feature and target normalisation (host arrays: 9 feature shifts and scales,
 * 2 target shifts and scales); x_norm = (x - shift) / scale.  Synchronous. */
int rtw_surrogate_set_normalization(rtw_surrogate* h, const float* feat_shift, const float* feat_scale,
                                    const float* target_shift, const float* target_scale);

/* FP32 parameters to / from host memory (synchronous). */
int rtw_surrogate_get_params(rtw_surrogate* h, float* host, size_t n);
int rtw_surrogate_set_params(rtw_surrogate* h, const float* host, size_t n);

/* A trained network to / from a file (synchronous): parameters and
 * normalisation, in this library's own format (magic "RTWS", version 1, the
 * parameter count, 22 normalisation floats -- 9 feature shifts, 9 feature
 * scales, 2 target shifts, 2 target scales -- then the FP32 parameters in the
 * order of get/set_params, host byte order).  Loading a file of another
 * network shape or format gives RTW_ERR_INVALID_ARG and leaves h unchanged. */
int rtw_surrogate_save(rtw_surrogate* h, const char* path);
int rtw_surrogate_load(rtw_surrogate* h, const char* path);

/* Predictions for n feature rows (DEVICE feats [n][9] FP32) into DEVICE pred
 * [n][4] FP32: ln I_x, ln I_y, ln sigma_x, ln sigma_y.  n <= max_rows.  One
 * kernel takes every layer of each tile of 128 rows, the activations held on
 * chip (160 KB of LDS per compute unit; 130 KB used).
 * rtw_surrogate_forward_layered computes the same predictions through the
 * per-layer products that training runs (pre-activations written to the
 * handle's buffers, as the gradient pass needs them); both sum every product
 * in the same order with the same rounding. */
int rtw_surrogate_forward(rtw_surrogate* h, int n, const float* feats, float* pred, void* hip_stream);
int rtw_surrogate_forward_layered(rtw_surrogate* h, int n, const float* feats, float* pred, void* hip_stream);

/* Loss and gradients of the mean beta-NLL over n rows (DEVICE feats
 * [n][9], DEVICE targets [n][2] = ln I_x, ln I_y); *loss (DEVICE float)
 * receives the loss in normalised units.  rtw_surrogate_get_grads reads the
 * gradients (synchronous, parameter order).  train_step also applies one Adam
 * step with learning rate lr. */
int rtw_surrogate_grad(rtw_surrogate* h, int n, const float* feats, const float* targets, float* loss,
                       void* hip_stream);
int rtw_surrogate_get_grads(rtw_surrogate* h, float* host, size_t n);
int rtw_surrogate_train_step(rtw_surrogate* h, int n, const float* feats, const float* targets, float lr,
                             float* loss, void* hip_stream);

/* Host-side features of every (particle, cell centre) pair: feats[p][c][9]
 * (HOST), cell centres given in degrees.  The surrogate models plane-wave
 * incidence and the far field: here and in rtw_surrogate_query a non-zero
 * inc->source_distance or inc->observation_radius gives RTW_ERR_UNSUPPORTED. */
int rtw_surrogate_features(int n_part, const rtw_particle* parts, const rtw_incident* inc, int n_cell,
                           const double* cell_theta_deg, const double* cell_phi_deg, float* feats);

/* ln of the cell average of a per-node intensity (DEVICE intensity
 * [n_part][n_pol][n_theta * n_phi] FP32, e.g. the out_incoh of rtw_batch on
 * the node grid `grid`) into DEVICE out [n_part][n_cells][n_pol]; cells no
 * node falls in give 0, cells of zero intensity ln(1e-30). */
int rtw_cell_log_intensity(int n_part, const float* intensity, int n_pol, const rtw_grid* grid, const rtw_cells* cells,
                           float* out, void* hip_stream);

/* Scratch bytes rtw_surrogate_query needs for these particles (worst case:
 * every particle re-computed). */
int rtw_surrogate_query_scratch_size(int n_part, const rtw_particle* parts, const int* grid_n,
                                     const rtw_incident* inc, const rtw_trace_opts* opts, const rtw_grid* grid,
                                     const rtw_cells* cells, size_t* bytes);

/* Answers n_query queries (DEVICE feats [n][9], q_part [n] particle index,
 * q_cell [n] cell index): the surrogate everywhere (DEVICE pred [n][4]), then
 * every particle with a query whose sigma exceeds tau is traced with rtw_batch
 * (mixed, two polarisations; parts and grid_n are HOST arrays [n_part]) and
 * its queries take the RTW cell values of the incoherent intensity.  DEVICE answer [n][2] = ln I_x, ln I_y;
 * DEVICE used_fallback [n] = 1 where RTW answered; *n_recomputed (host) = the
 * particles traced.  scratch: DEVICE, >= rtw_surrogate_query_scratch_size.
 * Synchronises hip_stream (after the surrogate pass, and before returning). */
int rtw_surrogate_query(rtw_surrogate* h, int n_query, const float* feats, const int32_t* q_part,
                        const int32_t* q_cell, float tau, int n_part, const rtw_particle* parts, const int* grid_n,
                        const rtw_incident* inc, const rtw_trace_opts* opts, const rtw_grid* grid,
                        const rtw_cells* cells, const rtw_tune* tune, float* pred, float* answer,
                        int32_t* used_fallback, void* scratch, size_t scratch_bytes, int* n_recomputed,
                        void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
