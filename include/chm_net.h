/* Learned initial Krylov guess for the time step of chm.h.
 *
 * Between time steps the solution changes smoothly, so the Krylov method can
 * start from a prediction of the new state instead of the old one.  This
 * library provides a small convolutional network that predicts the next
 * increment on the vertex grid of a structured 2D P1 mesh, the kernels that
 * train it, and the switch that lets chm_step start from a prediction.
 *
 * Grid and state layout.  A 2D mesh of nx x ny squares has H = ny + 1 rows
 * and W = nx + 1 columns of vertices, vertex v = row * W + col (the order of a
 * row-by-row structured mesh).  A "state vector" is the solver's block layout
 * of the four fields, 4 * H * W doubles: [2v] phi_p, [2v + 1] phi_n,
 * [2 H W + 2v] mu_p, [2 H W + 2v + 1] mu_n.
 *
 * Features (8 channels) from the states x2 (step n-2) and x1 (step n-1),
 * in the solver: the solutions of the solves of those steps (chm_set_guess):
 * d = x1 - x2 divided by its root mean square per field (sigma_c), and
 * x1 minus its mean divided by the root mean square of that (tau_c); a zero
 * root mean square gives zero features.  Each feature is rounded FP64 ->
 * FP32 -> BF16 (round to nearest even).
 *
 * Network: four 3x3 convolutions, 8 -> 32 -> 32 -> 32 -> 4 channels, with
 * reflective padding of one vertex at the grid boundary (the mirrored value,
 * the discrete form of the no-flux condition of the model's boundary).
 * Weights and activations are BF16, every sum is FP32 (MFMA), biases FP32,
 * ReLU after the first three layers (activations stored as BF16 after the
 * ReLU); the last layer's output y (4 channels, FP32) is not rounded.
 *
 * Guess: x1 + d + sigma_c * y_c, in FP64: linear extrapolation of the last
 * increment plus a learned correction measured in units of that increment.
 * A network whose last layer is zero therefore guesses linear extrapolation.
 *
 * Parameters: CHM_NET_NPARAMS FP32 values, per layer w[3][3][c_in][c_out]
 * (row-major; w[dy][dx] acts on the neighbour at (row + dy - 1, col + dx - 1))
 * followed by b[c_out].
 *
 * Training: the target is t_c = (x0_c - x1_c - d_c) / sigma_c for the
 * solution x0 at step n; the loss is the mean over the samples s of a batch
 * of w_s times the mean of (y - t)^2 over the 4 channels and the unmasked
 * vertices of s, with w_s = 1 / (q_s + 1e-4) and q_s the mean of t^2 over
 * the whole grid and the 4 channels (each sample counts by its error
 * relative to its own target), plus smooth times the same mean of
 * (e_p - e_q)^2 over neighbouring pixel pairs p, q (horizontal and vertical,
 * both unmasked), e = y - t, so that a rough error costs more than a smooth
 * one of the same size (a rough start costs the Krylov solve more
 * iterations); gradients of the loss and of every
 * activation are rounded to BF16, weight gradients are FP32 sums; Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) updates FP32 master
 * parameters.  Training runs on crops of the grid, each padded like the
 * full grid; outputs within 4 vertices (the receptive radius) of a crop edge
 * that lies inside the grid are masked out.
 *
 * Errors: every call returns CHM_OK (0) or a negative CHM_E* code of chm.h
 * and leaves a message for chm_net_last_error.  Device pointers must stay
 * valid until the call returns; calls on one network must not overlap.
 */
#ifndef CHM_NET_H
#define CHM_NET_H

#include <stdint.h>

#include "chm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define CHM_NET_IN 8
#define CHM_NET_WIDTH 32
#define CHM_NET_OUT 4
#define CHM_NET_NPARAMS 21988

/* Initial guess of each step's Krylov solve (chm_set_guess). */
#define CHM_GUESS_PREVIOUS 0   /* the state of the previous step */
#define CHM_GUESS_LINEAR 1     /* linear extrapolation 2 y1 - y2 */
#define CHM_GUESS_LEARNED 2    /* the network's guess (or linear extrapolation) */

typedef struct chm_net chm_net_t;

/* A network with zero parameters and work buffers for up to max_pixels
 * vertices per call (batch * h * w).  stream: a hipStream_t (NULL = default
 * stream) on which every call of this network runs. */
int chm_net_create(int64_t max_pixels, void *stream, chm_net_t **out);
int chm_net_destroy(chm_net_t *net);
const char *chm_net_last_error(const chm_net_t *net);

/* Host FP32 parameters in and out (CHM_NET_NPARAMS values).  set_params also
 * clears the Adam moments and step count. */
int chm_net_set_params(chm_net_t *net, const float *params);
int chm_net_get_params(chm_net_t *net, float *params);

/* Features of the state pair (x2, x1) on an H x W grid (device state
 * vectors) into a device FP32 array [H][W][8] holding the BF16 values, and
 * sigma[4] to the host (may be NULL).  H, W >= 2. */
int chm_net_features(chm_net_t *net, int32_t H, int32_t W, const double *x2, const double *x1,
                     float *feats, double *sigma);

/* Network output y [batch][h][w][4] (device FP32) for device FP32 features
 * [batch][h][w][8] (rounded to BF16 on entry).  h, w >= 2. */
int chm_net_forward(chm_net_t *net, int32_t batch, int32_t h, int32_t w, const float *feats,
                    float *y);

/* Loss and parameter gradients (host, CHM_NET_NPARAMS FP32 values, the layout
 * of the parameters) for device features [batch][h][w][8], targets
 * [batch][h][w][4] (FP32), mask [batch][h][w] (0 or 1), host sample
 * weights[batch] (NULL: all 1) and the neighbour-difference weight smooth
 * (>= 0, see the loss above).  loss may be NULL.  The parameters are not
 * changed. */
int chm_net_gradients(chm_net_t *net, int32_t batch, int32_t h, int32_t w, const float *feats,
                      const float *target, const uint8_t *mask, const double *weights,
                      float smooth, float *grads, double *loss);

/* One Adam step with host gradients grads[CHM_NET_NPARAMS] and step size lr. */
int chm_net_adam(chm_net_t *net, const float *grads, float lr);

/* The guess for step n from device state vectors x2 (step n-2) and x1
 * (step n-1) on an H x W grid, into the device state vector guess. */
int chm_net_guess(chm_net_t *net, int32_t H, int32_t W, const double *x2, const double *x1,
                  double *guess);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the guess
 * of chm_net_guess with every work buffer (frame statistics, features,
 * hidden activations, network output) in one fixed device array that the
 * library holds on each GPU it runs on until the process ends (about 11 MB),
 * instead of the network's own buffers.  The same kernels in the same order,
 * so the same bits as chm_net_guess.  The network's max_pixels does not
 * limit it; H * W must be at most CHM_NET_NOALLOC_MAX_PIXELS (a 257 x 257
 * vertex grid), else CHM_EINVAL.  It calls no hipMalloc, hipFree or other
 * allocating routine.  The work is enqueued on the network's stream and the
 * call returns without waiting for it (synchronise the stream before
 * reading guess).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (from any network, stream or thread) race, so the
 * caller serialises them. */
#define CHM_NET_NOALLOC_MAX_PIXELS 66049
int chm_net_guess_noalloc(chm_net_t *net, int32_t H, int32_t W, const double *x2,
                          const double *x1, double *guess);

/* One training step on a batch of crops: sample i takes the device state
 * vectors x2[i], x1[i], x0[i] (steps n-2, n-1, n of one run on the H x W
 * grid; the arrays of pointers are host arrays), the crop of crop_h x crop_w
 * vertices with top-left vertex (oy[i], ox[i]); features, targets and masks
 * as above, forward, loss (neighbour-difference weight smooth), backward and
 * one Adam step with step size lr.  loss (may be NULL) receives the batch
 * loss before the step. */
int chm_net_train_step(chm_net_t *net, int32_t batch, int32_t H, int32_t W, int32_t crop_h,
                       int32_t crop_w, const double *const *x2, const double *const *x1,
                       const double *const *x0, const int32_t *oy, const int32_t *ox, float lr,
                       float smooth, double *loss);

/* Choose how chm_step starts each Krylov solve (CHM_GUESS_*).  The
 * candidates are built from the last two solutions of the solve, y_{n-2} and
 * y_{n-1} (taken before the solvent removal, so that they extrapolate to the
 * next solution and not to the next stored state; the state set by
 * chm_set_fields counts as a solution), so the first step after chm_create or
 * chm_set_fields starts from the previous state.  LINEAR offers the linear
 * extrapolation 2 y_{n-1} - y_{n-2}, LEARNED that and the network's guess;
 * each species starts from whichever of the offered candidates and the
 * previous state has the smallest residual 2-norm in the first block row of
 * the saddle-point system (ties: the simpler one; chm_stats_t.guess_used and
 * .res0, the start's full relative residual, report the choice).
 * LEARNED needs net (used on the solver's stream, kept by the caller until
 * replaced or the solver is destroyed) and a structured mesh with
 * H * W = n_vertices in the vertex order described above (H, W >= 2, at most
 * the network's max_pixels). */
int chm_set_guess(chm_solver_t *s, int32_t mode, chm_net_t *net, int32_t H, int32_t W);

/* Copy a state vector (4 n_vertices doubles, layout above; run 0 of a batch)
 * into device memory: which = 0 the current state, 1 the last solution of the
 * solve (the current state before the solvent removal of the last step; the
 * state set by chm_set_fields before the first step).  The learned guess is
 * trained on the sequence of solutions (which = 1). */
int chm_get_state(chm_solver_t *s, int32_t which, double *state);

#ifdef __cplusplus
}
#endif

#endif /* CHM_NET_H */
