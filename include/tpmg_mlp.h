/*
 * tpmg_mlp.h -- learned initial guess for sequences of solves (C ABI).
 *
 * The pressure-correction equation is solved once per time step of the
 * semi-implicit scheme (Dedner, Mueller & Scheichl, Section 1 and Section
 * 2.1), and each solve stops at a relative residual, so a better first
 * iterate saves iterations. This module is a per-column multilayer
 * perceptron that predicts the nz values of the solution in a column from
 * the column's nz right-hand-side values plus the vertical means of the
 * right-hand sides of its three horizontal neighbours (n_in = nz + 3):
 *     x  = (features - mu_x) / sd_x
 *     h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3
 *     u0 = y * sd_y + mu_y
 * W1 [hidden][n_in], W2 [hidden][hidden], W3 [nz][hidden]. It is trained by
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the mean
 * squared error of standardised targets. Precision: FP32 master weights and
 * Adam moments; every matrix product runs on the matrix cores with both
 * operands rounded to bfloat16 (nearest, ties to even) and FP32
 * accumulation; biases, the loss and the standardisation are FP32.
 *
 * Conventions are those of tpmg.h: status returns, tpmg_last_error(),
 * caller-owned device buffers (the library allocates no device memory; it
 * carves the workspace given to tpmg_mlp_create), all device work on the
 * stream given at creation. Feature and target rows are FP32, row-major:
 * features [rows][nz + 3], targets [rows][nz]; parameters travel as one
 * packed FP32 array W1, b1, W2, b2, W3, b3 (row-major).
 */
#ifndef TPMG_MLP_H
#define TPMG_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "tpmg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tpmg_mlp tpmg_mlp;

/* Number of packed parameters: hidden (nz + 3) + hidden + hidden^2 + hidden
 * + nz hidden + nz (99,648 for nz 64, hidden 256). */
tpmg_status tpmg_mlp_param_count(int nz, int hidden, size_t* n);

/* Device workspace bytes for a network of this shape that processes at most
 * max_rows rows per call (inference over a grid of n columns needs
 * max_rows >= n; a training batch needs max_rows >= batch). Limits:
 * nz a multiple of 8 in 8..256, hidden in {64, 128, 256, 512},
 * 1 <= max_rows <= 2^22. */
tpmg_status tpmg_mlp_workspace_size(int nz, int hidden, int max_rows, size_t* bytes);

/* Carves d_workspace (device, >= tpmg_mlp_workspace_size bytes, 256-byte
 * aligned). Parameters start at zero and the scaling at mu = 0, sd = 1; set
 * them with tpmg_mlp_set_params / tpmg_mlp_set_scaling or
 * tpmg_mlp_fit_scaling. Errors: TPMG_ERR_ARG, TPMG_ERR_NOMEM. */
tpmg_status tpmg_mlp_create(int nz, int hidden, int max_rows, void* d_workspace, size_t bytes, void* hip_stream,
                            tpmg_mlp** out);

/* Host copies of the packed FP32 parameters (set also resets the Adam
 * moments and step count). Synchronise the stream. */
tpmg_status tpmg_mlp_set_params(tpmg_mlp* m, const float* params);
tpmg_status tpmg_mlp_get_params(tpmg_mlp* m, float* params);

/* Standardisation (host arrays, n_in and nz values; sd > 0 required for
 * set). Any output of get may be NULL. */
tpmg_status tpmg_mlp_set_scaling(tpmg_mlp* m, const double* mu_x, const double* sd_x, const double* mu_y,
                                 const double* sd_y);
tpmg_status tpmg_mlp_get_scaling(const tpmg_mlp* m, double* mu_x, double* sd_x, double* mu_y, double* sd_y);

/* Fits the scaling to rows of device features and targets: per-column mean
 * and population standard deviation, summed in FP64 in a fixed order; a
 * zero deviation becomes 1. Synchronises the stream. */
tpmg_status tpmg_mlp_fit_scaling(tpmg_mlp* m, const float* d_x, const float* d_y, size_t rows);

/* Features of every finest-grid column of mg from a right-hand side d_f
 * (tiled FP64, as tpmg_solve), written to d_x [n_cells][nz + 3]; targets
 * from a solution d_u, written to d_y [n_cells][nz]. mg's nz must equal the
 * network's and (features) n_cells <= max_rows. Asynchronous on the
 * network's stream. */
tpmg_status tpmg_mlp_features(tpmg_mlp* m, const tpmg_mg* mg, const double* d_f, float* d_x);
tpmg_status tpmg_mlp_targets(tpmg_mlp* m, const tpmg_mg* mg, const double* d_u, float* d_y);

/* Standardised outputs d_y [rows][nz] of the network for the raw features
 * d_x [rows][nz + 3] (rows <= max_rows). Asynchronous. */
tpmg_status tpmg_mlp_forward(tpmg_mlp* m, const float* d_x, int rows, float* d_y);

/* Loss (mean squared error of the standardised outputs over the batch) and
 * its gradients with respect to the packed parameters, for the batch of
 * rows d_rows[0 .. batch-1] (device int32 indices into the rows_total rows
 * of d_x and d_y, raw features and raw targets; 1 <= batch <= max_rows).
 * loss and grads are host outputs (either may be NULL). Synchronises the
 * stream. An index outside [0, rows_total) is never dereferenced: its row
 * counts as zeros and the call returns TPMG_ERR_ARG. */
tpmg_status tpmg_mlp_gradients(tpmg_mlp* m, const float* d_x, const float* d_y, size_t rows_total,
                               const int32_t* d_rows, int batch, float* loss, float* grads);

/* One Adam step with learning rate lr on the batch (as tpmg_mlp_gradients).
 * loss (host, optional): the batch loss before the step; passing it
 * synchronises the stream, NULL keeps the call asynchronous (an
 * out-of-range index is then reported by the next synchronising call:
 * train_step with loss, tpmg_mlp_gradients or tpmg_mlp_get_params). */
tpmg_status tpmg_mlp_train_step(tpmg_mlp* m, const float* d_x, const float* d_y, size_t rows_total,
                                const int32_t* d_rows, int batch, float lr, float* loss);

/* steps Adam steps in one call, step k on the batch d_perm[k * batch ..
 * (k + 1) * batch - 1] (device int32 row indices, steps * batch of them):
 * the same launches, in the same order, as steps calls of
 * tpmg_mlp_train_step, so the parameters end bit for bit the same, without
 * a return to the caller between steps. With loss_every > 0, losses (host,
 * at least (steps - 1) / loss_every + 2 floats) receives the batch loss
 * before the step of every step k with k % loss_every == 0 and of the last
 * step, in order; loss_every = 0 samples none (losses may be NULL).
 * Synchronises the stream at the end; an out-of-range row index is reported
 * then (TPMG_ERR_ARG). */
tpmg_status tpmg_mlp_train_epoch(tpmg_mlp* m, const float* d_x, const float* d_y, size_t rows_total,
                                 const int32_t* d_perm, int steps, int batch, float lr, int loss_every, float* losses);

/* Initial guess for mg's solve with right-hand side d_f: features,
 * standardisation, forward pass and de-standardisation (u_hat). relax = 0:
 * u_hat is written into the real columns of d_u0 (tiled FP64; padding
 * entries are not written). relax = 1: one undamped line-relaxation sweep
 * in FP64 follows, d_u0 = u_hat + A_T^-1 (f - A u_hat) (the column solves
 * of the smoother of Section 5, eq. BlockJacobi, with damping 1), which
 * removes the vertically rough part of the network's error, the part the
 * strongly anisotropic operator amplifies most; every entry of d_u0 is
 * written (padding entries stay zero when those of d_f are). Requires
 * n_cells <= max_rows and mg's stream to be the network's. Asynchronous. */
tpmg_status tpmg_mlp_infer(tpmg_mlp* m, const tpmg_mg* mg, const double* d_f, int relax, double* d_u0);

/* The same network on the increments of a sequence of solves. The operator
 * is linear, so between two steps of a sequence the solution changes by the
 * solution for the change of the right-hand side: u_t = u_{t-1} +
 * A^-1 (f_t - f_{t-1}). A network trained on features of f_t - f_{t-1}
 * (tpmg_mlp_features_increment) and targets u_t - u_{t-1}
 * (tpmg_mlp_targets_increment) predicts that change, and
 * tpmg_mlp_infer_increment forms d_u0 = d_u_prev + (the network's output
 * for the features of d_f - d_f_prev), followed with relax = 1 by one
 * undamped FP64 line-relaxation sweep with d_f (as tpmg_mlp_infer). All
 * vectors tiled FP64 as tpmg_solve; d_u0 must not alias an input; every
 * entry of d_u0 is written (padding entries: those of d_u_prev, or with
 * relax = 1 the sweep's). The difference vectors are formed in the
 * network's workspace. Same requirements as tpmg_mlp_features /
 * tpmg_mlp_targets / tpmg_mlp_infer; asynchronous. */
tpmg_status tpmg_mlp_features_increment(tpmg_mlp* m, const tpmg_mg* mg, const double* d_f, const double* d_f_prev,
                                        float* d_x);
tpmg_status tpmg_mlp_targets_increment(tpmg_mlp* m, const tpmg_mg* mg, const double* d_u, const double* d_u_prev,
                                       float* d_y);
tpmg_status tpmg_mlp_infer_increment(tpmg_mlp* m, const tpmg_mg* mg, const double* d_f, const double* d_f_prev,
                                     const double* d_u_prev, int relax, double* d_u0);

/* Parameters, scaling and shape in a binary file (little-endian). load
 * requires the file's shape to match m. */
tpmg_status tpmg_mlp_save(tpmg_mlp* m, const char* path);
tpmg_status tpmg_mlp_load(tpmg_mlp* m, const char* path);

void tpmg_mlp_destroy(tpmg_mlp* m);

#ifdef __cplusplus
}
#endif

#endif /* TPMG_MLP_H */
