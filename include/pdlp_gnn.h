/* C ABI of the learned warm start for the MI355X restarted-PDHG LP solver.
 *
 * A bipartite message-passing network over the constraint graph of an LP
 * (constraint node i and variable node j joined by each nonzero a_ij) predicts
 * a starting point (x0, y0) and a primal weight omega0 for pdlp_set_warm_start
 * / pdlp_set_warm_start_batch.  The network, its training and its inference run
 * in HIP kernels for gfx950: 64-wide CSR gathers for the messages and bfloat16
 * MFMA products with FP32 accumulation for the 128 x 64 transforms; FP32 master
 * weights updated by Adam.  The solver's own test decides on a prediction:
 * a warm start changes where Algorithm 1 starts, never its termination test.
 *
 * Network (width H = 64, R = 3 rounds):
 *   scales    s_c = max|c|, s_b = max|b|, s_a = max|a_ij| per LP (1 where 0)
 *   features  variable j: (c_j/s_c, l_j/s_b or 0, u_j/s_b or 0, [l_j finite], [u_j finite])
 *             constraint i: (b_i/s_b, [EQ], [GE], [LE])
 *   messages  mean over neighbours weighted by a_ij/s_a
 *   embed     h_v = relu(f_v W_v0 + b_v0), h_c = relu(f_c W_c0 + b_c0)
 *   round r   h_c = relu([h_c | mean_j w_ij h_v] Phi_r + phi_r)
 *             h_v = relu([h_v | mean_i w_ij h_c] Psi_r + psi_r)
 *   heads     x0_j = (h_v w_x + b_x) s_b/s_a, y0_i = (h_c w_y + b_y) s_c/s_a,
 *             omega0 = exp([mean h_v | mean h_c] w_o + b_o)
 * The flat parameter vector holds, in this order and row-major ([in][out]):
 * W_v0[5][64], b_v0[64], W_c0[4][64], b_c0[64], then for r = 0..2 Phi_r[128][64],
 * phi_r[64], Psi_r[128][64], psi_r[64], then w_x[64], b_x, w_y[64], b_y,
 * w_o[128], b_o: PDLP_GNN_PARAMS floats.
 *
 * Loss of one LP with a solution (x*, y*, omega*): w_x mean_j (xh_j - x*_j s_a/s_b)^2
 * + w_y mean_i (yh_i - y*_i s_a/s_c)^2 + w_o (oh - log omega*)^2, where xh, yh, oh
 * are the head outputs and (w_x, w_y, w_o) the term weights (1 unless set);
 * a step averages it over a range of LPs.
 *
 * Every function returns 0 (PDLP_OK) or a negative PDLP_ERR_* code of pdlp.h. */
#ifndef PDLP_GNN_H
#define PDLP_GNN_H

#include <stdint.h>

#include "pdlp.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PDLP_GNN_PARAMS 50499

typedef struct pdlp_gnn pdlp_gnn;

/* Upload `count` LPs (validated as in pdlp_create) as one graph set: the
 * features, the normalized edge weights and both CSR orientations are built on
 * the device.  x_star[sum n], y_star[sum m] (packed in LP order, user
 * orientation) and omega_star[count] are the training targets; pass NULL for
 * all three when the set is only used for prediction.  omega_star must be > 0.
 * The parameters start at zero; set them with pdlp_gnn_set_params.  The totals
 * of rows, columns and nonzeros must stay below 2^31. */
int pdlp_gnn_create(const pdlp_problem* ps, int32_t count, const double* x_star, const double* y_star,
                    const double* omega_star, void* hip_stream, pdlp_gnn** out);

/* Replace the FP32 master weights (theta[PDLP_GNN_PARAMS], host) and clear the
 * Adam moments and step count. */
int pdlp_gnn_set_params(pdlp_gnn* g, const float* theta);

/* Weights of the three loss terms (finite, >= 0; 1, 1, 1 after create): the
 * terms have very different scales (a primal weight spans decades across a
 * family while scaled x and y entries are small), so a caller balances them. */
int pdlp_gnn_set_loss_weights(pdlp_gnn* g, double w_x, double w_y, double w_o);

/* Copy the FP32 master weights to theta[PDLP_GNN_PARAMS] (host). */
int pdlp_gnn_get_params(pdlp_gnn* g, float* theta);

/* Forward and backward over LPs [first, first + count) of the set: *loss
 * receives the mean loss (NULL to skip), grad[PDLP_GNN_PARAMS] its gradient
 * (host, NULL to skip).  Needs targets.  Weights are not changed. */
int pdlp_gnn_loss_grad(pdlp_gnn* g, int32_t first, int32_t count, double* loss, float* grad);

/* One training step on LPs [first, first + count): forward, backward, then
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with rate lr on the
 * master weights.  *loss (may be NULL) receives the loss before the step. */
int pdlp_gnn_train_step(pdlp_gnn* g, int32_t first, int32_t count, float lr, double* loss);

/* Predictions for LPs [first, first + count), in the LPs' own units and user
 * orientation, packed in LP order: x0[sum n], y0[sum m], omega0[count] (host;
 * any may be NULL). */
int pdlp_gnn_predict(pdlp_gnn* g, int32_t first, int32_t count, double* x0, double* y0, double* omega0);

/* Last error of g, or of the last failed pdlp_gnn_create on this thread when g
 * is NULL.  Never NULL. */
const char* pdlp_gnn_last_error(const pdlp_gnn* g);

/* Release g (NULL-safe). */
void pdlp_gnn_destroy(pdlp_gnn* g);

#ifdef __cplusplus
}
#endif

#endif /* PDLP_GNN_H */
