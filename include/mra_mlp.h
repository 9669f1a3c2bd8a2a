/*
 * mra_mlp.h -- C ABI of the learned surrogate of the MRA log-likelihood: a
 * small fully connected network from log-parameters to log-likelihood, with
 * its own FP32 forward, backward and Adam kernels on gfx950.
 *
 * The likelihood it stands in for is the MRA log-likelihood of mra.h (the
 * likelihood mode of Sec. 2.2 of Huang, Blake & Hammerling).  The paper's
 * optimisation mode is a sequence of likelihood evaluations over the
 * covariance parameters sill, range and nugget (Sec. 2.2); the surrogate is
 * fitted to such evaluations and proposes parameters, which the exact MRA
 * then judges.  The network, its training and the proposal step are not part
 * of the paper.
 *
 * Network (fixed shape):
 *   u   = 2 (x - x_lo) / (x_hi - x_lo) - 1       x = (log sill, log range, log nugget)
 *   h_1 = silu(W_1 u + b_1),  W_1: 128 x 3
 *   h_k = silu(W_k h_{k-1} + b_k),  W_k: 128 x 128,  k = 2, 3, 4
 *   s   = w_5 . h_4 + b_5
 *   y   = y_mean + y_std * s                     (FP64 on output)
 * silu(t) = t / (1 + exp(-t)).
 *
 * Parameter vector (MRA_MLP_NPARAM floats, this order, row-major matrices):
 *   W_1 (128x3), b_1 (128), W_2 (128x128), b_2, W_3, b_3, W_4, b_4, w_5 (128), b_5 (1).
 *
 * Training loss on a batch of B pairs (x_b, y_b):
 *   L = (1/B) sum_b (s_b - t_b)^2,   t_b = (y_b - y_mean) / y_std.
 * Adam (Kingma & Ba): m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 *   p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t = step count.
 *
 * Memory: x (B x 3 floats) and y (B doubles) are host or device pointers, both
 * in the same space (device pointers: asynchronous on the given stream; host:
 * returns when done).  The network's parameters and Adam state live on the
 * device, owned by the handle.  All reductions are in a fixed order: results
 * are deterministic.  Status codes are those of mra.h; mra_last_error() holds
 * the message.
 */
#ifndef MRA_MLP_H
#define MRA_MLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mra_mlp mra_mlp;

#define MRA_MLP_WIDTH 128
#define MRA_MLP_NPARAM 50177

/*
 * Create a network with the given initial parameters (MRA_MLP_NPARAM floats,
 * host memory; the caller draws them).  Scaling defaults: x in [-1, 1]^3,
 * y_mean = 0, y_std = 1; Adam state zero, step count 0.
 */
int mra_mlp_create(const float *params, mra_mlp **out);

/* Input box (x_lo, x_hi: 3 values each, x_hi > x_lo) and target scaling (y_std > 0). */
int mra_mlp_set_scaling(mra_mlp *net, const double *x_lo, const double *x_hi, double y_mean, double y_std);

/* y[b] = network(x[b]) for B inputs, de-standardised, FP64 out. */
int mra_mlp_forward(mra_mlp *net, const float *x, int64_t B, double *y, void *stream);

/*
 * Loss L and its gradient with respect to every parameter (MRA_MLP_NPARAM
 * floats, written to grad in the memory space of x; may be NULL) on one batch;
 * parameters and Adam state unchanged.  loss: one double in the memory space
 * of x (may be NULL).
 */
int mra_mlp_loss_grad(mra_mlp *net, const float *x, const double *y, int64_t B, float *grad, double *loss,
                      void *stream);

/* One Adam step on one batch (forward, loss, backward, update); loss as above (before the update). */
int mra_mlp_train_step(mra_mlp *net, const float *x, const double *y, int64_t B, float lr, float beta1,
                       float beta2, float eps, double *loss, void *stream);

/* Copy the current parameters (MRA_MLP_NPARAM floats) to host or device memory. */
int mra_mlp_get_params(mra_mlp *net, float *params);

/* Release the network.  NULL is allowed. */
void mra_mlp_free(mra_mlp *net);

#ifdef __cplusplus
}
#endif
#endif /* MRA_MLP_H */
