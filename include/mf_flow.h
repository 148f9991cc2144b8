/*
 * mf_flow.h -- C ABI of the learned proposal: a coupling normalising flow on
 * the VEGAS y-space of an integrand (MI355X, gfx950).
 *
 * The paper lists new integration algorithms based on deep learning as its
 * next step (arXiv:2105.10529, Sec. 1 and Sec. 4); the proposal here is the
 * piecewise-quadratic coupling flow of Mueller et al., "Neural Importance
 * Sampling" (ACM TOG 38, 2019), on top of a frozen VEGAS grid:
 *
 *  - L coupling layers act on y in (0,1)^d.  Layer l keeps the coordinates
 *    of A_l and maps each coordinate j of B_l by a monotone piecewise-
 *    quadratic CDF whose 2K+1 parameters come from an MLP of y_{A_l}:
 *    d_A -> 256 -> 256 -> |B_l| (2K+1), LeakyReLU with slope 0.01.
 *  - Masks: with nb the bit length of d-1, layer l transforms the coordinates
 *    whose index has bit (l mod nb) set when floor(l/nb) is even, clear when
 *    it is odd.
 *  - Per transformed coordinate the outputs are K width logits then K+1
 *    vertex logits: W = softmax(width logits), V_k = exp(v_k) / N with
 *    N = sum_k W_k (exp(v_k) + exp(v_k+1)) / 2, so that the density is linear
 *    in each bin and integrates to one.
 *  - log q(y) is the sum of the log densities of every transformed coordinate
 *    of every layer.  "Forward" is the density direction y -> z, "inverse"
 *    the sampling direction z -> y.
 *  - Training minimises the forward KL divergence on weighted samples,
 *    L = - sum_i w_i log q(y_i) / sum_i w_i, with Adam.
 *
 * Arithmetic: the three dense layers run as BF16 matrix-core products with
 * FP32 accumulation (weights and activations rounded to BF16, biases FP32);
 * the PQ transform, its derivatives, the loss and Adam run in FP32; the
 * parameters are kept as FP32 master copies.
 *
 * Conventions (as in mf.h): every call returns mf_status and sets
 * mf_last_error(); "device" pointers are HIP device pointers owned by the
 * caller; points are [ndim][n] FP32 structure-of-arrays; `stream` is a
 * hipStream_t or NULL; calls are asynchronous unless stated otherwise.
 * A flow owns one more stream of its own (default priority, created with
 * the flow): mf_flow_loss_grad runs its weight-gradient products there,
 * ordered against `stream` by events, and leaves `stream` waiting for them,
 * so the gradient is complete in `stream` order when the call returns.
 * Calls on one flow must not overlap.
 *
 * Parameter layout (FP32, host): layer after layer, each as
 *   W1 [d_A][256], b1 [256], W2 [256][256], b2 [256],
 *   W3 [256][|B| (2K+1)], b3 [|B| (2K+1)]
 * (row-major [in][out]; output column c(2K+1) + r is output r of the c-th
 * transformed coordinate in increasing coordinate order; the inputs are the
 * kept coordinates in increasing order).  Zero W3 and b3 give the identity
 * map with log q = 0.
 */
#ifndef MF_FLOW_H
#define MF_FLOW_H

#include <stdint.h>

#include "mf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mf_flow mf_flow;

typedef enum {
  MF_FLOW_LOSS_KL = 0,       /* L = - sum w log q / sum w (forward KL) */
  MF_FLOW_LOSS_VARIANCE = 1  /* gradient of log sum w^2 / q: the KL gradient with
                                per-point weights w^2/q held fixed; the reported
                                value is the relative variance per event of
                                sampling q, n sum w^2/q / (sum w)^2 - 1 */
} mf_flow_loss;

typedef struct {
  int32_t ndim;       /* 2..16 */
  int32_t n_layers;   /* 1..8 */
  int32_t hidden;     /* hidden width; only 256 is built */
  int32_t bins;       /* K; only 32 is built */
  int64_t max_batch;  /* largest n accepted by mf_flow_loss_grad (sizes the
                         per-layer activation caches: about
                         n_layers * max_batch * (2 KB + 0.3 KB * ndim) bytes) */
  uint64_t seed;      /* Philox key word 0 of the initial weights */
} mf_flow_config;

/* Create a flow on the current device.  Initial parameters: the weights of
 * the first two dense layers of every coupling layer uniform in
 * +-sqrt(6 / fan_in), drawn from Philox4x64-10 with counter (parameter index,
 * 0, 0, 0) and key (seed, 3); all biases and the output layers zero, so the
 * flow is the identity map (log q = 0) while every parameter receives a
 * gradient.  MF_EINVAL for sizes outside the ranges above, MF_ENOTSUP for
 * another hidden width or bin count, MF_ENOMEM on allocation failure. */
mf_status mf_flow_create(const mf_flow_config* cfg, mf_flow** out);

/* Release the handle and its device memory (NULL is accepted). */
void mf_flow_destroy(mf_flow* f);

/* Number of dimensions of the flow, or 0 for NULL. */
int mf_flow_ndim(const mf_flow* f);

/* Number of FP32 parameters (the length of the layout above), or -1. */
int64_t mf_flow_param_count(const mf_flow* f);

/* Masks, host [n_layers][ndim]: 1 where the layer transforms the coordinate. */
mf_status mf_flow_masks(const mf_flow* f, uint8_t* out);

/* Copy all parameters in (host FP32, exactly param_count values), refresh the
 * BF16 copies, and reset the Adam moments and step counter.  Synchronous. */
mf_status mf_flow_set_params(mf_flow* f, const float* params, int64_t count);

/* Copy the FP32 master parameters out (host, param_count values).
 * Synchronous. */
mf_status mf_flow_get_params(const mf_flow* f, float* params, int64_t count);

/* Density direction: z = T(y) and log q(y) for n points.
 *   y:    device [ndim][n] FP32 in [0,1];   z: device [ndim][n] FP32 output
 *         (may equal y for an in-place transform);
 *   logq: device [n] FP32 output.
 * Any n >= 0 (no cache is kept).  MF_EINVAL for NULL buffers with n > 0. */
mf_status mf_flow_forward(mf_flow* f, const float* y, int64_t n, float* z, float* logq, void* stream);

/* Sampling direction: y = T^-1(z) and log q(y) (the density of the produced
 * point), same buffer conventions as mf_flow_forward. */
mf_status mf_flow_inverse(mf_flow* f, const float* z, int64_t n, float* y, float* logq, void* stream);

/* Loss of one batch of points y (uniform in the flow's space) with weights
 * w (mf_flow_loss) and its gradient with respect to every parameter (the
 * forward pass keeps the activations of the batch, the backward pass runs
 * through the PQ transforms and the layers).  The gradient is kept in the
 * handle for mf_flow_adam_step.
 *   y:    device [ndim][n] FP32;  w: device [n] FP32 with a positive sum
 *   grad: device [param_count] FP32 copy of the gradient, or NULL
 *   loss: host, receives the loss value (the call then synchronises
 *         `stream`), or NULL
 * 1 <= n <= max_batch and a known loss kind, else MF_EINVAL. */
mf_status mf_flow_loss_grad(mf_flow* f, const float* y, const float* w, int64_t n, int32_t loss_kind, float* grad,
                            double* loss, void* stream);

/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) of the
 * FP32 masters with the gradient of the last mf_flow_loss_grad, followed by
 * the refresh of the BF16 copies. */
mf_status mf_flow_adam_step(mf_flow* f, double lr, void* stream);

typedef struct {
  int32_t epochs;     /* passes over the data, >= 1 */
  int64_t batch;      /* events per step, 1..max_batch; the last short batch
                         of an epoch is used as it is */
  double lr;          /* initial learning rate, > 0 */
  double lr_final;    /* learning rate after the last step (cosine decay) */
  void* stream;
  int32_t loss;       /* mf_flow_loss */
} mf_flow_train_opts;

/* Train on n weighted points (mf_flow_loss_grad + mf_flow_adam_step per
 * batch, batches in order).  loss_per_epoch: host [epochs] mean batch loss
 * value, or NULL.  Blocks until done. */
mf_status mf_flow_train(mf_flow* f, const float* y, const float* w, int64_t n, const mf_flow_train_opts* o,
                        double* loss_per_epoch);

typedef struct {
  int32_t steps;         /* training steps, >= 1 */
  int64_t batch;         /* points per step, 2..max_batch of the flow */
  double lr;             /* initial learning rate, > 0 */
  double lr_final;       /* learning rate after the last step (cosine decay) */
  int32_t loss;          /* mf_flow_loss */
  double flow_mix;       /* fraction a of uniform points in the sampling mixture, [0,1) */
  uint64_t iter_offset;  /* Philox iteration word of the first step's batch */
  void* stream;
  int32_t group_steps;   /* steps pooled into one estimate of the integral
                            (0: all steps) */
  double target_rel_err; /* stop once the combined estimate reaches this
                            relative error (0: run all steps) */
} mf_flow_online_opts;

/* On-policy training on the integrand itself: each step draws a batch from
 * the mixture q_m = a + (1 - a) q of the current flow (key word 1, iteration
 * word iter_offset + step, as mf_weights), evaluates the integrand on the
 * frozen grid of the process, and takes a step on the gradient of
 * int p^2 / q_m (variance: per-point weights r^2 q/q_m with r = f J / q_m)
 * or of the forward KL (weights r q/q_m), followed by Adam.  The sample
 * weights r of every batch are unbiased estimates of the integral; the
 * batches of each group of group_steps steps are pooled into one estimate
 * and the groups are combined by inverse variance (as VEGAS combines its
 * iterations), which can stop the training at target_rel_err.
 *   loss_per_step: host [steps], the relative variance per event of each
 *                  batch's weights (n sum r^2 / (sum r)^2 - 1), 0 after an
 *                  early stop, or NULL.
 *   est:           host, receives the combined estimate (integral, error,
 *                  chi2_dof, n_iter_done = groups, n_events_total, seconds,
 *                  time_to_target; group estimates into iter_integral /
 *                  iter_error when those are given, with room for
 *                  ceil(steps / group_steps) values), or NULL.
 * MF_ERANGE (checked at the end of every group) if the proposal produced a
 * non-finite density or Jacobian for any point, which a diverged training
 * step causes; the flow is then left as the last step made it.
 * Blocks until done. */
mf_status mf_flow_train_online(mf_process* p, mf_flow* flow, const mf_flow_online_opts* o, double* loss_per_step,
                               mf_result* est);

#ifdef __cplusplus
}
#endif

#endif /* MF_FLOW_H */
