/*
 * Learned normalised/offset min-sum: the check update of Sec. III with its
 * constants lambda and beta replaced by one pair (a, b) per iteration t and
 * check-degree class c, unrolled over T iterations in binary32, with the
 * forward pass and its adjoint on the device (for training the pairs).
 *
 *   t_mn     = Z^(t-1)_n - L^(t-1)_mn,        Z^(0) = channel LLR, L^(0) = 0
 *   L^(t)_mn = prod_{n' != n} sgn(t_mn') * max(a[t,c_m] min_{n' != n} |t_mn'| - b[t,c_m], 0)
 *   Z^(t)_n  = Z^(0)_n + sum_{m in M(n)} L^(t)_mn   (ascending check order)
 *   loss_t   = sum_f sum_n softplus(s_fn Z^(t)_fn), s = 2x - 1 for the
 *              transmitted bit x (bit 0 wants Z > 0)
 * Classes: the distinct row degrees of H in ascending order (at most 8);
 * row degrees at most 32.  Binary32 as in the FP32 decoder: a*m rounded
 * before b is subtracted, no FMA.
 *
 * Conventions as in ldpc.h (device pointers on the handle's device,
 * asynchronous on `stream`, no allocation, no synchronisation).
 */
#ifndef LDPC_LEARN_H
#define LDPC_LEARN_H

#include "ldpc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of check-degree classes C and their degrees (host, C entries, or
 * NULL), ascending. */
ldpc_status ldpc_learn_classes(const ldpc_code *code, int32_t *n_classes, int32_t *degrees);

/* Workspace bytes of a forward/backward pair for n_frames frames, T
 * iterations and checkpoints every ckpt iterations (posteriors and messages
 * of iterations ckpt, 2 ckpt, ... are kept; the adjoint recomputes the rest). */
ldpc_status ldpc_learn_workspace_size(const ldpc_code *code, int32_t n_frames, int32_t T, int32_t ckpt,
                                      size_t *bytes);

/*
 * Forward pass.
 *  llr       device [F][N] float32 channel LLRs.
 *  target    device [F][N] uint8 transmitted bits, or NULL (all-zero word).
 *  weights   device [T][C][2] float32: (a, b) per iteration and class.
 *  loss      device [T] float32 out: loss_t (summed over frames and bits).
 *  post_out  device [F][N] float32 out: Z^(T), or NULL.
 * The workspace keeps the checkpoints for ldpc_learn_backward.
 * LDPC_EUNSUPPORTED: more than 8 classes, a row degree above 32, or a batch
 * whose frame-minor arrays exceed 2 GiB.
 */
ldpc_status ldpc_learn_forward(const ldpc_code *code, int32_t n_frames, const float *llr, const uint8_t *target,
                               int32_t T, const float *weights, int32_t ckpt, void *workspace,
                               size_t workspace_bytes, float *loss, float *post_out, void *stream);

/*
 * Adjoint of the summed loss with respect to the weights, after
 * ldpc_learn_forward with the same frames, target, T, weights, ckpt and
 * workspace.  grad: device [T][C][2] float32 out (overwritten).
 * Gradients are exact for the binary32 forward away from ties of |t| and
 * from a*m = b; their per-class sums are accumulated in an unspecified
 * order.
 */
ldpc_status ldpc_learn_backward(const ldpc_code *code, int32_t n_frames, const uint8_t *target, int32_t T,
                                const float *weights, int32_t ckpt, void *workspace, size_t workspace_bytes,
                                float *grad, void *stream);

/*
 * The same adjoint for the objective sum_t w_t loss_t: loss_weights is a
 * host array of T finite weights (read during the call), or NULL for all
 * ones (ldpc_learn_backward).  Weighting the early iterations more trains the
 * pairs towards decoding in fewer iterations (the paper indexes lambda and
 * beta by the iteration, Sec. III; the objective is this library's).
 * LDPC_EINVAL for a non-finite weight.
 */
ldpc_status ldpc_learn_backward_weighted(const ldpc_code *code, int32_t n_frames, const uint8_t *target,
                                         int32_t T, const float *weights, int32_t ckpt, void *workspace,
                                         size_t workspace_bytes, const float *loss_weights, float *grad,
                                         void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LDPC_LEARN_H */
