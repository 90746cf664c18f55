/*
 * mlp_closure.h -- C ABI of the learned drag closure in liblbimb.so.
 *
 * A multilayer perceptron 40 -> 128 -> 128 -> 128 -> 1 with SiLU on the hidden
 * layers maps per-particle features (local solid fraction, particle Reynolds
 * number, slip velocity, neighbour histogram) to a normalised drag.  Matrix
 * products run on gfx950 matrix cores with bfloat16 operands and binary32
 * accumulation; binary32 master weights are trained with Adam on the mean
 * squared error.  Resolved LB-IMB drag (lbimb.h) is the training data and the
 * judge; callers fall back to it outside the training envelope.
 *
 * Parameter vector (binary32, MLP_NPARAMS = 38401 values), in this order:
 *   W1[128][40], b1[128], W2[128][128], b2[128], W3[128][128], b3[128],
 *   W4[1][128], b4[1]         (row-major, output index first).
 *
 * Conventions: return 0 or a negative LBM_E_* code from lbimb.h; X, y and
 * outputs are device pointers on the context's GPU unless ptr_kind says
 * LBM_HOST; calls are ordered on the context's stream.  The caller owns the
 * workspace and all buffers.
 */
#ifndef MLP_CLOSURE_H
#define MLP_CLOSURE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLP_NIN 40
#define MLP_NHID 128
#define MLP_NPARAMS 38401

typedef struct mlp_ctx mlp_ctx;

/* Device bytes for a context that trains on minibatches of up to
 * `max_batch` rows (inference takes any number of rows). */
int mlp_workspace_bytes(int64_t max_batch, size_t *bytes);

int mlp_create(int64_t max_batch, void *workspace, size_t ws_bytes, void *hip_stream,
               mlp_ctx **out);
void mlp_destroy(mlp_ctx *ctx);

/* Set / get the binary32 master parameters (layout above).  Setting also
 * resets the Adam moments and step count. */
int mlp_set_params(mlp_ctx *ctx, const float *params, int ptr_kind);
int mlp_get_params(mlp_ctx *ctx, float *params, int ptr_kind);

/* Inference: y[n] = MLP(X[n][40]) with the current parameters (device
 * pointers, asynchronous on the context's stream). */
int mlp_forward(mlp_ctx *ctx, const float *X, int64_t n, float *y);

/* Input normalisation and training envelope for mlp_infer, 40 binary32 values
 * each: a raw input x_k enters the network as (x_k - mu[k]) / sd[k]; a row is
 * outside the envelope when some x_k < lo[k], x_k > hi[k] or is NaN.  Host or
 * device pointers per ptr_kind.  Errors: LBM_E_INVALID (null pointer; for
 * host input also sd[k] <= 0 or a non-finite mu or sd), LBM_E_HIP. */
int mlp_set_normaliser(mlp_ctx *ctx, const float *mu, const float *sd, const float *lo,
                       const float *hi, int ptr_kind);

/* Inference on raw inputs with the fallback flag: y[n] = MLP((X - mu) / sd)
 * with the current parameters, and out_of_envelope[n] (may be NULL) = 1 for
 * the rows outside the training envelope, where the caller uses the resolved
 * LB-IMB drag instead.  Device pointers, asynchronous on the context's stream.
 * Errors: LBM_E_INVALID, LBM_E_STATE (no mlp_set_normaliser yet), LBM_E_HIP. */
int mlp_infer(mlp_ctx *ctx, const float *X, int64_t n, float *y, uint8_t *out_of_envelope);

/* Gradient of the mean squared error (1/n) sum (MLP(X) - y)^2 with respect to
 * every parameter, without updating them; grads[MLP_NPARAMS] and *loss are
 * written (device pointers for X, y; grads and loss follow ptr_kind). */
int mlp_gradients(mlp_ctx *ctx, const float *X, const float *y, int64_t n, float *grads,
                  float *loss, int ptr_kind);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * minibatch X[n][40], y[n], n <= max_batch.  *loss (host) receives the
 * minibatch loss before the update when loss is not NULL. */
int mlp_train_step(mlp_ctx *ctx, const float *X, const float *y, int64_t n, float lr,
                   float *loss);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc): the
 * gradient and loss of mlp_gradients for the binary32 parameters `params`
 * (layout above), with no context and no workspace.  The intermediates live in
 * one fixed array of MLP_NOALLOC_SCRATCH_BYTES in device memory per GPU,
 * which the library holds until the process ends; the call allocates nothing.
 * params [MLP_NPARAMS], X [n][40], y [n] and grads [MLP_NPARAMS] are device
 * pointers on the current GPU; loss is a device pointer or NULL.  The work is
 * queued on hip_stream (NULL: the null stream) and the call returns without
 * waiting.  Results equal those of mlp_gradients on a context holding the same
 * parameters, bit for bit.  Calls that overlap on one GPU (on different
 * streams, or from different threads) share the array and race; order them.
 * Errors: LBM_E_INVALID for a null pointer or n outside
 * 1..MLP_NOALLOC_MAX_ROWS; LBM_E_HIP for a failed launch or symbol lookup. */
#define MLP_NOALLOC_MAX_ROWS 4096
#define MLP_NOALLOC_SCRATCH_BYTES 15380736
int mlp_gradients_noalloc(const float *params, const float *X, const float *y, int64_t n,
                          float *grads, float *loss, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MLP_CLOSURE_H */
