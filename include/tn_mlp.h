/*
 * tn_mlp.h -- learned pruning of level-2/3 terms: per-term features, a small
 * fully connected network trained on the GPU by the library's own forward,
 * backward and Adam kernels, and the pruning threshold.
 *
 * The method itself (Section IV, Algorithm 1) keeps every term up to level l;
 * this is an optional policy on top of it.  It predicts log X of each
 * candidate term and drops those below a threshold chosen on training terms
 * for a pruned-mass budget.  The full expansion remains the reference for the
 * error of a pruned estimate (tn_prune_opts in tn.h applies the keep flags).
 *
 * Device buffers are caller-owned.  State layout (float32):
 *   [ mean[n_in] | inv_std[n_in] | params P | grads P | adam m P | adam v P ]
 * params: per layer, W (out x in, row-major) then b (out); layers
 *   n_in -> width (ReLU) -> ... (depth hidden layers) -> 1 (linear).
 * Every call is asynchronous on `stream` unless stated.  Errors as in tn.h.
 */
#ifndef TN_MLP_H
#define TN_MLP_H
#include <stddef.h>
#include <stdint.h>
#include "tn.h"
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_in;    /* features per sample */
    int32_t width;   /* hidden width */
    int32_t depth;   /* hidden layers (>= 1) */
} tn_mlp_shape;

/* Parameter count, state bytes, and workspace bytes for batches up to `batch`.
 * Host only. */
int tn_mlp_sizes(const tn_mlp_shape* s, int64_t batch, int64_t* n_params, size_t* state_bytes,
                 size_t* ws_bytes);

/* He-initialised weights (seeded), zero biases, grads and Adam moments,
 * identity normalizer.  Synchronizes `stream`. */
int tn_mlp_init(const tn_mlp_shape* s, uint64_t seed, void* d_state, void* stream);

/* Set the input normalizer to the column mean and 1/std of d_x (n x n_in). */
int tn_mlp_fit_normalizer(const tn_mlp_shape* s, void* d_state, const float* d_x, int64_t n,
                          void* stream);

/* d_y[n] = network(d_x[n x n_in]). */
int tn_mlp_forward(const tn_mlp_shape* s, const void* d_state, const float* d_x, int64_t n,
                   float* d_y, void* d_ws, void* stream);

/* Loss (1/n) sum_r w_r (y_r - t_r)^2 into *d_loss (device float) and its
 * gradient into the grads region of the state.  d_w may be NULL (w = 1). */
int tn_mlp_gradients(const tn_mlp_shape* s, void* d_state, const float* d_x, const float* d_t,
                     const float* d_w, int64_t n, void* d_ws, float* d_loss, void* stream);

/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8) with step number >= 1. */
int tn_mlp_adam(const tn_mlp_shape* s, void* d_state, float lr, int32_t step, void* stream);

/* tn_mlp_gradients followed by tn_mlp_adam. */
int tn_mlp_train_step(const tn_mlp_shape* s, void* d_state, const float* d_x, const float* d_t,
                      const float* d_w, int64_t n, float lr, int32_t step, void* d_ws,
                      float* d_loss, void* stream);

/* The pruner's training and persistence exports.
 * tn_pruner_train_step: tn_mlp_train_step under the pruner's name.
 * tn_pruner_save: the model (normalizer and parameters, not gradients or Adam
 *   moments) into host memory h_buf: a TN_PRUNER_HEADER_BYTES header (the
 *   bytes "TNPRUNE1", then n_in, width, depth as int32 and the parameter count
 *   as int64, zero padded) followed by (2 n_in + P) float32.  *need_bytes
 *   receives the size; h_buf = NULL only queries it; a smaller buffer is
 *   TN_ENOMEM.  Synchronizes `stream`.
 * tn_pruner_load: the reverse into d_state (gradients and moments zeroed);
 *   TN_EINVAL if the header is not a saved model or its shape differs from
 *   `s`.  Synchronizes `stream`. */
#define TN_PRUNER_HEADER_BYTES 32
int tn_pruner_train_step(const tn_mlp_shape* s, void* d_state, const float* d_x, const float* d_t,
                         const float* d_w, int64_t n, float lr, int32_t step, void* d_ws, float* d_loss,
                         void* stream);
int tn_pruner_save(const tn_mlp_shape* s, const void* d_state, void* h_buf, size_t buf_bytes,
                   size_t* need_bytes, void* stream);
int tn_pruner_load(const tn_mlp_shape* s, void* d_state, const void* h_buf, size_t buf_bytes, void* stream);

/* Features of every term of a term set (n_terms x TN_N_FEATURES floats, host
 * memory): for up to three corrected noises in position order, presence,
 * log(d_i/d_0), correction one-hot, position in the circuit, past-light-cone
 * size, 2-qubit gates in that cone, and the log value of the level-1 term with
 * the same (noise, correction) taken from level1_x (X of a level >= 1 term set
 * of the same plan in enumeration order; NULL = 0); for each pair of them,
 * cone overlap and distance in the circuit; then log of the term weight, the
 * level, and (index 35) log of the term's rigorous bound
 * w prod_s ||sqrt(2) K_{c_s}||_2^2 -- the score of the policy without the
 * network.  Host only. */
#define TN_N_FEATURES 36

/* t[i] = log(max(x[i], floor)) as float (training targets), on the device. */
int tn_mlp_log_targets(const double* d_x, float* d_t, int64_t n, double floor, void* stream);
int tn_terms_features(tn_plan plan, tn_terms terms, const double* level1_x, float* out);

/* Pruning threshold: given predicted log values pred[n] and the true values
 * x[n] (x >= 0) of training candidates, the largest tau such that the
 * candidates with pred < tau hold at most `budget` (absolute) of sum x.  Host. */
int tn_prune_threshold(const float* pred, const double* x, int64_t n, double budget, float* tau);

#ifdef __cplusplus
}
#endif
#endif
