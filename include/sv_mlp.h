/*
 * libsv cost model: a two-hidden-layer ReLU MLP (FP32) that predicts the log
 * run time of one fused-gate sweep from its features, trained on the GPU by
 * these kernels on the library's own measured sweep times and used by the DP
 * planner of sv_plan.h.  (An addition to the paper, whose DP score is the
 * fixed gamma(k) = 4^k of Section IV-C.)
 *
 * Parameter vector (FP32, `sv_mlp_param_count(nin, hid)` entries, in order):
 *   W1[nin][hid], b1[hid], W2[hid][hid], b2[hid], W3[hid], b3[1]
 * y = W3 . relu(W2^T relu(W1^T x + b1) + b2) + b3.
 * Loss: 0.5 * mean over the batch of (y - t)^2.
 * All pointers are device pointers unless the name ends in _host; work is
 * enqueued on `stream`.  Reductions over the batch are done in a fixed order
 * (no atomics), so results are deterministic.
 */
#ifndef SV_MLP_H_
#define SV_MLP_H_

#include "sv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SV_MLP_FEATURES 12 /* N, k, 7 sorted physical target positions (padded), diagonal flag,
                              swept fraction and launches of a diagonal block (sv_plan.h) */
#define SV_MLP_HIDDEN 64

int sv_mlp_param_count(int nin, int hid);

/* Floats of activation cache sv_mlp_forward writes for a batch of B rows. */
int64_t sv_mlp_cache_floats(int hid, int batch);

/* y[B] = f(X[B][nin]); cache (may be NULL) keeps z1, z2 (pre-activations) for backward. */
int sv_mlp_forward(const float *params, int nin, int hid, const float *X, int batch, float *y, float *cache,
                   void *stream);

/* Loss into *loss (device float) and the full gradient into grads (param_count floats),
 * from the cache of the forward pass on the same X. */
int sv_mlp_backward(const float *params, int nin, int hid, const float *X, const float *target, int batch,
                    const float *y, const float *cache, float *grads, float *loss, void *stream);

/* One Adam step (Kingma and Ba) with bias correction at step t >= 1. */
int sv_mlp_adam(float *params, const float *grads, float *m, float *v, int count, int t, float lr, float beta1,
                float beta2, float eps, void *stream);

/* Host forward (FP64 arithmetic on FP32 parameters) for planning. */
int sv_mlp_forward_host(const float *params_host, int nin, int hid, const float *x_host, int batch,
                        double *y_host);

#ifdef __cplusplus
}
#endif
#endif /* SV_MLP_H_ */
