/*
 * sscs_mlp.h -- C ABI of the small multilayer perceptron that predicts warm
 * starts for a parametric family of cone programs (part of libsscs).
 *
 * Any starting point u0 is admissible for the iteration of Sec. IV-A
 * (equation (drs) converges from every u0) and u0 is an input of Algorithm 1.
 * The network maps a problem parameter vector to a predicted primal-dual
 * triple (x, y, s); the caller forms u0 = (x, y + s, 1), the DRS state whose
 * resolvent and projection reproduce (x, y, s) at a fixed point (Sec. III-A,
 * u = (chi, psi, tau) and v = (0, s, kappa)).
 *
 * Network: widths w0 -> w1 -> ... -> wL, ReLU after every layer but the last.
 * Arithmetic: BF16 operands on the matrix cores (v_mfma_f32_16x16x32_bf16),
 * FP32 accumulation, FP32 master weights, Adam on the mean squared error.
 *
 * Conventions
 *   - W_l is w_{l+1} x w_l row-major FP32, b_l has w_{l+1} entries.
 *   - Activations X (batch x w0), targets T and outputs Y (batch x wL) are
 *     row-major FP32 DEVICE pointers; parameter arrays of set/get and the
 *     gradient outputs of sscs_mlp_gradients are HOST pointers.
 *   - All work is enqueued on the stream given at create; every call returns
 *     after the stream has finished it.  Return codes are those of sscs.h.
 */
#ifndef SSCS_MLP_H
#define SSCS_MLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sscs_mlp sscs_mlp;

/* widths has nlayers + 1 entries (each >= 1); max_batch bounds every batch.
 * Weights and biases of layer l are initialised uniform in +-1/sqrt(w_l) from a
 * counter-based hash (splitmix64) of (seed, stream, index). */
int sscs_mlp_create(int32_t nlayers, const int32_t *widths, int32_t max_batch, uint64_t seed,
                    void *hip_stream, sscs_mlp **out);
int sscs_mlp_destroy(sscs_mlp *net);

/* Copies all weights and biases in (host FP32 arrays, one per layer). */
int sscs_mlp_set_params(sscs_mlp *net, const float *const *W, const float *const *b);
int sscs_mlp_get_params(sscs_mlp *net, float *const *W, float *const *b);

/* Y = net(X). */
int sscs_mlp_forward(sscs_mlp *net, int32_t batch, const float *X, float *Y);

/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on
 * L = mean((net(X) - T)^2); *loss gets L before the step (may be NULL). */
int sscs_mlp_train_step(sscs_mlp *net, int32_t batch, const float *X, const float *T, float lr, float *loss);

/* Gradients of L at the current parameters without updating them
 * (host outputs dW[l], db[l]); *loss gets L. */
int sscs_mlp_gradients(sscs_mlp *net, int32_t batch, const float *X, const float *T, float *const *dW,
                       float *const *db, float *loss);

/* C (M x N, FP32, row-major) = A (M x K) * B (N x K)^T, A and B given as FP32
 * device arrays and rounded to BF16 before the product -- the matrix-core
 * kernel the network uses, exposed for tests and measurement. */
int sscs_mlp_gemm_nt(int32_t M, int32_t N, int32_t K, const float *A, const float *B, float *C, void *hip_stream);

/* Warm starts from predictions: pred is count x (n + 2m) FP32 (device), each
 * row (x, y, s); u0 is count x (n + m + 1) FP64 (device), each row
 * (x, y + s, 1) -- the DRS state of Sec. IV-A whose fixed point carries the
 * primal-dual triple (x, y, s) with tau = 1 (Sec. III-A). */
int sscs_assemble_u0(int32_t count, int32_t n, int32_t m, const float *pred, double *u0, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SSCS_MLP_H */
