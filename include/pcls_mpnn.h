/*
 * pcls_mpnn - kernels of the learned restart initialiser (libpcls.so).
 *
 * A message-passing network on the bipartite variable-constraint graph of a
 * formula proposes a starting point x_hat in [-1,1]^n for the restarts of the
 * continuous local search (the paper's solver starts from given assignments:
 * Case Studies, "Costas Arrays", "starting assignments"; the network itself is
 * this library's addition, trained on assignments the plain search finds).
 *
 * Conventions: all pointers are device pointers, caller-owned; work is
 * asynchronous on the given HIP stream (void* hipStream_t, NULL = null stream);
 * hidden width is 64; activations are float32 row-major; weights used by the
 * matrix products are bf16 bit patterns (uint16) and products accumulate in
 * float32, each float32 operand rounded to bf16 (nearest even).
 * Status codes: 0 ok, 1 invalid argument, 4 scratch too small, 5 HIP error;
 * pcls_mpnn_last_error() describes the last failure on this thread.
 */
#ifndef PCLS_MPNN_H
#define PCLS_MPNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Y[N x M] = beta*Y + A[N x K] op(W) + bias (bias[M] or NULL); if Y_relu is not
 * NULL it also receives max(Y, 0).  op(W) = W^T for W stored [M][K]
 * (trans_w = 0) or W for W stored [K][M] (trans_w = 1).  K a multiple of 32 in
 * [32, 128]; M a multiple of 16 in [16, 128]; A has row stride lda >= K and Y
 * (and Y_relu) row stride ldy >= M. */
int32_t pcls_mpnn_gemm(const float* A, int32_t lda, int32_t N, int32_t K, const uint16_t* W, int32_t M,
                       int32_t trans_w, const float* bias, float* Y, int32_t ldy, int32_t beta, float* Y_relu,
                       void* hip_stream);

/* dW[M x K] = (accumulate ? dW : 0) + sum_n dZ[n][m] X[n][k] (row strides ldz, ldx);
 * M, K multiples of 16.  Operands are split into bf16 high and low parts and the
 * products hi*hi + hi*lo + lo*hi accumulated in float32 (about 16 bits of operand
 * precision).  scratch: device float buffer of pcls_mpnn_gemm_tn_scratch bytes
 * (per-chunk partial sums, reduced in a fixed order). */
size_t pcls_mpnn_gemm_tn_scratch(int32_t N, int32_t M, int32_t K);
int32_t pcls_mpnn_gemm_tn(const float* dZ, int32_t ldz, const float* X, int32_t ldx, int32_t N, int32_t M, int32_t K,
                          float* dW, int32_t accumulate, float* scratch, size_t scratch_bytes, void* hip_stream);

/* CSR gather over rows (ptr[rows+1], idx[] = (source << 1) | negated, w[] per entry):
 *  mode 0 (message): Out[r][d] += sum_j w_j In[src_j][d + 64*neg_j]  (In holds the
 *          positive- and negative-literal transforms side by side, ld_in >= 128);
 *          H_relu (or NULL) receives max(Out, 0).
 *  mode 1 (transposed message): Out[r][d + 64*neg] = sum over entries of that sign
 *          of w_j In[src_j][d]  (ld_out >= 128). */
int32_t pcls_mpnn_gather(const int32_t* ptr, const int32_t* idx, const float* w, int32_t rows, const float* In,
                         int32_t ld_in, float* Out, int32_t ld_out, float* H_relu, int32_t mode, void* hip_stream);

/* dZ = dH * [Z > 0], elementwise over count floats. */
int32_t pcls_mpnn_relu_grad(const float* dH, const float* Z, float* dZ, int32_t count, void* hip_stream);

/* out64[d] = (accumulate ? out64[d] : 0) + sum_n X[n][d], d < 64; scratch of
 * pcls_mpnn_colsum_scratch bytes. */
size_t pcls_mpnn_colsum_scratch(int32_t N);
int32_t pcls_mpnn_colsum(const float* X, int32_t ld, int32_t N, float* out64, int32_t accumulate, float* scratch,
                         size_t scratch_bytes, void* hip_stream);

/* Output head: xhat[v] = tanh(H[v] . w + b[0]) (H [N][64]). */
int32_t pcls_mpnn_head_forward(const float* H, int32_t N, const float* w, const float* b, float* xhat,
                               void* hip_stream);
/* dlogit = dxhat (1 - xhat^2); dH[v][d] = dlogit[v] w[d]. */
int32_t pcls_mpnn_head_backward(const float* xhat, const float* dxhat, int32_t N, const float* w, float* dH,
                                float* dlogit, void* hip_stream);

/* dwb65[0..63] (+)= sum_v dlogit[v] H[v][d] and dwb65[64] (+)= sum_v dlogit[v];
 * scratch of pcls_mpnn_head_grad_scratch bytes. */
size_t pcls_mpnn_head_grad_scratch(int32_t N);
int32_t pcls_mpnn_head_grad(const float* H, const float* dlogit, int32_t N, float* dwb65, int32_t accumulate,
                            float* scratch, size_t scratch_bytes, void* hip_stream);

/* Restart proposal X[v][r] = clip(gamma xhat[v] + sigma U[v][r], -1, 1) for r < R,
 * with U and X laid out [n][round_up(R, 64)] (U e.g. from pcls_init_restarts). */
int32_t pcls_mpnn_propose(const float* xhat, int32_t n, const float* U, int32_t R, float gamma, float sigma, float* X,
                          void* hip_stream);

/* Mean squared error over N rows: dxhat = 2 (xhat - y) / N; loss_partial[b] holds
 * block partial sums of (xhat - y)^2 / N (ceil(N/256) entries; scratch size
 * pcls_mpnn_mse_scratch). */
size_t pcls_mpnn_mse_scratch(int32_t N);
int32_t pcls_mpnn_mse(const float* xhat, const float* y, int32_t N, float* dxhat, float* loss_partial,
                      void* hip_stream);

/* Adam (Kingma and Ba) on float32 master weights p with moments m, v and step
 * number step >= 1 (bias correction); p_bf16 (or NULL) receives the rounded copy. */
int32_t pcls_mpnn_adam(float* p, const float* g, float* m, float* v, int32_t count, float lr, float b1, float b2,
                       float eps, int32_t step, float weight_decay, uint16_t* p_bf16, void* hip_stream);

/* y = bf16(x), nearest even. */
int32_t pcls_mpnn_to_bf16(const float* x, uint16_t* y, int32_t count, void* hip_stream);

const char* pcls_mpnn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PCLS_MPNN_H */
