// Message-passing network on the variable-constraint graph: gfx950 kernels for
// the forward pass, the backward pass and the optimiser of the learned restart
// initialiser.  Dense products use bf16 MFMA (v_mfma_f32_16x16x32_bf16) with
// float32 accumulation: weight matrices are stored in bf16; float32
// activations (and output gradients) enter as two bf16 operands, the value
// rounded to bf16 and the rounded remainder, whose sum holds 16 significant
// bits, so a product with a bf16 weight is exact to about 2^-16 relative.
// Sparse message passing is a CSR gather (one wave per row, one lane per
// hidden unit).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/pcls_mpnn.h"

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const char* what) {
  g_err = what;
  return code;
}

int32_t hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return 0;
  (void)hipGetLastError();  // clear the sticky error
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return 5;
}

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

union Pack8 {
  bf16x8 v;
  uint16_t u[8];
};

// ------------------------------------------------------------------ GEMM
// Y[N x M] = beta * Y + A[N x K] op(W) + bias, optionally ReLU'd into Yr;
// A = A_hi + A_lo in bf16 (two MFMA products per k step), W in bf16.
// op(W) = W^T for W stored [M][K] (trans_w = 0), W for W stored [K][M] (1).
// K a multiple of 32 up to 128; M a multiple of 16 up to 128; A row stride lda.
// Block: 4 waves, 64 rows; op(W) is staged in LDS as Bt[col][k].
constexpr int kMaxM = 128, kMaxK = 128;

__global__ void __launch_bounds__(256) gemm_kernel(const float* __restrict__ A, int lda, int N, int K,
                                                   const uint16_t* __restrict__ W, int M, int trans_w,
                                                   const float* __restrict__ bias, float* __restrict__ Y, int ldy,
                                                   int beta, float* __restrict__ Yr) {
  __shared__ uint16_t Bt[kMaxM][kMaxK + 8];  // Bt[col][k] = op(W)[k][col]
  for (int i = threadIdx.x; i < M * K; i += blockDim.x) {
    int col, k;
    if (trans_w == 0) {
      col = i / K;
      k = i % K;
    } else {
      k = i / M;
      col = i % M;
    }
    Bt[col][k] = W[i];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = blockIdx.x * 64 + wave * 16;
  const int r = i0 + (lane & 15);
  const int kq = (lane >> 4) * 8;  // this lane's 8 k-values within a 32-wide k step
  for (int j0 = 0; j0 < M; j0 += 16) {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
      Pack8 a, al, b;
      if (r < N) {
        const float* ap = A + (size_t)r * lda + k0 + kq;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float v = ap[e];
          a.u[e] = f2bf(v);
          al.u[e] = f2bf(v - bf2f(a.u[e]));
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) a.u[e] = al.u[e] = 0;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) b.u[e] = Bt[j0 + (lane & 15)][k0 + kq + e];
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al.v, b.v, acc, 0, 0, 0);
    }
    // lane holds C[4 * (lane / 16) + e][lane % 16]
    const int col = j0 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = i0 + (lane >> 4) * 4 + e;
      if (row < N) {
        float v = acc[e] + (bias ? bias[col] : 0.f);
        float* yp = Y + (size_t)row * ldy + col;
        if (beta) v += *yp;
        *yp = v;
        if (Yr) Yr[(size_t)row * ldy + col] = v > 0.f ? v : 0.f;
      }
    }
  }
}

// dW[M x K] (+)= sum_n dZ[n][m] X[n][k]: one wave per 16x16 output tile and
// chunk of rows; chunk partials are summed in a second pass (deterministic).
// Both operands are split into bf16 high and low parts (x = hi + lo) and the
// three significant cross products are accumulated: a weight gradient is a
// long sum over rows that may cancel, so it gets about 16 bits of operand
// precision instead of 8.
__global__ void __launch_bounds__(64) gemm_tn_kernel(const float* __restrict__ dZ, int ldz,
                                                     const float* __restrict__ X, int ldx, int N, int M, int K,
                                                     int rows_per_chunk, float* __restrict__ partial) {
  const int tiles_k = K / 16;
  const int tm = blockIdx.x / tiles_k, tk = blockIdx.x % tiles_k;
  const int chunk = blockIdx.y;
  const int lane = threadIdx.x;
  const int m = tm * 16 + (lane & 15), k = tk * 16 + (lane & 15);
  const int nq = (lane >> 4) * 8;
  const int n_begin = chunk * rows_per_chunk, n_end = min(N, n_begin + rows_per_chunk);
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int n0 = n_begin; n0 < n_end; n0 += 32) {
    Pack8 ah, al, bh, bl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int n = n0 + nq + e;
      const float za = n < n_end ? dZ[(size_t)n * ldz + m] : 0.f;
      const float xb = n < n_end ? X[(size_t)n * ldx + k] : 0.f;
      ah.u[e] = f2bf(za);
      al.u[e] = f2bf(za - bf2f(ah.u[e]));
      bh.u[e] = f2bf(xb);
      bl.u[e] = f2bf(xb - bf2f(bh.u[e]));
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah.v, bh.v, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah.v, bl.v, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al.v, bh.v, acc, 0, 0, 0);
  }
  float* out = partial + (size_t)chunk * M * K;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int mm = tm * 16 + (lane >> 4) * 4 + e;
    out[(size_t)mm * K + tk * 16 + (lane & 15)] = acc[e];
  }
}

__global__ void sum_chunks_kernel(const float* __restrict__ partial, int chunks, int count, float* __restrict__ out,
                                  int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += partial[(size_t)c * count + i];
  out[i] = accumulate ? out[i] + s : s;
}

// ---------------------------------------------------------------- gathers
// Forward message (mode 0): Z[row][d] += sum_j w_j * In[idx_j][d + (neg_j ? H : 0)],
//   then Hr[row][d] = max(Z, 0) if Hr != NULL.
// Transposed message (mode 1): Out[row][d + (neg_j ? H : 0)] = sum_j w_j * In[idx_j][d].
// idx entries are (index << 1) | neg.  One wave per row; H == 64.
__global__ void __launch_bounds__(256) gather_kernel(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                                     const float* __restrict__ w, int rows, const float* __restrict__ In,
                                                     int ld_in, float* __restrict__ Out, int ld_out,
                                                     float* __restrict__ Hr, int mode) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int d = threadIdx.x & 63;
  if (row >= rows) return;
  const int b = ptr[row], e = ptr[row + 1];
  float acc_p = 0.f, acc_n = 0.f;
  for (int j = b; j < e; ++j) {
    const int code = idx[j];
    const int src = code >> 1;
    const bool neg = code & 1;
    const float wj = w[j];
    if (mode == 0) {
      acc_p = fmaf(wj, In[(size_t)src * ld_in + d + (neg ? 64 : 0)], acc_p);
    } else {
      const float v = wj * In[(size_t)src * ld_in + d];
      if (neg)
        acc_n += v;
      else
        acc_p += v;
    }
  }
  if (mode == 0) {
    const float z = Out[(size_t)row * ld_out + d] + acc_p;
    Out[(size_t)row * ld_out + d] = z;
    if (Hr) Hr[(size_t)row * ld_out + d] = z > 0.f ? z : 0.f;
  } else {
    Out[(size_t)row * ld_out + d] = acc_p;
    Out[(size_t)row * ld_out + d + 64] = acc_n;
  }
}

// dZ = dH * [Z > 0]
__global__ void relu_grad_kernel(const float* __restrict__ dH, const float* __restrict__ Z, float* __restrict__ dZ,
                                 int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dZ[i] = Z[i] > 0.f ? dH[i] : 0.f;
}

// column sums of X[N x 64] into partial[blocks][64]
__global__ void __launch_bounds__(256) colsum_kernel(const float* __restrict__ X, int ld, int N, int rows_per_block,
                                                     float* __restrict__ partial) {
  __shared__ float red[4][64];
  const int d = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int n0 = blockIdx.x * rows_per_block, n1 = min(N, n0 + rows_per_block);
  float s = 0.f;
  for (int n = n0 + q; n < n1; n += 4) s += X[(size_t)n * ld + d];
  red[q][d] = s;
  __syncthreads();
  if (q == 0) partial[(size_t)blockIdx.x * 64 + d] = red[0][d] + red[1][d] + red[2][d] + red[3][d];
}

// ------------------------------------------------------------------ head
// xhat[v] = tanh(H[v] . w + b); one wave per row
__global__ void __launch_bounds__(256) head_forward_kernel(const float* __restrict__ H, int N,
                                                           const float* __restrict__ w, const float* __restrict__ b,
                                                           float* __restrict__ xhat) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int d = threadIdx.x & 63;
  if (row >= N) return;
  float s = H[(size_t)row * 64 + d] * w[d];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (d == 0) xhat[row] = tanhf(s + b[0]);
}

// head weight gradient partials: dw[d] = sum_v dlogit[v] H[v][d], db = sum_v dlogit[v]
__global__ void __launch_bounds__(256) head_grad_kernel(const float* __restrict__ H, const float* __restrict__ dlogit,
                                                        int N, int rows_per_block, float* __restrict__ partial) {
  __shared__ float red[4][65];
  const int d = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int n0 = blockIdx.x * rows_per_block, n1 = min(N, n0 + rows_per_block);
  float s = 0.f, sb = 0.f;
  for (int n = n0 + q; n < n1; n += 4) {
    const float g = dlogit[n];
    s = fmaf(g, H[(size_t)n * 64 + d], s);
    sb += g;
  }
  red[q][d] = s;
  if (d == 0) red[q][64] = sb;
  __syncthreads();
  if (q == 0) {
    float* out = partial + (size_t)blockIdx.x * 65;
    out[d] = red[0][d] + red[1][d] + red[2][d] + red[3][d];
    if (d == 0) out[64] = red[0][64] + red[1][64] + red[2][64] + red[3][64];
  }
}

// restart proposal: X[v][r] = clip(gamma * xhat[v] + sigma * U[v][r], -1, 1)
// for r < R (U uniform in [-1, 1), e.g. from pcls_init_restarts); padding untouched
__global__ void propose_kernel(const float* __restrict__ xhat, int n, const float* __restrict__ U, int R, int ldx,
                               float gamma, float sigma, float* __restrict__ X) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (r >= R || v >= n) return;
  const float x = fmaf(gamma, xhat[v], sigma * U[(size_t)v * ldx + r]);
  X[(size_t)v * ldx + r] = fminf(1.f, fmaxf(-1.f, x));
}

// dlogit = dxhat (1 - xhat^2); dH[v][d] = dlogit w[d]; dlogit written for the
// weight gradient (dw = H^T dlogit, db = sum dlogit)
__global__ void head_backward_kernel(const float* __restrict__ xhat, const float* __restrict__ dxhat, int N,
                                     const float* __restrict__ w, float* __restrict__ dH,
                                     float* __restrict__ dlogit) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * 64) return;
  const int row = i >> 6, d = i & 63;
  const float x = xhat[row];
  const float g = dxhat[row] * (1.f - x * x);
  dH[i] = g * w[d];
  if (d == 0) dlogit[row] = g;
}

// loss = mean (xhat - y)^2 over rows with mask != 0; dxhat = 2 (xhat - y) / count
__global__ void mse_kernel(const float* __restrict__ xhat, const float* __restrict__ y, int N, float inv_count,
                           float* __restrict__ dxhat, float* __restrict__ loss_partial) {
  __shared__ float red[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < N) {
    const float e = xhat[i] - y[i];
    dxhat[i] = 2.f * e * inv_count;
    l = e * e * inv_count;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_partial[blockIdx.x] = red[0];
}

// Adam with float32 master weights; writes the bf16 copy used by the GEMMs
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int count, float lr, float b1, float b2, float eps, float c1,
                            float c2, float wd, uint16_t* __restrict__ p_bf16) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i] + wd * p[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  if (p_bf16) p_bf16[i] = f2bf(pi);
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = f2bf(x[i]);
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

const char* pcls_mpnn_last_error(void) { return g_err.c_str(); }

int32_t pcls_mpnn_gemm(const float* A, int32_t lda, int32_t N, int32_t K, const uint16_t* W, int32_t M,
                       int32_t trans_w, const float* bias, float* Y, int32_t ldy, int32_t beta, float* Y_relu,
                       void* stream) {
  if (!A || !W || !Y || N < 0) return fail(1, "gemm: NULL pointer or N < 0");
  if (K < 32 || K > kMaxK || K % 32 || M < 16 || M > kMaxM || M % 16 || ldy < M || lda < K)
    return fail(1, "gemm: K a multiple of 32 in [32, 128], M a multiple of 16 in [16, 128], ldy >= M, lda >= K");
  if (N == 0) return 0;
  hipLaunchKernelGGL(gemm_kernel, dim3((N + 63) / 64), dim3(256), 0, (hipStream_t)stream, A, lda, N, K, W, M,
                     trans_w, bias, Y, ldy, beta, Y_relu);
  return hip_check(hipGetLastError(), "gemm launch");
}

size_t pcls_mpnn_gemm_tn_scratch(int32_t N, int32_t M, int32_t K) {
  const int chunks = (N + 1023) / 1024;
  return (size_t)(chunks > 0 ? chunks : 1) * M * K * sizeof(float);
}

int32_t pcls_mpnn_gemm_tn(const float* dZ, int32_t ldz, const float* X, int32_t ldx, int32_t N, int32_t M, int32_t K,
                          float* dW, int32_t accumulate, float* scratch, size_t scratch_bytes, void* stream) {
  if (!dZ || !X || !dW || !scratch || N < 0) return fail(1, "gemm_tn: NULL pointer or N < 0");
  if (M % 16 || K % 16 || M < 16 || K < 16 || ldz < M || ldx < K) return fail(1, "gemm_tn: bad shape");
  if (scratch_bytes < pcls_mpnn_gemm_tn_scratch(N, M, K)) return fail(4, "gemm_tn: scratch too small");
  const int chunks = N > 0 ? (N + 1023) / 1024 : 1;
  hipStream_t s = (hipStream_t)stream;
  if (N > 0) {
    hipLaunchKernelGGL(gemm_tn_kernel, dim3((M / 16) * (K / 16), chunks), dim3(64), 0, s, dZ, ldz, X, ldx, N, M, K,
                       1024, scratch);
    int32_t st = hip_check(hipGetLastError(), "gemm_tn launch");
    if (st) return st;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3((M * K + 255) / 256), dim3(256), 0, s, scratch, chunks, M * K, dW,
                       accumulate);
  } else if (!accumulate) {
    hipLaunchKernelGGL(sum_chunks_kernel, dim3((M * K + 255) / 256), dim3(256), 0, s, scratch, 0, M * K, dW, 0);
  }
  return hip_check(hipGetLastError(), "sum_chunks launch");
}

int32_t pcls_mpnn_gather(const int32_t* ptr, const int32_t* idx, const float* w, int32_t rows, const float* In,
                         int32_t ld_in, float* Out, int32_t ld_out, float* H_relu, int32_t mode, void* stream) {
  if (!ptr || !In || !Out || rows < 0 || (mode != 0 && mode != 1)) return fail(1, "gather: bad argument");
  if (mode == 0 && ld_in < 128) return fail(1, "gather: forward input must hold both sign halves (ld_in >= 128)");
  if (mode == 1 && ld_out < 128) return fail(1, "gather: transposed output needs ld_out >= 128");
  if (rows == 0) return 0;
  hipLaunchKernelGGL(gather_kernel, dim3((rows + 3) / 4), dim3(256), 0, (hipStream_t)stream, ptr, idx, w, rows, In,
                     ld_in, Out, ld_out, H_relu, mode);
  return hip_check(hipGetLastError(), "gather launch");
}

int32_t pcls_mpnn_relu_grad(const float* dH, const float* Z, float* dZ, int32_t count, void* stream) {
  if (!dH || !Z || !dZ || count < 0) return fail(1, "relu_grad: bad argument");
  if (count == 0) return 0;
  hipLaunchKernelGGL(relu_grad_kernel, dim3((count + 255) / 256), dim3(256), 0, (hipStream_t)stream, dH, Z, dZ,
                     count);
  return hip_check(hipGetLastError(), "relu_grad launch");
}

size_t pcls_mpnn_colsum_scratch(int32_t N) { return (size_t)((N + 1023) / 1024 + 1) * 64 * sizeof(float); }

int32_t pcls_mpnn_colsum(const float* X, int32_t ld, int32_t N, float* out64, int32_t accumulate, float* scratch,
                         size_t scratch_bytes, void* stream) {
  if (!X || !out64 || !scratch || N < 0 || ld < 64) return fail(1, "colsum: bad argument");
  if (scratch_bytes < pcls_mpnn_colsum_scratch(N)) return fail(4, "colsum: scratch too small");
  const int blocks = N > 0 ? (N + 1023) / 1024 : 0;
  hipStream_t s = (hipStream_t)stream;
  if (blocks > 0) {
    hipLaunchKernelGGL(colsum_kernel, dim3(blocks), dim3(256), 0, s, X, ld, N, 1024, scratch);
    int32_t st = hip_check(hipGetLastError(), "colsum launch");
    if (st) return st;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(1), dim3(64), 0, s, scratch, blocks, 64, out64, accumulate);
  }
  return hip_check(hipGetLastError(), "colsum reduce launch");
}

int32_t pcls_mpnn_head_forward(const float* H, int32_t N, const float* w, const float* b, float* xhat, void* stream) {
  if (!H || !w || !b || !xhat || N < 0) return fail(1, "head_forward: bad argument");
  if (N == 0) return 0;
  hipLaunchKernelGGL(head_forward_kernel, dim3((N + 3) / 4), dim3(256), 0, (hipStream_t)stream, H, N, w, b, xhat);
  return hip_check(hipGetLastError(), "head_forward launch");
}

int32_t pcls_mpnn_head_backward(const float* xhat, const float* dxhat, int32_t N, const float* w, float* dH,
                                float* dlogit, void* stream) {
  if (!xhat || !dxhat || !w || !dH || !dlogit || N < 0) return fail(1, "head_backward: bad argument");
  if (N == 0) return 0;
  hipLaunchKernelGGL(head_backward_kernel, dim3((N * 64 + 255) / 256), dim3(256), 0, (hipStream_t)stream, xhat,
                     dxhat, N, w, dH, dlogit);
  return hip_check(hipGetLastError(), "head_backward launch");
}

size_t pcls_mpnn_head_grad_scratch(int32_t N) { return (size_t)((N + 1023) / 1024 + 1) * 65 * sizeof(float); }

int32_t pcls_mpnn_head_grad(const float* H, const float* dlogit, int32_t N, float* dwb65, int32_t accumulate,
                            float* scratch, size_t scratch_bytes, void* stream) {
  if (!H || !dlogit || !dwb65 || !scratch || N < 0) return fail(1, "head_grad: bad argument");
  if (scratch_bytes < pcls_mpnn_head_grad_scratch(N)) return fail(4, "head_grad: scratch too small");
  const int blocks = N > 0 ? (N + 1023) / 1024 : 0;
  hipStream_t s = (hipStream_t)stream;
  if (blocks > 0) {
    hipLaunchKernelGGL(head_grad_kernel, dim3(blocks), dim3(256), 0, s, H, dlogit, N, 1024, scratch);
    int32_t st = hip_check(hipGetLastError(), "head_grad launch");
    if (st) return st;
  }
  hipLaunchKernelGGL(sum_chunks_kernel, dim3(1), dim3(128), 0, s, scratch, blocks, 65, dwb65, accumulate);
  return hip_check(hipGetLastError(), "head_grad reduce launch");
}

int32_t pcls_mpnn_propose(const float* xhat, int32_t n, const float* U, int32_t R, float gamma, float sigma, float* X,
                          void* stream) {
  if (!xhat || !U || !X || n < 0 || R < 0) return fail(1, "propose: bad argument");
  if (n == 0 || R == 0) return 0;
  const int ldx = (R + 63) / 64 * 64;
  hipLaunchKernelGGL(propose_kernel, dim3((R + 63) / 64, n), dim3(64), 0, (hipStream_t)stream, xhat, n, U, R, ldx,
                     gamma, sigma, X);
  return hip_check(hipGetLastError(), "propose launch");
}

size_t pcls_mpnn_mse_scratch(int32_t N) { return (size_t)((N + 255) / 256 + 1) * sizeof(float); }

int32_t pcls_mpnn_mse(const float* xhat, const float* y, int32_t N, float* dxhat, float* loss_partial, void* stream) {
  if (!xhat || !y || !dxhat || !loss_partial || N < 1) return fail(1, "mse: bad argument");
  hipLaunchKernelGGL(mse_kernel, dim3((N + 255) / 256), dim3(256), 0, (hipStream_t)stream, xhat, y, N, 1.f / N, dxhat,
                     loss_partial);
  return hip_check(hipGetLastError(), "mse launch");
}

int32_t pcls_mpnn_adam(float* p, const float* g, float* m, float* v, int32_t count, float lr, float b1, float b2,
                       float eps, int32_t step, float weight_decay, uint16_t* p_bf16, void* stream) {
  if (!p || !g || !m || !v || count < 0 || step < 1) return fail(1, "adam: bad argument");
  if (count == 0) return 0;
  const float c1 = 1.f / (1.f - powf(b1, (float)step));
  const float c2 = 1.f / (1.f - powf(b2, (float)step));
  hipLaunchKernelGGL(adam_kernel, dim3((count + 255) / 256), dim3(256), 0, (hipStream_t)stream, p, g, m, v, count, lr,
                     b1, b2, eps, c1, c2, weight_decay, p_bf16);
  return hip_check(hipGetLastError(), "adam launch");
}

int32_t pcls_mpnn_to_bf16(const float* x, uint16_t* y, int32_t count, void* stream) {
  if (!x || !y || count < 0) return fail(1, "to_bf16: bad argument");
  if (count == 0) return 0;
  hipLaunchKernelGGL(to_bf16_kernel, dim3((count + 255) / 256), dim3(256), 0, (hipStream_t)stream, x, y, count);
  return hip_check(hipGetLastError(), "to_bf16 launch");
}

}  // extern "C"
