// Internal interface of the surrogate-network kernels (k_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcmd {

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3 };

// C[M][N] = sum_k A(m, k) B(n, k) with the operand layouts of k_gemm and a fused epilogue.
struct GemmArgs {
  int M, N, K;
  const __bf16 *A;
  int lda;
  const __bf16 *B;
  int ldb;
  float *C;           // FP32 output (EPI_STORE, EPI_BIAS, EPI_BIAS_GELU)
  int ldc;
  __bf16 *Cb;         // BF16 output (EPI_BIAS_GELU: GELU(z); EPI_GELU_GRAD: dz_prev)
  int ldcb;
  const float *bias;  // [N]
  const float *Z;     // FP32 pre-activations for GELU' (EPI_GELU_GRAD)
  int ldz;
  float *part;        // split-K partial products [splits][M][N] (set by launch_gemm)
  int kchunk;         // K elements per split (a multiple of the K step)
};

struct AdamArgs {
  int n_out, n_in, update;
  float *master, *m, *v;
  const float *grad;
  void *w_bf16, *wt_bf16;
  float lr, beta1, beta2, eps, bc1, bc2;
};

// Workspace (bytes) launch_gemm needs for an M x N x K product: transposed copies of K-major
// operands (at: A(m, k) = A[k][m]; bt: B(n, k) = B[k][n]) and split-K partials.
size_t gemm_workspace_bytes(int M, int N, int K, bool at, bool bt);
hipError_t launch_gemm(const GemmArgs &g, bool at, bool bt, int epi, void *ws, size_t ws_bytes, hipStream_t s);
hipError_t launch_f32_to_bf16(const float *x, void *y, int64_t n, hipStream_t s);
hipError_t launch_mse_grad(const float *y, const float *t, int64_t n, double scale, void *dy, double *part,
                           float *loss_out, hipStream_t s);
hipError_t launch_colsum(const void *dz, int n, int m, float *db, hipStream_t s);
hipError_t launch_adam_layer(const AdamArgs &a, hipStream_t s);
// lnfact64[k] = ln k! for k < nlf (lgamma beyond, or everywhere when lnfact64 is NULL)
hipError_t launch_surrogate_loglike(const float *y, int n, int nbins, const uint32_t *d, double *out,
                                   const double *lnfact64, int nlf, hipStream_t s);

}  // namespace pcmd
