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
// y[k][j] = bf16(x[row k][j]), row k = rows[k] (or k when rows is NULL; rows outside [0, n_total)
// read row 0 and set STATUS_BAD_ROW).
hipError_t launch_gather_f32_to_bf16(const float *x, const int32_t *rows, int64_t n_total, int d, int64_t n, void *y,
                                     uint32_t *status, hipStream_t s);
// Per-block partial sums of the squared error of y [n / M][M] against the target rows (as in the
// gather), the BF16 gradient 2 (y - t) scale into dy (unless NULL) and, if loss_out is given,
// scale x the sum.  part holds MSE_BLOCKS doubles.
constexpr int MSE_BLOCKS = 256;
hipError_t launch_mse_grad(const float *y, const float *t, int64_t n, int M, const int32_t *rows, int64_t n_total,
                           double scale, void *dy, double *part, float *loss_out, uint32_t *status, hipStream_t s);
// out[0] = scale x the sum of part[0 .. nb) in an order fixed by nb.
hipError_t launch_sum_partials(const double *part, int64_t nb, double scale, double *out, hipStream_t s);
// out[r][j] = ln((h[r][j] + 1/2) / (N_r + nbins / 2)) for n rows of nbins counts.
hipError_t launch_log_hess_target(const uint32_t *h, int n, int nbins, float *out, hipStream_t s);
hipError_t launch_colsum(const void *dz, int n, int m, float *db, hipStream_t s);
hipError_t launch_adam_layer(const AdamArgs &a, hipStream_t s);
// lnfact64[k] = ln k! for k < nlf (lgamma beyond, or everywhere when lnfact64 is NULL)
hipError_t launch_surrogate_loglike(const float *y, int n, int nbins, const uint32_t *d, double *out,
                                   const double *lnfact64, int nlf, hipStream_t s);

}  // namespace pcmd
