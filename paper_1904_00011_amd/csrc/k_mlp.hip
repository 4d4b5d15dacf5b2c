// Surrogate network kernels (gfx950): BF16 MFMA matrix products with FP32 accumulation and fused
// epilogues (bias, GELU, GELU derivative), MSE gradient, bias gradients, Adam with BF16 shadow
// weights, and the surrogate Poisson log-likelihood.
#include <math.h>

#include "pcmd_device.h"
#include "pcmd_internal.h"
#include "pcmd_mlp.h"

namespace pcmd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
}

// ---------------------------------------------------------------------------------------
// C[M][N] = sum_k A[m][k] B[n][k] on v_mfma_f32_32x32x16_bf16 (both operands K-contiguous).
// (64 MI) x 128 block tile, 4 waves of (32 MI) x 64 (MI x 2 MFMA tiles of 32 x 32): MI = 2 for
// most products, MI = 4 for large ones, where a wave's larger share of A halves the LDS reads per
// multiply-add of B.  K step 32 staged in
// LDS as [row][k] (row stride 40 halves = 80 bytes, so every 8-element run is 16-byte aligned).
// Two LDS buffers: the next K step's global loads are issued into registers before the MFMAs of
// the current one and written to the other buffer after them, one barrier per K step.  An
// operand stored K-major (A(m, k) = A[k][m]) is first transposed into the workspace by
// k_transpose_bf16, so that every product runs this one layout with 16-byte loads and stores.
// ---------------------------------------------------------------------------------------
constexpr int GBM = 128, GBN = 128, GBK = 32, GLDS = GBK + 8;

// One thread's share of a (rows) x GBK operand tile: RUNS = rows GBK / (256 8) runs of 8 elements.
template <int RUNS>
struct TileRegs {
  bf16x8 v[RUNS];
};

// rows x K row-major: run idx takes row idx / (GBK / 8), k run idx mod (GBK / 8)
template <int RUNS>
__device__ __forceinline__ void load_regs(TileRegs<RUNS> &t, const __bf16 *__restrict__ src, int ld, int rows, int K,
                                          int r0, int k0, bool vec_ok) {
#pragma unroll
  for (int it = 0; it < RUNS; ++it) {
    const int idx = threadIdx.x + 256 * it;
    const int gr = r0 + idx / (GBK / 8), gk = k0 + (idx % (GBK / 8)) * 8;
    if (vec_ok && gr < rows && gk + 8 <= K) {
      t.v[it] = *reinterpret_cast<const bf16x8 *>(src + (size_t)gr * ld + gk);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) t.v[it][i] = (gr < rows && gk + i < K) ? src[(size_t)gr * ld + gk + i] : (__bf16)0.0f;
    }
  }
}

template <int RUNS>
__device__ __forceinline__ void store_lds(__bf16 *lds, const TileRegs<RUNS> &t) {
#pragma unroll
  for (int it = 0; it < RUNS; ++it) {
    const int idx = threadIdx.x + 256 * it;
    *reinterpret_cast<bf16x8 *>(lds + (idx / (GBK / 8)) * GLDS + (idx % (GBK / 8)) * 8) = t.v[it];
  }
}

// dst[c][r] = src[r][c] for r < rows, c < cols (64 x 64 tiles through LDS, padded rows so that
// the column reads hit distinct banks).
__global__ void __launch_bounds__(256) k_transpose_bf16(const __bf16 *__restrict__ src, int lds_, int rows, int cols,
                                                        __bf16 *__restrict__ dst, int ldd) {
  __shared__ uint16_t tile[64][66];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const uint16_t *s16 = reinterpret_cast<const uint16_t *>(src);
  uint16_t *d16 = reinterpret_cast<uint16_t *>(dst);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = r0 + ty + 4 * i, c = c0 + tx;
    tile[ty + 4 * i][tx] = (r < rows && c < cols) ? s16[(size_t)r * lds_ + c] : (uint16_t)0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int c = c0 + ty + 4 * i, r = r0 + tx;
    if (c < cols && r < rows) d16[(size_t)c * ldd + r] = tile[tx][ty + 4 * i];
  }
}

template <int EPI>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs &g, int row, int col, float v) {
  if (EPI == EPI_STORE) {
    g.C[(size_t)row * g.ldc + col] = v;
  } else if (EPI == EPI_BIAS) {
    g.C[(size_t)row * g.ldc + col] = v + g.bias[col];
  } else if (EPI == EPI_BIAS_GELU) {
    v += g.bias[col];
    g.C[(size_t)row * g.ldc + col] = v;
    g.Cb[(size_t)row * g.ldcb + col] = (__bf16)gelu_f(v);
  } else {  // EPI_GELU_GRAD: dz_prev = bf16(dx * GELU'(z_prev))
    g.Cb[(size_t)row * g.ldcb + col] = (__bf16)(v * gelu_grad_f(g.Z[(size_t)row * g.ldz + col]));
  }
}

// The same for four consecutive columns (col a multiple of 4, 16-byte aligned rows).
template <int EPI>
__device__ __forceinline__ void gemm_epilogue4(const GemmArgs &g, int row, int col, float4 v) {
  float *c = g.C + (size_t)row * g.ldc + col;
  if (EPI == EPI_STORE) {
    *reinterpret_cast<float4 *>(c) = v;
  } else {
    const float4 b = *reinterpret_cast<const float4 *>(g.bias + col);
    v.x += b.x;
    v.y += b.y;
    v.z += b.z;
    v.w += b.w;
    *reinterpret_cast<float4 *>(c) = v;
    if (EPI == EPI_BIAS_GELU) {
      bf16x4 o;
      o[0] = (__bf16)gelu_f(v.x);
      o[1] = (__bf16)gelu_f(v.y);
      o[2] = (__bf16)gelu_f(v.z);
      o[3] = (__bf16)gelu_f(v.w);
      *reinterpret_cast<bf16x4 *>(g.Cb + (size_t)row * g.ldcb + col) = o;
    }
  }
}

constexpr int GEPI_LD = 72;  // epilogue slab row stride (floats): 32 x 72 x 4 B per wave
static_assert(4 * 32 * GEPI_LD * 4 <= 2 * (GBM + GBN) * GLDS * 2, "epilogue slabs fit in the tile buffers");

// MI = 2: 64 VGPRs of accumulators, compiled for four waves per SIMD; MI = 4: 128, two waves.
template <int EPI, int MI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MI == 2 ? 4 : 2, 8))) k_gemm(GemmArgs g) {
  constexpr int BM = 64 * MI;                          // block tile rows
  constexpr int RA = BM * GBK / (256 * 8), RB = GBN * GBK / (256 * 8);
  // the two A and two B tiles, and after the loop the epilogue slabs
  __shared__ __attribute__((aligned(16))) __bf16 smem[2 * (BM + GBN) * GLDS];
  __bf16 (*As)[BM * GLDS] = reinterpret_cast<__bf16 (*)[BM * GLDS]>(smem);
  __bf16 (*Bs)[GBN * GLDS] = reinterpret_cast<__bf16 (*)[GBN * GLDS]>(smem + 2 * BM * GLDS);
  const int bm = blockIdx.y * BM, bn = blockIdx.x * GBN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = (wave >> 1) * 32 * MI, wn = (wave & 1) * 64;
  const bool va = (g.lda % 8 == 0) && (((uintptr_t)g.A & 15) == 0);
  const bool vb = (g.ldb % 8 == 0) && (((uintptr_t)g.B & 15) == 0);
  f32x16 acc[MI][2];
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[mi][ni][i] = 0.0f;
  const int r = lane & 31, kh = (lane >> 5) * 8;
  // split over K: block z of a split product covers [z kchunk, (z + 1) kchunk)
  const int kb = g.part ? (int)blockIdx.z * g.kchunk : 0;
  const int ke = g.part ? min(g.K, kb + g.kchunk) : g.K;
  const int nk = (ke - kb + GBK - 1) / GBK;
  TileRegs<RA> ra;
  TileRegs<RB> rb;
  load_regs(ra, g.A, g.lda, g.M, ke, bm, kb, va);
  load_regs(rb, g.B, g.ldb, g.N, ke, bn, kb, vb);
  store_lds(As[0], ra);
  store_lds(Bs[0], rb);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) {
      load_regs(ra, g.A, g.lda, g.M, ke, bm, kb + (kt + 1) * GBK, va);
      load_regs(rb, g.B, g.ldb, g.N, ke, bn, kb + (kt + 1) * GBK, vb);
    }
    const __bf16 *as = As[cur];
    const __bf16 *bs = Bs[cur];
#pragma unroll
    for (int ks = 0; ks < GBK; ks += 16) {
      bf16x8 a[MI], b[2];
#pragma unroll
      for (int mi = 0; mi < MI; ++mi) a[mi] = *reinterpret_cast<const bf16x8 *>(&as[(wm + mi * 32 + r) * GLDS + ks + kh]);
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) b[ni] = *reinterpret_cast<const bf16x8 *>(&bs[(wn + ni * 32 + r) * GLDS + ks + kh]);
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
    if (more) {
      store_lds(As[cur ^ 1], ra);
      store_lds(Bs[cur ^ 1], rb);
    }
    __syncthreads();
  }
  // Epilogue through LDS (the A/B buffers are free after the last barrier): accumulator element e
  // of a 32 x 32 tile sits at row 8 (e / 4) + 4 (lane / 32) + e % 4, column lane % 32, so a lane
  // holds no two neighbours of a row.  Each wave writes its (32 MI) x 64 sub-tile in MI parts of 32
  // rows into its own LDS slab (row stride GEPI_LD floats: the two half-waves of one store land
  // in different banks), then reads them back four consecutive columns per lane and writes 16
  // bytes per lane (C) or 8 bytes (BF16 outputs).
  float *part = g.part ? g.part + (size_t)blockIdx.z * g.M * g.N : nullptr;
  float *slab = reinterpret_cast<float *>(smem) + wave * (32 * GEPI_LD);
  const int ldo = part ? g.N : g.ldc;
  const bool v4 = part ? (g.N % 4 == 0 && ((uintptr_t)part & 15) == 0)
                       : (EPI != EPI_GELU_GRAD && g.ldc % 4 == 0 && ((uintptr_t)g.C & 15) == 0 &&
                          (EPI == EPI_STORE || ((uintptr_t)g.bias & 15) == 0) &&
                          (EPI != EPI_BIAS_GELU || (g.ldcb % 4 == 0 && ((uintptr_t)g.Cb & 7) == 0)));
#pragma unroll
  for (int mi = 0; mi < MI; ++mi) {
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int e = 0; e < 16; ++e)
        slab[(8 * (e >> 2) + 4 * (lane >> 5) + (e & 3)) * GEPI_LD + ni * 32 + (lane & 31)] = acc[mi][ni][e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // 32 rows x 16 runs of 4 columns = 512 runs, 8 per lane; 16 lanes cover one row
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = it * 64 + lane;
      const int rr = idx >> 4, c4 = (idx & 15) * 4;
      const int row = bm + wm + mi * 32 + rr, col = bn + wn + c4;
      if (row >= g.M) continue;
      const float4 v = *reinterpret_cast<const float4 *>(&slab[rr * GEPI_LD + c4]);
      if (v4 && col + 4 <= g.N) {
        if (part) {
          *reinterpret_cast<float4 *>(&part[(size_t)row * ldo + col]) = v;
        } else {
          gemm_epilogue4<EPI>(g, row, col, v);
        }
      } else {
        const float vv[4] = {v.x, v.y, v.z, v.w};
        for (int q = 0; q < 4; ++q) {
          if (col + q >= g.N) break;
          if (part)
            part[(size_t)row * ldo + col + q] = vv[q];
          else
            gemm_epilogue<EPI>(g, row, col + q, vv[q]);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Sum of the split-K partial products in split order, then the epilogue.
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_splitk_reduce(GemmArgs g, int splits) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t mn = (int64_t)g.M * g.N;
  if (idx >= mn) return;
  float v = 0.0f;
  for (int z = 0; z < splits; ++z) v += g.part[(size_t)z * mn + idx];
  gemm_epilogue<EPI>(g, (int)(idx / g.N), (int)(idx % g.N), v);
}

// Split over K when the output tile grid cannot fill the chip and K is long enough: about two
// blocks per CU, at least 256 K elements per split.
static int gemm_splits(int M, int N, int K, int &kchunk) {
  const int blocks = ((M + GBM - 1) / GBM) * ((N + GBN - 1) / GBN);
  kchunk = K;
  if (blocks >= 128 || K < 512) return 1;
  int splits = min((512 + blocks - 1) / blocks, K / 256);
  if (splits < 2) return 1;
  kchunk = ((K + splits - 1) / splits + GBK - 1) / GBK * GBK;
  return (K + kchunk - 1) / kchunk;
}

// Workspace layout: [A transposed: M x ldk bf16][B transposed: N x ldk bf16][split-K partials:
// splits x M x N FP32], each part 256-byte aligned and present only when needed.
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static int transposed_ld(int K) { return (K + 7) & ~7; }  // keeps the 16-byte loads of k_gemm

size_t gemm_workspace_bytes(int M, int N, int K, bool at, bool bt) {
  int kchunk;
  const int splits = gemm_splits(M, N, K, kchunk);
  const size_t lk = (size_t)transposed_ld(K);
  size_t b = 0;
  if (at) b += align256((size_t)M * lk * 2);
  if (bt) b += align256((size_t)N * lk * 2);
  if (splits > 1) b += (size_t)splits * M * N * 4;
  return b;
}

static hipError_t launch_transpose(const __bf16 *src, int ld, int rows, int cols, __bf16 *dst, int ldd, hipStream_t s) {
  dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
  hipLaunchKernelGGL(k_transpose_bf16, grid, dim3(256), 0, s, src, ld, rows, cols, dst, ldd);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs &g0, bool at, bool bt, int epi, void *ws, size_t ws_bytes, hipStream_t s) {
  GemmArgs g = g0;
  if (ws_bytes < gemm_workspace_bytes(g.M, g.N, g.K, at, bt)) return hipErrorInvalidValue;
  char *w = (char *)ws;
  const int lk = transposed_ld(g.K);
  if (at) {  // A(m, k) = A[k][m]: K rows of M
    __bf16 *t = (__bf16 *)w;
    const hipError_t e = launch_transpose(g.A, g.lda, g.K, g.M, t, lk, s);
    if (e != hipSuccess) return e;
    g.A = t;
    g.lda = lk;
    w += align256((size_t)g.M * lk * 2);
  }
  if (bt) {
    __bf16 *t = (__bf16 *)w;
    const hipError_t e = launch_transpose(g.B, g.ldb, g.K, g.N, t, lk, s);
    if (e != hipSuccess) return e;
    g.B = t;
    g.ldb = lk;
    w += align256((size_t)g.N * lk * 2);
  }
  int kchunk;
  const int splits = gemm_splits(g.M, g.N, g.K, kchunk);
  const bool split = splits > 1;
  g.part = split ? (float *)w : nullptr;
  g.kchunk = split ? kchunk : g.K;
  // 256-row block tiles where the product is large enough to keep every CU busy with them
  const bool tall = !split && g.M >= 4096 && g.N >= 2048;
  dim3 grid((g.N + GBN - 1) / GBN, (g.M + (tall ? 2 * GBM : GBM) - 1) / (tall ? 2 * GBM : GBM), split ? splits : 1);
  const unsigned rblocks = (unsigned)(((int64_t)g.M * g.N + 255) / 256);
#define PCMD_GEMM_CASE(E_)                                                                             \
  if (epi == E_) {                                                                                     \
    if (tall)                                                                                          \
      hipLaunchKernelGGL((k_gemm<E_, 4>), grid, dim3(256), 0, s, g);                                   \
    else                                                                                               \
      hipLaunchKernelGGL((k_gemm<E_, 2>), grid, dim3(256), 0, s, g);                                   \
    if (split) hipLaunchKernelGGL((k_gemm_splitk_reduce<E_>), dim3(rblocks), dim3(256), 0, s, g, splits); \
    return hipGetLastError();                                                                          \
  }
  PCMD_GEMM_CASE(EPI_STORE)
  PCMD_GEMM_CASE(EPI_BIAS)
  PCMD_GEMM_CASE(EPI_BIAS_GELU)
  PCMD_GEMM_CASE(EPI_GELU_GRAD)
#undef PCMD_GEMM_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------
// Elementwise and reduction kernels.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_f32_to_bf16(const float *__restrict__ x, __bf16 *__restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (__bf16)x[i];
}

hipError_t launch_f32_to_bf16(const float *x, void *y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, (__bf16 *)y, n);
  return hipGetLastError();
}

// Row index of batch sample k: rows[k] when a row vector is given (one outside [0, n_total) is
// taken as row 0 and flagged in *status), else k.
__device__ __forceinline__ int64_t batch_row(const int32_t *__restrict__ rows, int64_t k, int64_t n_total,
                                             uint32_t *status) {
  if (!rows) return k;
  const int32_t r = rows[k];
  if (r < 0 || (int64_t)r >= n_total) {
    atomicOr(status, STATUS_BAD_ROW);
    return 0;
  }
  return r;
}

// y[k][j] = bf16(x[row k][j]) for a batch of n samples of d inputs.
__global__ void __launch_bounds__(256) k_gather_f32_to_bf16(const float *__restrict__ x, const int32_t *__restrict__ rows,
                                                            int64_t n_total, int d, int64_t n, __bf16 *__restrict__ y,
                                                            uint32_t *status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * d) return;
  const int64_t k = i / d, j = i - k * d;
  y[i] = (__bf16)x[batch_row(rows, k, n_total, status) * d + j];
}

hipError_t launch_gather_f32_to_bf16(const float *x, const int32_t *rows, int64_t n_total, int d, int64_t n, void *y,
                                     uint32_t *status, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_f32_to_bf16, dim3((unsigned)((n * d + 255) / 256)), dim3(256), 0, s, x, rows, n_total, d,
                     n, (__bf16 *)y, status);
  return hipGetLastError();
}

// Training targets of the surrogate: out[r][j] = ln((H[r][j] + 1/2) / (N_r + n_bins / 2)) with
// N_r the row's total, in FP64 (one block per row; the total is exact in FP64 below 2^53).
__global__ void __launch_bounds__(256) k_log_hess_target(const uint32_t *__restrict__ h, int nbins,
                                                         float *__restrict__ out) {
  __shared__ uint64_t red[256];
  const uint32_t *hr = h + (size_t)blockIdx.x * nbins;
  float *o = out + (size_t)blockIdx.x * nbins;
  const int t = threadIdx.x;
  uint64_t n = 0;
  for (int j = t; j < nbins; j += 256) n += hr[j];
  red[t] = n;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (t < k) red[t] += red[t + k];
    __syncthreads();
  }
  const double den = (double)red[0] + 0.5 * (double)nbins;
  for (int j = t; j < nbins; j += 256) o[j] = (float)log(((double)hr[j] + 0.5) / den);
}

hipError_t launch_log_hess_target(const uint32_t *h, int n, int nbins, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_log_hess_target, dim3(n), dim3(256), 0, s, h, nbins, out);
  return hipGetLastError();
}

// dy = 2 (y - t) / (n M) stored in BF16 (skipped when dy is NULL); per-block partial sums of
// (y - t)^2 in FP64.  y is [n / M][M]; the target row of sample k is batch_row(rows, k).  Threads
// take runs of four elements (16-byte loads, 8-byte stores) when the pointers and the row length
// allow it.
__global__ void __launch_bounds__(256) k_mse_grad(const float *__restrict__ y, const float *__restrict__ t, int64_t n,
                                                  int M, const int32_t *__restrict__ rows, int64_t n_total,
                                                  double scale, __bf16 *__restrict__ dy, double *__restrict__ part,
                                                  uint32_t *status) {
  __shared__ double red[256];
  double s = 0.0;
  const float g = (float)(2.0 * scale);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool vec = ((((uintptr_t)y) | ((uintptr_t)t)) & 15) == 0 && (((uintptr_t)dy) & 7) == 0 && (M & 3) == 0;
  const int64_t n4 = vec ? n / 4 : 0;
  for (int64_t i = first; i < n4; i += stride) {
    const int64_t k = (4 * i) / M, j = 4 * i - k * M;
    const float4 a = reinterpret_cast<const float4 *>(y)[i];
    const float4 b = *reinterpret_cast<const float4 *>(t + batch_row(rows, k, n_total, status) * M + j);
    const float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z, d3 = a.w - b.w;
    if (dy) {
      bf16x4 o;
      o[0] = (__bf16)(g * d0);
      o[1] = (__bf16)(g * d1);
      o[2] = (__bf16)(g * d2);
      o[3] = (__bf16)(g * d3);
      reinterpret_cast<bf16x4 *>(dy)[i] = o;
    }
    s += (double)d0 * (double)d0;
    s += (double)d1 * (double)d1;
    s += (double)d2 * (double)d2;
    s += (double)d3 * (double)d3;
  }
  for (int64_t i = 4 * n4 + first; i < n; i += stride) {
    const int64_t k = i / M, j = i - k * M;
    const float d = y[i] - t[batch_row(rows, k, n_total, status) * M + j];
    if (dy) dy[i] = (__bf16)(g * d);
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Loss = scale x the sum of the MSE_BLOCKS partials, by a fixed tree over one block.
__global__ void __launch_bounds__(256) k_loss_final(const double *__restrict__ part, int nb, double scale,
                                                    float *__restrict__ out) {
  __shared__ double red[256];
  red[threadIdx.x] = threadIdx.x < (unsigned)nb ? part[threadIdx.x] : 0.0;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < (unsigned)k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(red[0] * scale);
}

hipError_t launch_mse_grad(const float *y, const float *t, int64_t n, int M, const int32_t *rows, int64_t n_total,
                           double scale, void *dy, double *part, float *loss_out, uint32_t *status, hipStream_t s) {
  hipLaunchKernelGGL(k_mse_grad, dim3(MSE_BLOCKS), dim3(256), 0, s, y, t, n, M, rows, n_total, scale, (__bf16 *)dy,
                     part, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !loss_out) return e;
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, part, MSE_BLOCKS, scale, loss_out);
  return hipGetLastError();
}

// out = scale x the sum of nb partials: thread t sums partials t, t + 256, ... in order, then a
// fixed tree over the block (the order depends on nb alone).
__global__ void __launch_bounds__(256) k_sum_partials(const double *__restrict__ part, int64_t nb, double scale,
                                                      double *__restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < nb; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < (unsigned)k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}

hipError_t launch_sum_partials(const double *part, int64_t nb, double scale, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, nb, scale, out);
  return hipGetLastError();
}

// db[m] = sum_n dz[n][m] in FP32.  A block takes 64 columns (one per lane, so every row read is
// 128 contiguous bytes) and its COLSUM_WAVES waves split the rows: wave w sums rows w,
// w + COLSUM_WAVES, ... in order, and the partial sums are added in wave order.  The order is
// fixed by n alone, so results do not depend on the launch.
constexpr int COLSUM_WAVES = 16;

__global__ void __launch_bounds__(64 * COLSUM_WAVES) k_colsum(const __bf16 *__restrict__ dz, int n, int m,
                                                              float *__restrict__ db) {
  __shared__ float part[COLSUM_WAVES][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  float s = 0.0f;
  if (c < m) {
#pragma unroll 8
    for (int r = w; r < n; r += COLSUM_WAVES) s += (float)dz[(size_t)r * m + c];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && c < m) {
    float t = part[0][lane];
#pragma unroll
    for (int k = 1; k < COLSUM_WAVES; ++k) t += part[k][lane];
    db[c] = t;
  }
}

hipError_t launch_colsum(const void *dz, int n, int m, float *db, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((m + 63) / 64), dim3(64 * COLSUM_WAVES), 0, s, (const __bf16 *)dz, n, m, db);
  return hipGetLastError();
}

// Adam on one layer's FP32 master weights [out][in] and biases, refreshing the BF16 copies
// W [out][in] and W^T [in][out].  With update == 0 only the BF16 copies are refreshed.
__global__ void __launch_bounds__(256) k_adam_layer(AdamArgs a) {
  const int64_t nw = (int64_t)a.n_out * a.n_in;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw + a.n_out) return;
  float w = a.master[i];
  if (a.update) {
    const float g = a.grad[i];
    const float m = a.beta1 * a.m[i] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * a.v[i] + (1.0f - a.beta2) * g * g;
    a.m[i] = m;
    a.v[i] = v;
    const float mh = m / a.bc1, vh = v / a.bc2;
    w = w - a.lr * mh / (sqrtf(vh) + a.eps);
    a.master[i] = w;
  }
  if (i < nw) {
    const int o = (int)(i / a.n_in), k = (int)(i - (int64_t)o * a.n_in);
    const __bf16 wb = (__bf16)w;
    ((__bf16 *)a.w_bf16)[i] = wb;
    ((__bf16 *)a.wt_bf16)[(size_t)k * a.n_out + o] = wb;
  }
}

hipError_t launch_adam_layer(const AdamArgs &a, hipStream_t s) {
  const int64_t n = (int64_t)a.n_out * a.n_in + a.n_out;
  hipLaunchKernelGGL(k_adam_layer, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Surrogate log-likelihood: one block per sample, lam_j = N_d exp(y_j - max) / sum exp(y - max).
__global__ void __launch_bounds__(256) k_surrogate_loglike(const float *__restrict__ y, int nbins,
                                                           const uint32_t *__restrict__ d, double *__restrict__ out,
                                                           const double *__restrict__ lnfact64, int nlf) {
  __shared__ double red[256];
  const float *ys = y + (size_t)blockIdx.x * nbins;
  const int t = threadIdx.x;
  double mx = -INFINITY, nd = 0.0;
  for (int j = t; j < nbins; j += 256) {
    mx = fmax(mx, (double)ys[j]);
    nd += (double)d[j];
  }
  red[t] = mx;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (t < k) red[t] = fmax(red[t], red[t + k]);
    __syncthreads();
  }
  mx = red[0];
  __syncthreads();
  double se = 0.0;
  for (int j = t; j < nbins; j += 256) se += exp((double)ys[j] - mx);
  red[t] = se;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (t < k) red[t] += red[t + k];
    __syncthreads();
  }
  se = red[0];
  __syncthreads();
  red[t] = nd;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (t < k) red[t] += red[t + k];
    __syncthreads();
  }
  nd = red[0];
  __syncthreads();
  double acc = 0.0;
  for (int j = t; j < nbins; j += 256) {
    const double lam = nd * exp((double)ys[j] - mx) / se;
    const double dj = (double)d[j];
    const double lf = (lnfact64 && dj < (double)nlf) ? lnfact64[(int)dj] : lgamma(dj + 1.0);
    acc += dj * log(lam) - lam - lf;
  }
  red[t] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (t < k) red[t] += red[t + k];
    __syncthreads();
  }
  if (t == 0) out[blockIdx.x] = red[0];
}

hipError_t launch_surrogate_loglike(const float *y, int n, int nbins, const uint32_t *d, double *out,
                                   const double *lnfact64, int nlf, hipStream_t s) {
  hipLaunchKernelGGL(k_surrogate_loglike, dim3(n), dim3(256), 0, s, y, nbins, d, out, lnfact64, nlf);
  return hipGetLastError();
}

}  // namespace pcmd
