// Image-plane kernels (gfx950): periodic PSF convolution (LDS-tiled direct sum), sky / noise /
// flux -> magnitude.  Sec. 2.1 of the paper: each band's image is convolved with its PSF, sky and
// shot noise are added and pixel counts become magnitudes.
#include <math.h>

#include "pcmd_device.h"
#include "pcmd_internal.h"

namespace pcmd {

// One block per band: check that the PSF is finite, non-negative and sums to one within 1e-3
// (a failure sets a status bit reported by pcmd_sync).
__device__ __forceinline__ void psf_check_body(const ConvArgs &a) {
  __shared__ double red[256];
  __shared__ int bad;
  const int b = blockIdx.x;
  const int KK = a.K * a.K;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double s = 0.0;
  for (int i = threadIdx.x; i < KK; i += 256) {
    const float v = a.psf[(size_t)b * KK + i];
    if (!(v >= 0.0f) || !isfinite(v)) bad = 1;
    s += (double)v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0 && (bad || !(fabs(red[0] - 1.0) <= 1e-3))) atomicOr(a.status, STATUS_BAD_PSF);
}

__global__ void __launch_bounds__(256) k_psf_check(ConvArgs a) { psf_check_body(a); }
__global__ void __launch_bounds__(256) k_psf_check_job(const ConvArgs *__restrict__ t, int j) {
  const ConvArgs a = t[j];
  psf_check_body(a);
}

hipError_t launch_psf_check(const ConvArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_psf_check, dim3(a.B), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_psf_check_job(const ConvArgs *table, int j, int B, hipStream_t s) {
  hipLaunchKernelGGL(k_psf_check_job, dim3(B), dim3(256), 0, s, table, j);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_copy_f32(const float *__restrict__ src, float *__restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_copy_f32(const float *src, float *dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Direct periodic convolution.  G[y][x] = sum_{u,v} P[u][v] F[(y-u+h) mod N][(x-v+h) mod N].
// A 64 x 32 output tile per 256-thread block; each thread owns a column strip of CRY = 8
// outputs.  The input tile (with its K-1 halo, wrapped periodically) and the PSF are staged in
// LDS as FP32.  For every input row the thread forms, for each of its outputs that the row
// touches, the K-term dot product with the matching PSF row in FP32 (all terms positive), and
// adds it to an FP64 accumulator.
// ---------------------------------------------------------------------------------------
constexpr int CT_X = 64, CT_Y = 32, CRY = 8;

size_t conv_direct_lds_bytes(int K) {
  return ((size_t)(CT_Y + K - 1) * (CT_X + K - 1) + (size_t)K * K) * sizeof(float);
}

__device__ __forceinline__ void conv_direct_body(const ConvArgs &ca) {
  extern __shared__ float lds[];
  const float *__restrict__ F = ca.F;
  const float *__restrict__ psf = ca.psf;
  float *__restrict__ G = ca.G;
  const int N = ca.N, K = ca.K;
  const int b = blockIdx.z;
  const int h = (K - 1) >> 1;
  const int TW = CT_X + K - 1, TH = CT_Y + K - 1;
  float *tile = lds;
  float *P = lds + TW * TH;
  const int ox = blockIdx.x * CT_X, oy = blockIdx.y * CT_Y;
  const float *Fb = F + (size_t)b * N * N;
  // tile row ty holds input row oy - h + ty (outputs [oy, oy + CT_Y) read rows y - h .. y + h)
  for (int idx = threadIdx.x; idx < TW * TH; idx += 256) {
    const int ty = idx / TW, tx = idx - ty * TW;
    int gy = (oy - h + ty) % N;
    if (gy < 0) gy += N;
    int gx = (ox - h + tx) % N;
    if (gx < 0) gx += N;
    tile[idx] = Fb[(size_t)gy * N + gx];
  }
  // PSF stored flipped: Pf[a][c] = P[K-1-a][K-1-c], so output row j reads tile row ly0 + j + a
  for (int idx = threadIdx.x; idx < K * K; idx += 256) {
    const int a = idx / K, c = idx - a * K;
    P[idx] = psf[(size_t)b * K * K + (size_t)(K - 1 - a) * K + (K - 1 - c)];
  }
  __syncthreads();
  const int lx = threadIdx.x & (CT_X - 1);
  const int ly0 = (threadIdx.x >> 6) * CRY;
  double acc[CRY];
#pragma unroll
  for (int j = 0; j < CRY; ++j) acc[j] = 0.0;
  // output (ly0 + j, lx) = sum_{a,c} Pf[a][c] tile[ly0 + j + a][lx + c]; tile row r = j + a
  for (int r = 0; r < CRY + K - 1; ++r) {
    const float *trow = tile + (ly0 + r) * TW + lx;
    float dot[CRY];
#pragma unroll
    for (int j = 0; j < CRY; ++j) dot[j] = 0.0f;
    for (int c = 0; c < K; ++c) {
      const float val = trow[c];
#pragma unroll
      for (int j = 0; j < CRY; ++j) {
        const int a = r - j;
        if (a >= 0 && a < K) dot[j] = fmaf(P[a * K + c], val, dot[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < CRY; ++j) acc[j] += (double)dot[j];
  }
  const int x = ox + lx;
  if (x < N) {
#pragma unroll
    for (int j = 0; j < CRY; ++j) {
      const int y = oy + ly0 + j;
      if (y < N) G[(size_t)b * N * N + (size_t)y * N + x] = (float)acc[j];
    }
  }
}

__global__ void __launch_bounds__(256) k_conv_direct(ConvArgs a) { conv_direct_body(a); }
__global__ void __launch_bounds__(256) k_conv_direct_job(const ConvArgs *__restrict__ t, int j) {
  const ConvArgs a = t[j];
  conv_direct_body(a);
}

hipError_t launch_conv_direct(const ConvArgs &a, hipStream_t s) {
  const size_t lds = conv_direct_lds_bytes(a.K);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  dim3 grid((a.N + CT_X - 1) / CT_X, (a.N + CT_Y - 1) / CT_Y, a.B);
  hipLaunchKernelGGL(k_conv_direct, grid, dim3(256), lds, s, a);
  return hipGetLastError();
}
hipError_t launch_conv_direct_job(const ConvArgs *table, int j, int B, int N, int K, hipStream_t s) {
  const size_t lds = conv_direct_lds_bytes(K);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  dim3 grid((N + CT_X - 1) / CT_X, (N + CT_Y - 1) / CT_Y, B);
  hipLaunchKernelGGL(k_conv_direct_job, grid, dim3(256), lds, s, table, j);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Noise and magnitudes (FP64 arithmetic per pixel, FP32 storage).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void noise_mag_body(const NoiseArgs &a, int p) {
  if (p >= a.npx) return;
  for (int b = 0; b < a.B; ++b) {
    const double G = (double)a.G[(size_t)b * a.npx + p];
    double m;
    if (a.noise_model == PCMD_NOISE_NONE) {
      m = G > 0.0 ? -2.5 * log10(G) : INFINITY;
    } else {
      const u4 w = philox10((uint32_t)p, (uint32_t)b, TAG_NOISE, 0u, a.k0, a.k1);
      const double z = box_muller(w.x, w.y);
      if (a.noise_model == PCMD_NOISE_GAUSS_MAG) {
        m = G > 0.0 ? -2.5 * log10(G) + a.sigma[b] * z : INFINITY;
      } else {
        const double t = a.exptime[b];
        const double c = G * t * exp10(0.4 * a.zp[b]) + a.sky[b];
        const double c2 = c + sqrt(c > 0.0 ? c : 0.0) * z - a.sky[b];
        m = c2 > 0.0 ? -2.5 * log10(c2 / t) + a.zp[b] : INFINITY;
      }
    }
    a.mags[(size_t)b * a.npx + p] = (float)m;
  }
}

__global__ void __launch_bounds__(256) k_noise_mag(NoiseArgs a) { noise_mag_body(a, blockIdx.x * blockDim.x + threadIdx.x); }
__global__ void __launch_bounds__(256) k_noise_mag_job(const NoiseArgs *__restrict__ t, int j) {
  const NoiseArgs a = t[j];
  noise_mag_body(a, blockIdx.x * blockDim.x + threadIdx.x);
}

hipError_t launch_noise_mag_job(const NoiseArgs *table, int j, int npx, hipStream_t s) {
  hipLaunchKernelGGL(k_noise_mag_job, dim3((npx + 255) / 256), dim3(256), 0, s, table, j);
  return hipGetLastError();
}

hipError_t launch_noise_mag(const NoiseArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_noise_mag, dim3((a.npx + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace pcmd
